// HIP kernels (gfx950) of the HHG P1 hot path: stencil apply (Alg. 3),
// staged multicolour Gauss-Seidel, residual, restriction, prolongation,
// ghost-copy refresh, norms, coarse Jacobi-PCG and layout conversion.
//
// Stencils follow from the P1 stiffness matrix (a stencil is a row of it,
// sec. 1.1 / 4.2).  On a macro-face every micro-triangle is a translate of
// the scaled macro-face or of its point reflection, so with constant k the
// face-interior stencil is
//   centre 2 (c0 + c1 + c2), (i+-1, j): -c2, (i, j+-1): -c1,
//   (i+1, j-1) and (i-1, j+1): -c0,
// with c_m the cotangent of the macro-face angle at vertex m.  With a
// variable coefficient each micro-triangle T contributes -1/2 kbar_T cot to
// the weight of the micro-edge opposite the angle, kbar_T being the mean of
// the nodal k at T's corners (computed on the fly, sec. 1.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>

#include <cstdint>

#include "hhg_device.hpp"

namespace hhg {

// ------------------------------------------------------------------ stencils

template <class T>
struct W7 { T c, e, w, n, s, se, nw; };   // face point weights

template <class T>
struct WE { T c, al, ah, l0, h0, l1, h1; };   // edge point weights

// Face-interior weights at offset p; up/dn: offsets to the row above/below.
template <class T>
__device__ __forceinline__ W7<T> face_weights(int op, const FaceInfo& fi, double inv4l,
                                              const T* kap, int64_t p, int64_t up, int64_t dn) {
    W7<T> w;
    if (op == OP_MASS) {
        const T a = (T)(fi.area * inv4l), o = (T)(fi.area * inv4l / 6.0);
        w.c = a; w.e = w.w = w.n = w.s = w.se = w.nw = o;
        return w;
    }
    const T c0 = (T)fi.cot[0], c1 = (T)fi.cot[1], c2 = (T)fi.cot[2];
    if (op == OP_LAPLACE) {
        w.c = (T)(2.0 * (fi.cot[0] + fi.cot[1] + fi.cot[2]));
        w.e = w.w = -c2;
        w.n = w.s = -c1;
        w.se = w.nw = -c0;
        return w;
    }
    const T k0 = kap[p], kE = kap[p + 1], kW = kap[p - 1], kN = kap[p + up], kS = kap[p - dn];
    const T kSE = kap[p - dn + 1], kNW = kap[p + up - 1];
    const T third = (T)(1.0 / 3.0), h = (T)0.5;
    // the six micro-triangles around the point
    const T t1 = (k0 + kE + kN) * third;     // up   (i, j)
    const T t2 = (kSE + kE + k0) * third;    // down (i, j-1)
    const T t3 = (kW + k0 + kNW) * third;    // up   (i-1, j)
    const T t4 = (kS + k0 + kW) * third;     // down (i-1, j-1)
    const T t5 = (k0 + kN + kNW) * third;    // down (i-1, j)
    const T t6 = (kS + kSE + k0) * third;    // up   (i, j-1)
    w.e = -h * c2 * (t1 + t2);
    w.w = -h * c2 * (t3 + t4);
    w.n = -h * c1 * (t1 + t5);
    w.s = -h * c1 * (t6 + t4);
    w.se = -h * c0 * (t6 + t2);
    w.nw = -h * c0 * (t3 + t5);
    w.c = -(w.e + w.w + w.n + w.s + w.se + w.nw);
    return w;
}

// Interior-edge point k: neighbours k-1, k+1 on the edge and g_s[k-1], g_s[k]
// in the ghost row of face s (s = 0, 1).
template <class T>
__device__ __forceinline__ WE<T> edge_weights(int op, const EdgeInfo& ei, double inv4l,
                                              const T* kap, int64_t m, int64_t g0, int64_t g1,
                                              int k) {
    WE<T> w;
    if (op == OP_MASS) {
        const double a0 = ei.area[0] * inv4l, a1 = ei.area[1] * inv4l;
        w.al = w.ah = (T)((a0 + a1) / 12.0);
        w.l0 = w.h0 = (T)(a0 / 6.0);
        w.l1 = w.h1 = (T)(a1 / 6.0);
        w.c = (T)((a0 + a1) / 2.0);
        return w;
    }
    if (op == OP_LAPLACE) {
        w.al = w.ah = (T)(-0.5 * (ei.cA[0] + ei.cA[1]));
        w.l0 = (T)(-ei.cL[0]); w.h0 = (T)(-ei.cH[0]);
        w.l1 = (T)(-ei.cL[1]); w.h1 = (T)(-ei.cH[1]);
        w.c = (T)(ei.cA[0] + ei.cL[0] + ei.cH[0] + ei.cA[1] + ei.cL[1] + ei.cH[1]);
        return w;
    }
    const T third = (T)(1.0 / 3.0), h = (T)0.5;
    const T km = kap[m + k - 1], k0 = kap[m + k], kp = kap[m + k + 1];
    const T a0 = kap[g0 + k - 1], b0 = kap[g0 + k];
    const T a1 = kap[g1 + k - 1], b1 = kap[g1 + k];
    // per face s: T1(k) = (k, k+1, g[k]), T1(k-1) = (k-1, k, g[k-1]),
    // T2(k) = (k, g[k], g[k-1])
    const T t1_0 = (k0 + kp + b0) * third, t1m_0 = (km + k0 + a0) * third, t2_0 = (k0 + b0 + a0) * third;
    const T t1_1 = (k0 + kp + b1) * third, t1m_1 = (km + k0 + a1) * third, t2_1 = (k0 + b1 + a1) * third;
    const T cA0 = (T)ei.cA[0], cA1 = (T)ei.cA[1];
    w.al = -h * (cA0 * t1m_0 + cA1 * t1m_1);
    w.ah = -h * (cA0 * t1_0 + cA1 * t1_1);
    w.h0 = -h * (T)ei.cH[0] * (t1_0 + t2_0);
    w.l0 = -h * (T)ei.cL[0] * (t2_0 + t1m_0);
    w.h1 = -h * (T)ei.cH[1] * (t1_1 + t2_1);
    w.l1 = -h * (T)ei.cL[1] * (t2_1 + t1m_1);
    w.c = -(w.al + w.ah + w.l0 + w.h0 + w.l1 + w.h1);
    return w;
}

// Weight of interior vertex v towards its ghost slot q (the edge point next
// to v on incident edge q).
template <class T>
__device__ __forceinline__ T vertex_weight(int op, const VertexInfo& vi, double inv4l,
                                           const T* kap, int64_t vb, int q) {
    if (op == OP_MASS)
        return (T)((vi.area[q][0] + vi.area[q][1]) * inv4l / 12.0);
    if (op == OP_LAPLACE)
        return (T)(-0.5 * (vi.cA[q][0] + vi.cA[q][1]));
    const T third = (T)(1.0 / 3.0);
    const T kv = kap[vb], kq = kap[vb + 1 + q];
    T s = (T)0;
    for (int f = 0; f < vi.nfe[q]; ++f) {
        const T kp = kap[vb + 1 + vi.partner[q][f]];
        s += (T)vi.cA[q][f] * ((kv + kq + kp) * third);
    }
    return (T)-0.5 * s;
}

// Vertex kernels read deg and boundary as one 8-byte load.
static_assert(offsetof(VertexInfo, deg) == 0 && offsetof(VertexInfo, boundary) == 4 && alignof(VertexInfo) >= 8,
              "deg and boundary must form an aligned pair");

// s = sum_q w_q x[ring q] and c = sum_q w_q over the ring of a vertex, in
// ring order (deg = vi.deg, read by the caller).  For the Laplacian the ring
// values and weights are loaded four
// at a time (indices clamped into the ring, so the loads need no branch):
// the loads of a group are in flight together instead of one round trip per
// neighbour.  The sums are formed in the same order as the plain loop.
template <class T>
__device__ __forceinline__ void vertex_ring_sums(int op, const VertexInfo& vi, int deg, double inv4l,
                                                 const T* kap, const T* x, int64_t vb, T& s, T& c) {
    if (op == OP_LAPLACE) {
        for (int q0 = 0; q0 < deg; q0 += 4) {
            T xq[4], wq[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int q = q0 + k < deg ? q0 + k : q0;
                xq[k] = x[vb + 1 + q];
                wq[k] = (T)(-0.5 * (vi.cA[q][0] + vi.cA[q][1]));
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (q0 + k < deg) {
                    s += wq[k] * xq[k];
                    c += wq[k];
                }
        }
        return;
    }
    for (int q = 0; q < deg; ++q) {
        const T wq = vertex_weight<T>(op, vi, inv4l, kap, vb, q);
        s += wq * x[vb + 1 + q];
        c += wq;
    }
}

// ------------------------------------------------------------------ kernels

// Copy ghost entries [lo, hi) of the ghost table.
template <class T>
__global__ __launch_bounds__(NT) void k_sync(T* __restrict__ x, const int64_t* __restrict__ dst,
                                             const int64_t* __restrict__ src, int64_t lo, int64_t hi) {
    for (int64_t t = lo + blockIdx.x * (int64_t)NT + threadIdx.x; t < hi; t += (int64_t)gridDim.x * NT)
        x[dst[t]] = x[src[t]];
}

template <class T>
__global__ __launch_bounds__(NT) void k_fill(T* __restrict__ x, int64_t n, T v) {
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        x[t] = v;
}

template <class T>
__device__ __forceinline__ T edge_apply(int op, const LevelDev& L, const EdgeInfo& ei, const T* x,
                                        const T* kap, int64_t m, int64_t g0, int64_t g1, int k) {
    const WE<T> w = edge_weights<T>(op, ei, L.inv4l, kap, m, g0, g1, k);
    return w.c * x[m + k] + w.al * x[m + k - 1] + w.ah * x[m + k + 1] + w.l0 * x[g0 + k - 1] +
           w.h0 * x[g0 + k] + w.l1 * x[g1 + k - 1] + w.h1 * x[g1 + k];
}

template <class T>
__device__ __forceinline__ T vertex_apply(int op, const LevelDev& L, const VertexInfo& vi, const T* x,
                                          const T* kap, int64_t vb) {
    T s = (T)0, c = (T)0;
    vertex_ring_sums<T>(op, vi, vi.deg, L.inv4l, kap, x, vb, s, c);
    c = (op == OP_MASS) ? c : -c;
    return c * x[vb] + s;
}

// Residuals f - A x at edge point k of an interior edge e and at an interior
// vertex, with the arithmetic of apply_low_item's residual mode.
template <class T>
__device__ __forceinline__ T edge_resid(int op, const LevelDev& L, const EdgeInfo& ei, int e, const T* x,
                                        const T* f, const T* kap, int k) {
    const int64_t m = edge_main(L, e), g0 = edge_ghost(L, e, 0), g1 = edge_ghost(L, e, 1);
    const WE<T> w = edge_weights<T>(op, ei, L.inv4l, kap, m, g0, g1, k);
    const T v = w.c * x[m + k] + w.al * x[m + k - 1] + w.ah * x[m + k + 1] + w.l0 * x[g0 + k - 1] +
                w.h0 * x[g0 + k] + w.l1 * x[g1 + k - 1] + w.h1 * x[g1 + k];
    return f[m + k] - v;
}

template <class T>
__device__ __forceinline__ T vertex_resid(int op, const LevelDev& L, const VertexInfo& vi, int deg, const T* x,
                                          const T* f, const T* kap, int64_t vb) {
    T s = (T)0, c = (T)0;
    vertex_ring_sums<T>(op, vi, deg, L.inv4l, kap, x, vb, s, c);
    c = (op == OP_MASS) ? c : -c;
    return f[vb] - (c * x[vb] + s);
}

// Point operator at edge/vertex item t (edge points first, ne of them, then
// vertices), with all copies of the result; see k_apply_low for the modes.
template <class T, int MODE>
__device__ __forceinline__ void apply_low_item(const LevelDev& L, int op, const T* __restrict__ x,
                                               const T* __restrict__ f, T* __restrict__ y,
                                               const T* __restrict__ kap, int64_t t, int64_t ne, double& acc) {
    const int n = L.n;
    T v = (T)0;
    if (t < ne) {
        const int e = (int)(t / (n - 2)), k = (int)(t % (n - 2)) + 1;
        const EdgeInfo& ei = L.edges[e];
        const int64_t m = edge_main(L, e);
        if (!ei.boundary) {
            const int64_t g0 = edge_ghost(L, e, 0), g1 = edge_ghost(L, e, 1);
            const WE<T> w = edge_weights<T>(op, ei, L.inv4l, kap, m, g0, g1, k);
            if (MODE == 3) {
                v = x[m + k] / w.c;
            } else {
                v = w.c * x[m + k] + w.al * x[m + k - 1] + w.ah * x[m + k + 1] + w.l0 * x[g0 + k - 1] +
                    w.h0 * x[g0 + k] + w.l1 * x[g1 + k - 1] + w.h1 * x[g1 + k];
                if (MODE >= 1) v = f[m + k] - v;
                if (MODE == 1 || MODE == 4) acc += (double)v * (double)v;
                if (MODE == 2) v = v / w.c;
            }
        }
        if (MODE == 4) return;
        y[m + k] = v;
        push_edge(L, y, ei, k, v, true);
    } else {
        const int vv = (int)(t - ne);
        const VertexInfo& vi = L.verts[vv];
        const int64_t vb = vert_off(L, vv);
        const int2 db = *reinterpret_cast<const int2*>(&vi.deg);   // deg, boundary in one load
        if (!db.y) {
            T s = (T)0, c = (T)0;
            vertex_ring_sums<T>(op, vi, db.x, L.inv4l, kap, x, vb, s, c);
            c = (op == OP_MASS) ? c : -c;
            if (MODE == 3) {
                v = x[vb] / c;
            } else {
                v = c * x[vb] + s;
                if (MODE >= 1) v = f[vb] - v;
                if (MODE == 1 || MODE == 4) acc += (double)v * (double)v;
                if (MODE == 2) v = v / c;
            }
        }
        if (MODE == 4) return;
        y[vb] = v;
        push_vertex(L, y, vi, v);
    }
}

// Point operator of the edge and vertex points, with all copies of the
// result (the face points are k_apply_tiled's):
//   MODE 0: y = A x              MODE 1: y = f - A x (+ per-block sums of y^2)
//   MODE 2: y = (f - A x) / a_pp MODE 3: y = x / a_pp
// and 0 on Dirichlet rows; MODE 4 only sums (f - A x)^2 and writes nothing.
template <class T, int MODE>
__global__ __launch_bounds__(NT) void k_apply_low(LevelDev L, int op, const T* __restrict__ x,
                                                  const T* __restrict__ f, T* __restrict__ y,
                                                  const T* __restrict__ kap, double* partials) {
    __shared__ double sm[NT / 64 + 1];
    double acc = 0.0;
    LOW_LOOP(L, 0) { apply_low_item<T, MODE>(L, op, x, f, y, kap, t, ne_, acc); }
    if ((MODE == 1 || MODE == 4) && partials) {
        const double s = block_sum<NT>(acc, sm);
        if (threadIdx.x == 0) partials[blockIdx.x] = s;
    }
}

// Mixed-precision outer step at edge/vertex item t (see k_mp_step_tiled).
template <bool UPD>
__device__ __forceinline__ void mp_low_item(const LevelDev& L, int op, const double* __restrict__ x,
                                            const float* __restrict__ e, const double* __restrict__ f,
                                            double* __restrict__ xo, float* __restrict__ r,
                                            const double* __restrict__ kap, int64_t t, int64_t ne_,
                                            double& acc) {
    const int nl_ = L.n;
    auto V = [&](int64_t q) -> double { return UPD ? x[q] + (double)e[q] : x[q]; };
    if (t < ne_) {
        const int ed = (int)(t / (nl_ - 2)), k = (int)(t % (nl_ - 2)) + 1;
        const EdgeInfo& ei = L.edges[ed];
        const int64_t m = edge_main(L, ed);
        double v = 0.0, v0 = x[m + k];
        if (!ei.boundary) {
            v0 = V(m + k);
            const int64_t g0 = edge_ghost(L, ed, 0), g1 = edge_ghost(L, ed, 1);
            const WE<double> w = edge_weights<double>(op, ei, L.inv4l, kap, m, g0, g1, k);
            v = f[m + k] - (w.c * v0 + w.al * V(m + k - 1) + w.ah * V(m + k + 1) +
                            w.l0 * V(g0 + k - 1) + w.h0 * V(g0 + k) + w.l1 * V(g1 + k - 1) +
                            w.h1 * V(g1 + k));
            acc += v * v;
        }
        r[m + k] = (float)v;
        push_edge(L, r, ei, k, (float)v, true);
        if (UPD) {
            xo[m + k] = v0;
            push_edge(L, xo, ei, k, v0, true);
        }
    } else {
        const int vv = (int)(t - ne_);
        const VertexInfo& vi = L.verts[vv];
        const int64_t vb = vert_off(L, vv);
        double v = 0.0, v0 = x[vb];
        if (!vi.boundary) {
            v0 = V(vb);
            double sn = 0.0, c = 0.0;
            for (int q = 0; q < vi.deg; ++q) {
                const double wq = vertex_weight<double>(op, vi, L.inv4l, kap, vb, q);
                sn += wq * V(vb + 1 + q);
                c += wq;
            }
            v = f[vb] - (-c * v0 + sn);
            acc += v * v;
        }
        r[vb] = (float)v;
        push_vertex(L, r, vi, (float)v);
        if (UPD) {
            xo[vb] = v0;
            push_vertex(L, xo, vi, v0);
        }
    }
}

// Per-block sums of x*y over owned interior points (faces, interior edge
// points, interior vertices): each unknown once.
template <class T>
__global__ __launch_bounds__(NT) void k_dot(LevelDev L, const T* __restrict__ x, const T* __restrict__ y,
                                            int gf, double* partials) {
    __shared__ double sm[NT / 64 + 1];
    double acc = 0.0;
    if ((int)blockIdx.x < gf) {
        FACE_ALL_LOOP(L, gf)
        (void)fi;
        if (interior) acc += (double)x[p] * (double)y[p];
        }
    } else {
        const int n = L.n;
        const int64_t ne = (int64_t)L.n_iedges * (n - 2);
        for (int64_t t = (int64_t)(blockIdx.x - gf) * NT + threadIdx.x; t < ne + L.n_iverts;
             t += (int64_t)(gridDim.x - gf) * NT) {
            int64_t q;
            if (t < ne) q = edge_main(L, L.iedges[t / (n - 2)]) + (t % (n - 2)) + 1;
            else q = vert_off(L, L.iverts[t - ne]);
            acc += (double)x[q] * (double)y[q];
        }
    }
    const double s = block_sum<NT>(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

template <class T>
__global__ __launch_bounds__(NT) void k_axpby(int64_t n, T alpha, const T* __restrict__ x, T beta,
                                              const T* __restrict__ y, T* __restrict__ z) {
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        z[t] = alpha * x[t] + beta * y[t];
}

// Sum partials[0, count) in a fixed order; optional square root.
__global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ partials,
                                                       int64_t count, double* out, int do_sqrt) {
    __shared__ double sm[1024 / 64 + 1];
    double a = 0.0;
    for (int64_t t = threadIdx.x; t < count; t += 1024) a += partials[t];
    const double s = block_sum<1024>(a, sm);
    if (threadIdx.x == 0) *out = do_sqrt ? sqrt(s) : s;
}

// Linear interpolation of coarse face values at fine face point (i, j):
// coincident points copy, midpoints of coarse micro-edges average the two
// ends (horizontal, vertical, and the diagonal from (I+1, J) to (I, J+1)).
// Branch-free over the parities: the two ends are (I + (io & jo), J) and
// (I + (io & !jo), J + jo); at a coincident point both are (I, J), and
// 0.5 (x + x) = x exactly.
template <class T>
__device__ __forceinline__ T prol_face(const T* __restrict__ uc, int64_t cb, int nc, int i, int j) {
    const int I = i >> 1, J = j >> 1, io = i & 1, jo = j & 1;
    const T a = uc[cb + row_start(nc, J) + I + (io & jo)];
    const T b = uc[cb + row_start(nc, J + jo) + I + (io & (jo ^ 1))];
    return (T)0.5 * (a + b);
}

// Dirichlet status of face point (i, j) (ring points on boundary sides or
// at boundary vertices).
__device__ __forceinline__ bool face_dirichlet(const FaceInfo& fi, int n, int i, int j) {
    if (i >= 1 && j >= 1 && i + j <= n - 2) return false;
    if (j == 0 && i == 0) return fi.bvtx[0];
    if (j == 0 && i == n - 1) return fi.bvtx[1];
    if (i == 0 && j == n - 1) return fi.bvtx[2];
    if (j == 0) return fi.bside[0];
    if (i == 0) return fi.bside[1];
    return fi.bside[2];
}

// The same from a mask of the face's Dirichlet flags (bits 0-2 vertices,
// 3-5 sides), read once per tile so that lane-divergent code tests registers.
__device__ __forceinline__ int face_dirichlet_mask(const FaceInfo& fi) {
    return (fi.bvtx[0] ? 1 : 0) | (fi.bvtx[1] ? 2 : 0) | (fi.bvtx[2] ? 4 : 0) | (fi.bside[0] ? 8 : 0) |
           (fi.bside[1] ? 16 : 0) | (fi.bside[2] ? 32 : 0);
}
__device__ __forceinline__ bool face_dirichlet_m(int m, int n, int i, int j) {
    if (i >= 1 && j >= 1 && i + j <= n - 2) return false;
    if (j == 0 && i == 0) return m & 1;
    if (j == 0 && i == n - 1) return m & 2;
    if (i == 0 && j == n - 1) return m & 4;
    if (j == 0) return m & 8;
    if (i == 0) return m & 16;
    return m & 32;
}

// Prolongation of one entry of the edge and vertex blocks (edge main
// k = 0..n-1, vertex value and ghost slots): the value to add, 0 at
// Dirichlet points and padding.
template <class T>
__device__ __forceinline__ T prol_low(const LevelDev& Lf, const LevelDev& Lc, const T* __restrict__ uc,
                                      int64_t t) {
    const int n = Lf.n;
    const int64_t ne = (int64_t)Lf.E * n;
    if (t < ne) {
        const int e = (int)(t / n), k = (int)(t % n);
        const EdgeInfo& ei = Lf.edges[e];
        if (ei.boundary) return (T)0;
        const int64_t mc = edge_main(Lc, e);
        if (k == 0) return Lf.verts[ei.a].boundary ? (T)0 : uc[mc];
        if (k == n - 1) return Lf.verts[ei.b].boundary ? (T)0 : uc[mc + Lc.n - 1];
        return (k & 1) ? (T)0.5 * (uc[mc + (k >> 1)] + uc[mc + (k >> 1) + 1]) : uc[mc + (k >> 1)];
    }
    const int64_t tv = t - ne;
    const int v = (int)(tv / Lf.vert_stride), slot = (int)(tv % Lf.vert_stride);
    const VertexInfo& vi = Lf.verts[v];
    if (vi.boundary || slot > vi.deg) return (T)0;
    const int64_t vc = vert_off(Lc, v);
    const T cv = uc[vc];
    return slot == 0 ? cv : (T)0.5 * (cv + uc[vc + slot]);
}

// Fused multicolour face smoother.  A tile of TI x TJ points plus a halo of
// H points sits in LDS (TI + 2 H = GS_W values per row); colour stage s (of
// ncol) is applied on the tile grown by ncol - 1 - s points, so every stage
// sees exactly the values that separate colour passes over the whole face
// would give it, and u, f are read once and u written once per sweep.  Tiles
// would otherwise read halo points a neighbour tile has already overwritten,
// so the sweep reads uin and writes uout; the same launch copies the face
// rings, edge points and vertex blocks into uout and writes the near-edge
// rows into uout's edge ghost rows, leaving uout a complete, consistent
// field.  The residual variant (H = GS_HE) grows every stage by one more
// point, so that after the last colour the values one point beyond the tile
// are final too; it then forms f - A u at the tile's interior points from LDS
// and stores it as well (one more write stream instead of a separate pass
// that reads u and f again).
constexpr int GS_NT = 512;                      // threads per block
constexpr int GS_NW = GS_NT / 64;               // waves per block
constexpr int GS_COPY_BLOCKS = 32;

// Shape of a tile of TJ updated rows with halo H: tile width, LDS rows, rows
// loaded per wave, and the per-stage row (three colours) or slot (two
// colours) iterations; stages grow by at most H - 1 (three colours) or
// H - 2 (two colours) points.
template <int TJ, int H>
struct GsTile {
    static constexpr int TI = GS_W - 2 * H;
    static constexpr int R = TJ + 2 * H;
    static constexpr int RPW = (R + GS_NW - 1) / GS_NW;
    static constexpr int IT3 = (TJ + 2 * (H - 1) + GS_NW - 1) / GS_NW;
    static constexpr int IT2 = ((TJ + 2 * (H - 2)) * (GS_W / 2) + GS_NT - 1) / GS_NT;
};

__device__ __forceinline__ int pmod(int a, int m) { return ((a % m) + m) % m; }

// Halo and tile list of the smoother variants: RES = 0 plain sweep, 1 with
// the residual, 2 with the residual norm, 3 with the restricted residual.
__host__ __device__ constexpr int gs_halo(int res) { return res == 3 ? GS_HR : (res ? GS_HE : GS_H); }
__host__ __device__ constexpr int gs_list(int res) { return res == 3 ? 2 : (res ? 1 : 0); }

// Variable-coefficient weights of the point at LDS position (r, tx), from the
// coefficient tile: the same arithmetic as face_weights.
template <class T>
__device__ __forceinline__ W7<T> gs_weights_lds(const FaceInfo& fi, T (*ks)[GS_W], int r, int tx) {
    const T c0 = (T)fi.cot[0], c1 = (T)fi.cot[1], c2 = (T)fi.cot[2];
    const T k0 = ks[r][tx], kE = ks[r][tx + 1], kW = ks[r][tx - 1], kN = ks[r + 1][tx];
    const T kS = ks[r - 1][tx], kSE = ks[r - 1][tx + 1], kNW = ks[r + 1][tx - 1];
    const T third = (T)(1.0 / 3.0), hf = (T)0.5;
    const T t1 = (k0 + kE + kN) * third, t2 = (kSE + kE + k0) * third;
    const T t3 = (kW + k0 + kNW) * third, t4 = (kS + k0 + kW) * third;
    const T t5 = (k0 + kN + kNW) * third, t6 = (kS + kSE + k0) * third;
    W7<T> w;
    w.e = -hf * c2 * (t1 + t2);
    w.w = -hf * c2 * (t3 + t4);
    w.n = -hf * c1 * (t1 + t5);
    w.s = -hf * c1 * (t6 + t4);
    w.se = -hf * c0 * (t6 + t2);
    w.nw = -hf * c0 * (t3 + t5);
    w.c = -(w.e + w.w + w.n + w.s + w.se + w.nw);
    return w;
}

// Stage update of one face point at LDS position (r, tx).
template <class T, bool VARK>
__device__ __forceinline__ T gs_point(const FaceInfo& fi, const W7<T>& w, T invc, T fv,
                                      T (*us)[GS_W], T (*ks)[GS_W], int r, int tx) {
    const T uE = us[r][tx + 1], uW = us[r][tx - 1], uN = us[r + 1][tx], uS = us[r - 1][tx];
    const T uSE = us[r - 1][tx + 1], uNW = us[r + 1][tx - 1];
    if (!VARK) return (fv - (w.e * (uE + uW) + w.n * (uN + uS) + w.se * (uSE + uNW))) * invc;
    const W7<T> v = gs_weights_lds<T>(fi, ks, r, tx);
    return (fv - (v.e * uE + v.w * uW + v.n * uN + v.s * uS + v.se * uSE + v.nw * uNW)) / v.c;
}

// Residual f - A u of the point at LDS position (r, tx), in the order of the
// residual kernel's point formula.
template <class T, bool VARK>
__device__ __forceinline__ T gs_resid(const FaceInfo& fi, const W7<T>& wl, T fv, T (*us)[GS_W],
                                      T (*ks)[GS_W], int r, int tx) {
    const W7<T> w = VARK ? gs_weights_lds<T>(fi, ks, r, tx) : wl;
    return fv - (w.c * us[r][tx] + w.e * us[r][tx + 1] + w.w * us[r][tx - 1] + w.n * us[r + 1][tx] +
                 w.s * us[r - 1][tx] + w.se * us[r - 1][tx + 1] + w.nw * us[r + 1][tx - 1]);
}

// Tile rows into registers: wave w takes LDS rows w + GS_NW q, lane l columns
// l, l + 64, l + 128.  The caller stores them to LDS after issuing f loads.
// Coarse correction added while a tile is loaded (the first sweep after
// the prolongation): uc is the coarse field, cb its face base, nc its n.
template <class T>
struct ProlTile {
    const T* uc;
    int64_t cb;
    int nc;
};

template <class T, bool VARK, bool PROL, int TJ, int H>
__device__ __forceinline__ void gs_load_u(int n, int i0, int j0, int64_t fb, const T* __restrict__ uin,
                                          const T* __restrict__ kap, T (*ur)[3], T (*kr)[3],
                                          const FaceInfo& fi, const ProlTile<T>& pt, T (*us)[GS_W]) {
    const int wv = wave_id(), lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < GsTile<TJ, H>::RPW; ++q) {
        const int r = wv + GS_NW * q, j = j0 + r;
        const int64_t rb = fb + row_start(n, j < 0 ? 0 : (j > n ? n : j));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = i0 + lane + 64 * c;
            const bool in = r < GsTile<TJ, H>::R && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
            ur[q][c] = in ? uin[rb + i] : (T)0;
            if (VARK) kr[q][c] = in ? kap[rb + i] : (T)0;
        }
    }
    if (!PROL) return;
    // The coarse values the tile interpolates, staged in LDS (the u tile's
    // space is free until the tile is stored): coarse rows and columns from
    // half the tile origin, one more each for the odd fine rows and columns.
    constexpr int CW = GS_W / 2 + 2, CH = GsTile<TJ, H>::R / 2 + 2;
    static_assert(CW * CH <= GsTile<TJ, H>::R * GS_W, "coarse tile must fit the u tile");
    T* cs = &us[0][0];
    const int nc = pt.nc, Ilo = (i0 < 0 ? 0 : i0) >> 1, Jlo = (j0 < 0 ? 0 : j0) >> 1;
    constexpr int NCS = (CW * CH + GS_NT - 1) / GS_NT;
    T cr[NCS];                                   // loads first, LDS stores after
#pragma unroll
    for (int q = 0; q < NCS; ++q) {
        const int t = threadIdx.x + q * GS_NT;
        const int J = Jlo + t / CW, I = Ilo + t % CW;
        cr[q] = (t < CW * CH && J <= nc - 1 && I <= nc - 1 - J) ? pt.uc[pt.cb + row_start(nc, J) + I] : (T)0;
    }
#pragma unroll
    for (int q = 0; q < NCS; ++q) {
        const int t = threadIdx.x + q * GS_NT;
        if (t < CW * CH) cs[t] = cr[q];
    }
    __syncthreads();
    // linear interpolation as in prol_face, from LDS
    const int dm = face_dirichlet_mask(fi);
#pragma unroll
    for (int q = 0; q < GsTile<TJ, H>::RPW; ++q) {
        const int r = wv + GS_NW * q, j = j0 + r;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int i = i0 + lane + 64 * c;
            const bool in = r < GsTile<TJ, H>::R && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
            if (!in || face_dirichlet_m(dm, n, i, j)) continue;
            const int I = (i >> 1) - Ilo, J = (j >> 1) - Jlo, io = i & 1, jo = j & 1;
            const T a = cs[J * CW + I + (io & jo)];
            const T b = cs[(J + jo) * CW + I + (io & (jo ^ 1))];
            ur[q][c] += (T)0.5 * (a + b);
        }
    }
    __syncthreads();
}

template <class T, bool VARK, int TJ, int H>
__device__ __forceinline__ void gs_store_u(T (*us)[GS_W], T (*ks)[GS_W], T (*ur)[3], T (*kr)[3]) {
    const int wv = wave_id(), lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < GsTile<TJ, H>::RPW; ++q) {
        const int r = wv + GS_NW * q;
        if (r < GsTile<TJ, H>::R) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                us[r][lane + 64 * c] = ur[q][c];
                if (VARK) ks[r][lane + 64 * c] = kr[q][c];
            }
        }
    }
}

// Three colours ((i - j) mod 3): wave w handles LDS rows lo + w + GS_NW it of
// the stage region.  In a row the colour-c points are every third column and
// lane l owns columns 3 l .. 3 l + 2, so each lane updates exactly one point
// per row; the row, the colour offset and the bounds are wave-uniform.
// `out` stores the tile's u once the stages are done; with the residual
// (H = GS_HE) the residuals then replace the interior tile values in LDS.
// With RES = 3 (H = GS_HR) they also replace the values one point beyond
// the interior on the low-i and low-j sides, where the three stages have
// left u final two points out.

template <class T, bool VARK, bool PROL, int TJ, int RES, class Out>
__device__ __forceinline__ void gs_tile3(const LevelDev& L, const FaceInfo& fi, int n, int i0, int j0,
                                         int64_t fb, const T* __restrict__ uin, const T* __restrict__ f,
                                         const T* __restrict__ kap, int backward, T (*us)[GS_W],
                                         T (*ks)[GS_W], const ProlTile<T>& pt, Out out, double& acc) {
    constexpr int H = gs_halo(RES);
    // first LDS row and column of the residual region
    constexpr int RL = RES == 3 ? H - 1 : H;
    using G = GsTile<TJ, H>;
    const int wv = wave_id(), lane = threadIdx.x & 63;
    T ur[G::RPW][3], kr[VARK ? G::RPW : 1][3], fr[3][G::IT3];
    gs_load_u<T, VARK, PROL, TJ, H>(n, i0, j0, fb, uin, kap, ur, kr, fi, pt, us);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int c = backward ? 2 - s : s, h = H - 1 - s;
        const int lo = H - h, hi_i = H + G::TI + h, hi_j = H + TJ + h;
#pragma unroll
        for (int it = 0; it < G::IT3; ++it) {
            const int r = lo + wv + GS_NW * it, j = j0 + r;
            const int tx = pmod(c + j - i0, 3) + 3 * lane, i = i0 + tx;
            const bool upd = r < hi_j && tx >= lo && tx < hi_i && j >= 1 && i >= 1 && i + j <= n - 2;
            fr[s][it] = upd ? f[fb + row_start(n, upd ? j : 0) + i] : (T)0;
        }
    }
    gs_store_u<T, VARK, TJ, H>(us, ks, ur, kr);
    const W7<T> w = face_weights<T>(OP_LAPLACE, fi, L.inv4l, (const T*)nullptr, 0, 0, 0);
    const T invc = (T)1 / w.c;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int c = backward ? 2 - s : s, h = H - 1 - s;
        const int lo = H - h, hi_i = H + G::TI + h, hi_j = H + TJ + h;
#pragma unroll
        for (int it = 0; it < G::IT3; ++it) {
            const int r = lo + wv + GS_NW * it, j = j0 + r;
            if (r >= hi_j) break;
            int tx = pmod(c + j - i0, 3) + 3 * lane;
            const int i = i0 + tx;
            const bool upd = tx >= lo && tx < hi_i && j >= 1 && i >= 1 && i + j <= n - 2;
            tx = upd ? tx : H;        // keep the neighbour reads inside the tile
            const T val = gs_point<T, VARK>(fi, w, invc, fr[s][it], us, ks, r, tx);
            if (upd) us[r][tx] = val;
        }
        __syncthreads();
    }
    if (RES == 0) {
        out();
        return;
    }
    if (RES == 2) {
        // squared residuals of the tile's core points (no neighbour on a
        // macro-edge, whose values the later edge stages still change)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int c = backward ? 2 - s : s, lo = 1 + s;
#pragma unroll
            for (int it = 0; it < G::IT3; ++it) {
                const int r = lo + wv + GS_NW * it, j = j0 + r;
                if (r < H || r >= H + TJ) continue;
                int tx = pmod(c + j - i0, 3) + 3 * lane;
                const int i = i0 + tx;
                const bool core = tx >= H && tx < H + G::TI && j >= 2 && i >= 2 && i + j <= n - 3;
                tx = core ? tx : H;
                const double v = (double)gs_resid<T, VARK>(fi, w, fr[s][it], us, ks, r, tx);
                acc += core ? v * v : 0.0;
            }
        }
        out();
        return;
    }
    // residual at the interior tile points, each found in the stage of its colour
    T res[3][G::IT3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int c = backward ? 2 - s : s, lo = 1 + s;
#pragma unroll
        for (int it = 0; it < G::IT3; ++it) {
            const int r = lo + wv + GS_NW * it, j = j0 + r;
            res[s][it] = (T)0;
            if (r < RL || r >= H + TJ) continue;
            int tx = pmod(c + j - i0, 3) + 3 * lane;
            const int i = i0 + tx;
            const bool in = tx >= RL && tx < H + G::TI && j >= 1 && i >= 1 && i + j <= n - 2;
            tx = in ? tx : H;
            const T v = gs_resid<T, VARK>(fi, w, fr[s][it], us, ks, r, tx);
            res[s][it] = in ? v : (T)0;
        }
    }
    out();
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int c = backward ? 2 - s : s, lo = 1 + s;
#pragma unroll
        for (int it = 0; it < G::IT3; ++it) {
            const int r = lo + wv + GS_NW * it, j = j0 + r;
            if (r < RL || r >= H + TJ) continue;
            const int tx = pmod(c + j - i0, 3) + 3 * lane, i = i0 + tx;
            if (tx >= RL && tx < H + G::TI && j >= 1 && i >= 1 && i + j <= n - 2) us[r][tx] = res[s][it];
        }
    }
    __syncthreads();
}

// Two colours (faces with an exact right angle): slots map densely onto the
// colour-c points, every second column or every second row.

template <int TJ, int H>
__device__ __forceinline__ bool gs_decode2(int idx, int rule, int c, int h, int i0, int j0, int& r,
                                           int& tx) {
    const int lo = H - h, hi_i = H + GsTile<TJ, H>::TI + h, hi_j = H + TJ + h;
    if (rule == 3) {
        const int rr = idx / GS_W, m = idx - rr * GS_W;
        r = lo + pmod(c - (j0 + lo), 2) + 2 * rr;
        tx = m;
        if (tx < lo) return false;
    } else {
        const int rr = idx / (GS_W / 2), m = idx - rr * (GS_W / 2);
        r = lo + rr;
        const int off = rule == 1 ? pmod(c - (j0 + r) - i0, 2) : pmod(c - i0, 2);
        tx = lo + pmod(off - lo, 2) + 2 * m;
    }
    return r < hi_j && tx < hi_i;
}

template <class T, bool VARK, bool PROL, int TJ, int RES, class Out>
__device__ __forceinline__ void gs_tile2(const LevelDev& L, const FaceInfo& fi, int n, int i0, int j0,
                                         int64_t fb, const T* __restrict__ uin, const T* __restrict__ f,
                                         const T* __restrict__ kap, int backward, T (*us)[GS_W],
                                         T (*ks)[GS_W], const ProlTile<T>& pt, Out out,
                                         T* __restrict__ rout, double& acc) {
    constexpr int H = RES ? GS_HE : GS_H;
    using G = GsTile<TJ, H>;
    const int rule = fi.colour_rule;
    const FaceGhosts gh = face_ghosts(L, fi);
    T ur[G::RPW][3], kr[VARK ? G::RPW : 1][3], fr[2][G::IT2];
    gs_load_u<T, VARK, PROL, TJ, H>(n, i0, j0, fb, uin, kap, ur, kr, fi, pt, us);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int c = backward ? 1 - s : s, h = H - 2 - s;
#pragma unroll
        for (int it = 0; it < G::IT2; ++it) {
            int r, tx;
            const bool ok = gs_decode2<TJ, H>(threadIdx.x + it * GS_NT, rule, c, h, i0, j0, r, tx);
            const int j = j0 + r, i = i0 + tx;
            const bool upd = ok && j >= 1 && i >= 1 && i + j <= n - 2;
            fr[s][it] = upd ? f[fb + row_start(n, upd ? j : 0) + i] : (T)0;
        }
    }
    gs_store_u<T, VARK, TJ, H>(us, ks, ur, kr);
    const W7<T> w = face_weights<T>(OP_LAPLACE, fi, L.inv4l, (const T*)nullptr, 0, 0, 0);
    const T invc = (T)1 / w.c;
    __syncthreads();
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int c = backward ? 1 - s : s, h = H - 2 - s;
#pragma unroll
        for (int it = 0; it < G::IT2; ++it) {
            int r, tx;
            const bool ok = gs_decode2<TJ, H>(threadIdx.x + it * GS_NT, rule, c, h, i0, j0, r, tx);
            const int j = j0 + r, i = i0 + tx;
            if (!(ok && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
            us[r][tx] = gs_point<T, VARK>(fi, w, invc, fr[s][it], us, ks, r, tx);
        }
        __syncthreads();
    }
    out();
    if (RES == 0) return;
    if (RES == 2) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int c = backward ? 1 - s : s, h = H - 2 - s;
#pragma unroll
            for (int it = 0; it < G::IT2; ++it) {
                int r, tx;
                const bool ok = gs_decode2<TJ, H>(threadIdx.x + it * GS_NT, rule, c, h, i0, j0, r, tx);
                const int j = j0 + r, i = i0 + tx;
                if (!(ok && r >= H && r < H + TJ && tx >= H && tx < H + G::TI && j >= 2 && i >= 2 &&
                      i + j <= n - 3))
                    continue;
                const double v = (double)gs_resid<T, VARK>(fi, w, fr[s][it], us, ks, r, tx);
                acc += v * v;
            }
        }
        return;
    }
    // residuals straight from the final LDS values to rout with their
    // ghost-row copies (faces with a right angle are few, so this path keeps
    // registers low rather than staging through LDS)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int c = backward ? 1 - s : s, h = H - 2 - s;
#pragma unroll
        for (int it = 0; it < G::IT2; ++it) {
            int r, tx;
            const bool ok = gs_decode2<TJ, H>(threadIdx.x + it * GS_NT, rule, c, h, i0, j0, r, tx);
            const int j = j0 + r, i = i0 + tx;
            if (!(ok && r >= H && r < H + TJ && tx >= H && tx < H + G::TI && j >= 1 && i >= 1 && i + j <= n - 2))
                continue;
            const T v = gs_resid<T, VARK>(fi, w, fr[s][it], us, ks, r, tx);
            rout[fb + row_start(n, j) + i] = v;
            push_face_near(gh, n, rout, i, j, v);
        }
    }
}

// NCOL selects the faces this launch handles (3: general faces, 2: faces
// with a right angle); copies of edge and vertex blocks are done by the
// extra blocks of the launch with with_copy = 1.  PROL: the sweep starts
// from uin + P uc (the coarse correction of level Lc), which is then never
// stored on its own: tiles add it as they load, copy blocks as they copy.
// RES: the residual variant; rout receives f - A uout at the interior face
// points and their copies in the edge ghost rows (the edge and vertex
// residuals and the remaining copies are left to an edge/vertex pass).
// Three-colour tiles stage the residuals through LDS for row-wise stores;
// two-colour tiles store them point by point.  RES = 2 (backward sweeps):
// every block writes partials[blockIdx.x], the sum of the squared residuals
// of its tile's core points (0 for blocks without a tile); the points next
// to or on the macro-edges are left to a pass after the edge stages.
// RES = 3 (three colours only): the residual is restricted where it is
// formed.  Every coarse interior face point of level Lc has its fine point
// in exactly one tile interior (the tile origins and sizes are even), and
// its fine neighbours lie in that interior or one point beyond it on the
// low sides, where the residual is formed too; fcout receives the
// restriction there, with the weights and summation order of k_restrict.
// rout then receives only the ghost-row copies of the near-edge residuals,
// which the edge restriction reads; the face residuals themselves are never
// stored.
template <class T, bool VARK, int NCOL, bool PROL, int TJ, int RES>
__global__ __launch_bounds__(GS_NT) void k_face_gs_fused(LevelDev L, const T* __restrict__ uin,
                                                         T* __restrict__ uout, const T* __restrict__ f,
                                                         const T* __restrict__ kap, int backward,
                                                         int nblk_tiles, int with_copy, LevelDev Lc,
                                                         const T* __restrict__ uc, T* __restrict__ rout,
                                                         double* __restrict__ partials, T* __restrict__ fcout) {
    static_assert(RES != 3 || NCOL == 3, "the restricting sweep is three-colour only");
    constexpr int H = gs_halo(RES);
    constexpr int TI = GsTile<TJ, H>::TI;
    constexpr int T16 = TJ == GS_TJ16 ? 1 : 0;
    static_assert(RES == 3 ? (TJ == GS_TJ16 || TJ == GS_TJR) : (TJ == GS_TJ16 || TJ == GS_TJ),
                  "tile height must match the tile list");
    __shared__ T us[GsTile<TJ, H>::R][GS_W];
    __shared__ T ks[VARK ? GsTile<TJ, H>::R : 1][GS_W];
    __shared__ double sm[RES == 2 ? GS_NW + 1 : 1];
    const int G = gridDim.x;                              // multiple of 8
    const int b = blockIdx.x;
    const int logical = (b & 7) * (G >> 3) + (b >> 3);    // contiguous tiles per XCD
    const int n = L.n;
    if (logical >= nblk_tiles) {
        if (RES == 2 && threadIdx.x == 0) partials[b] = 0.0;
        if (!with_copy) return;
        // edge points (k = 0..n-1) and vertex blocks
        const int cb = logical - nblk_tiles, ncb = G - nblk_tiles;
        const int64_t ne = (int64_t)L.E * n, nv = (int64_t)L.V * L.vert_stride;
        for (int64_t t = (int64_t)cb * GS_NT + threadIdx.x; t < ne + nv; t += (int64_t)ncb * GS_NT) {
            const int64_t off = t < ne ? L.edge_base + (t / n) * L.edge_stride + (t % n)
                                       : L.vert_base + (t - ne);
            T v = uin[off];
            if (PROL) v += prol_low<T>(L, Lc, uc, t);
            uout[off] = v;
        }
        return;
    }
    const int ntl = L.n_gs_tl[gs_list(RES)][T16];
    const int face = logical / ntl;
    const FaceInfo& fi = L.faces[face];
    if (fi.ncolours != NCOL) {
        if (RES == 2 && threadIdx.x == 0) partials[b] = 0.0;
        return;
    }
    const int2 tl = L.gs_tl[gs_list(RES)][T16][logical % ntl];
    const int i0 = tl.x * TI - H, j0 = tl.y * TJ - H;   // LDS origin
    const int64_t fb = face_base(L, face);
    const ProlTile<T> pt{uc, PROL ? face_base(Lc, face) : 0, Lc.n};
    const int wv = wave_id(), lane = threadIdx.x & 63;
    auto out = [&]() {
        // tile points (interior updated, ring copied) to uout
        for (int r = H + wv; r < H + TJ; r += GS_NW) {
            const int j = j0 + r;
            if (j >= n) break;
            const int64_t rb = fb + row_start(n, j);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int tx = lane + 64 * c, i = i0 + tx;
                if (tx >= H && tx < H + TI && i <= n - 1 - j) uout[rb + i] = us[r][tx];
            }
        }
        // near-edge rows into the edge ghost rows of uout (edge order)
        if (!fi.bside[0] && tl.y == 0) {            // (m, 1)
            for (int t = threadIdx.x; t < TI; t += GS_NT) {
                const int m = tl.x * TI + t;
                if (m <= n - 2)
                    uout[edge_ghost(L, fi.edge[0], fi.slot[0]) + (fi.rev[0] ? n - 2 - m : m)] = us[1 - j0][H + t];
            }
        }
        if (!fi.bside[1] && tl.x == 0) {            // (1, m)
            for (int t = threadIdx.x; t < TJ; t += GS_NT) {
                const int m = tl.y * TJ + t;
                if (m <= n - 2)
                    uout[edge_ghost(L, fi.edge[1], fi.slot[1]) + (fi.rev[1] ? n - 2 - m : m)] = us[H + t][1 - i0];
            }
        }
        if (!fi.bside[2]) {                         // (n-2-m, m)
            for (int t = threadIdx.x; t < TJ; t += GS_NT) {
                const int m = tl.y * TJ + t, i = n - 2 - m;
                if (m <= n - 2 && i >= tl.x * TI && i < tl.x * TI + TI)
                    uout[edge_ghost(L, fi.edge[2], fi.slot[2]) + (fi.rev[2] ? n - 2 - m : m)] = us[H + t][i - i0];
            }
        }
    };
    double acc = 0.0;
    if constexpr (NCOL == 3)
        gs_tile3<T, VARK, PROL, TJ, RES>(L, fi, n, i0, j0, fb, uin, f, kap, backward, us, VARK ? ks : nullptr,
                                         pt, out, acc);
    else
        gs_tile2<T, VARK, PROL, TJ, RES>(L, fi, n, i0, j0, fb, uin, f, kap, backward, us, VARK ? ks : nullptr,
                                         pt, out, rout, acc);
    if (RES == 2) {
        const double t = block_sum<GS_NT>(acc, sm);
        if (threadIdx.x == 0) partials[b] = t;
        return;
    }
    if ((RES != 1 && RES != 3) || NCOL == 2) return;
    if (RES == 3) {
        // coarse points whose fine point (2I, 2J) lies in the tile interior
        static_assert(TI % 2 == 0 && TJ % 2 == 0, "tiles must start on coarse points");
        constexpr int CI = TI / 2, CJ = TJ / 2;
        const int nc = Lc.n, I0 = tl.x * CI, J0 = tl.y * CJ;
        const int64_t cb = face_base(Lc, face);
        for (int t = threadIdx.x; t < CI * CJ; t += GS_NT) {
            const int jj = t / CI, ii = t - jj * CI, I = I0 + ii, J = J0 + jj;
            if (I < 1 || J < 1 || I + J > nc - 2) continue;
            const int r = H + 2 * jj, tx = H + 2 * ii;
            const T nb = us[r][tx + 1] + us[r][tx - 1] + us[r + 1][tx] + us[r - 1][tx] + us[r - 1][tx + 1] +
                         us[r + 1][tx - 1];
            fcout[cb + row_start(nc, J) + I] = us[r][tx] + (T)0.5 * nb;
        }
    }
    // interior residuals (now in LDS) to rout, with the ghost-row copies of
    // the near-edge ones: rows 1 .. n-3 hold interior points
    for (int r = H + wv; RES == 1 && r < H + TJ; r += GS_NW) {
        const int j = j0 + r;
        if (j > n - 3) break;
        if (j < 1) continue;
        const int64_t rb = fb + row_start(n, j);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int tx = lane + 64 * c, i = i0 + tx;
            if (tx >= H && tx < H + TI && i >= 1 && i + j <= n - 2) rout[rb + i] = us[r][tx];
        }
    }
    if (!fi.bside[0] && tl.y == 0) {                // (m, 1)
        for (int t = threadIdx.x; t < TI; t += GS_NT) {
            const int m = tl.x * TI + t;
            if (m >= 1 && m <= n - 3)
                rout[edge_ghost(L, fi.edge[0], fi.slot[0]) + (fi.rev[0] ? n - 2 - m : m)] = us[1 - j0][H + t];
        }
    }
    if (!fi.bside[1] && tl.x == 0) {                // (1, m)
        for (int t = threadIdx.x; t < TJ; t += GS_NT) {
            const int m = tl.y * TJ + t;
            if (m >= 1 && m <= n - 3)
                rout[edge_ghost(L, fi.edge[1], fi.slot[1]) + (fi.rev[1] ? n - 2 - m : m)] = us[H + t][1 - i0];
        }
    }
    if (!fi.bside[2]) {                             // (n-2-m, m)
        for (int t = threadIdx.x; t < TJ; t += GS_NT) {
            const int m = tl.y * TJ + t, i = n - 2 - m;
            if (m >= 1 && m <= n - 3 && i >= tl.x * TI && i < tl.x * TI + TI)
                rout[edge_ghost(L, fi.edge[2], fi.slot[2]) + (fi.rev[2] ? n - 2 - m : m)] = us[H + t][i - i0];
        }
    }
}

// Streamed multicolour face sweep (plain sweep of the three-colour faces).
// One wave per smoother tile (TI = GS_W - 2 GS_H columns from i0, GS_TJ
// rows from j0); lane l keeps columns i0 - 3 + 3 l .. i0 - 1 + 3 l of the
// rows it holds in registers, so that in every colour stage it updates
// exactly one point of a row (colour (i - j) mod 3, i0 a multiple of 3).
// Walking up the rows, at row s the wave applies the first stage to row
// s + 2, the second to row s + 1 and the third to row s, in place: a stage
// reads only points of the other two colours, which then hold the values
// that separate colour passes over the whole face would give them, so row s
// is final and is stored.  The east and west neighbours of a lane's outer
// columns come from the neighbouring lanes by whole-wave shifts; the three
// outer columns on each side are the strip's halo, wrong after the first
// stage but never read by the stored columns.  Rows live in register rings
// of NU rows (the window s - 1 .. s + 3 plus rows loaded NU - 5 steps
// ahead; f rows s .. s + 2 plus rows loaded NU - 3 steps ahead), each lane's
// three values in one vector load that is always issued (rows clamped into
// the face), so that no load is waited on before its row is used.  Reads
// uin and writes uout like the tile sweep (extra blocks copy edges and
// vertex blocks; the face rings are stored with the rows); no LDS, no
// barrier.  The arithmetic of a point is that of gs_point.  Used for the
// plain FP32 sweep of levels with at least GS_STREAM_MIN tiles.
template <class T>
__device__ __forceinline__ T gs_lane_next(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
    } else {
        typedef int int2v __attribute__((ext_vector_type(2)));
        const int2v a = __builtin_bit_cast(int2v, v);
        const int2v r = {__builtin_amdgcn_update_dpp(0, a[0], 0x130, 0xf, 0xf, false),
                         __builtin_amdgcn_update_dpp(0, a[1], 0x130, 0xf, 0xf, false)};
        return __builtin_bit_cast(T, r);
    }
}
template <class T>
__device__ __forceinline__ T gs_lane_prev(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
    } else {
        typedef int int2v __attribute__((ext_vector_type(2)));
        const int2v a = __builtin_bit_cast(int2v, v);
        const int2v r = {__builtin_amdgcn_update_dpp(0, a[0], 0x138, 0xf, 0xf, false),
                         __builtin_amdgcn_update_dpp(0, a[1], 0x138, 0xf, 0xf, false)};
        return __builtin_bit_cast(T, r);
    }
}

// New value of the lane's column M of row c (rows s below, nn above; k rows
// likewise for the variable coefficient).
template <class T, bool VARK, int M>
__device__ __forceinline__ T gs_stream_point(const T* cot, const W7<T>& w, T invc, T fv, const T* rs,
                                             const T* rc, const T* rn, const T* ks, const T* kc, const T* kn) {
    const T uW = M == 0 ? gs_lane_prev(rc[2]) : rc[M == 0 ? 0 : M - 1];
    const T uE = M == 2 ? gs_lane_next(rc[0]) : rc[M == 2 ? 2 : M + 1];
    const T uS = rs[M], uN = rn[M];
    const T uSE = M == 2 ? gs_lane_next(rs[0]) : rs[M == 2 ? 2 : M + 1];
    const T uNW = M == 0 ? gs_lane_prev(rn[2]) : rn[M == 0 ? 0 : M - 1];
    if (!VARK) return (fv - (w.e * (uE + uW) + w.n * (uN + uS) + w.se * (uSE + uNW))) * invc;
    const T k0 = kc[M], kN = kn[M], kS = ks[M];
    const T kW = M == 0 ? gs_lane_prev(kc[2]) : kc[M == 0 ? 0 : M - 1];
    const T kE = M == 2 ? gs_lane_next(kc[0]) : kc[M == 2 ? 2 : M + 1];
    const T kSE = M == 2 ? gs_lane_next(ks[0]) : ks[M == 2 ? 2 : M + 1];
    const T kNW = M == 0 ? gs_lane_prev(kn[2]) : kn[M == 0 ? 0 : M - 1];
    const T c0 = cot[0], c1 = cot[1], c2 = cot[2];
    const T third = (T)(1.0 / 3.0), hf = (T)0.5;
    const T t1 = (k0 + kE + kN) * third, t2 = (kSE + kE + k0) * third;
    const T t3 = (kW + k0 + kNW) * third, t4 = (kS + k0 + kW) * third;
    const T t5 = (k0 + kN + kNW) * third, t6 = (kS + kSE + k0) * third;
    W7<T> v;
    v.e = -hf * c2 * (t1 + t2);
    v.w = -hf * c2 * (t3 + t4);
    v.n = -hf * c1 * (t1 + t5);
    v.s = -hf * c1 * (t6 + t4);
    v.se = -hf * c0 * (t6 + t2);
    v.nw = -hf * c0 * (t3 + t5);
    v.c = -(v.e + v.w + v.n + v.s + v.se + v.nw);
    return (fv - (v.e * uE + v.w * uW + v.n * uN + v.s * uS + v.se * uSE + v.nw * uNW)) / v.c;
}

template <class T>
struct alignas(sizeof(T)) GsTrip { T v[3]; };   // a lane's three columns of a row

constexpr int GS_SNT = 256;     // threads per block of the streamed sweep (independent waves)
constexpr bool GS_STREAM = true; // plain FP32 sweeps of three-colour faces use the streamed kernel
constexpr int GS_NU = 6;         // its register ring rows
constexpr int GS_STREAM_MIN = 4096;   // fewest tiles (waves) for which it is used

template <class T, bool VARK, bool BACK, int NU>
__global__ __launch_bounds__(GS_SNT) void k_face_gs_stream(LevelDev L, const T* __restrict__ uin,
                                                           T* __restrict__ uout, const T* __restrict__ f,
                                                           const T* __restrict__ kap, int nblk) {
    constexpr int TI = GS_W - 2 * GS_H, TJ = GS_TJ;
    static_assert(TI % 3 == 0 && TJ % 3 == 0 && NU % 3 == 0 && NU >= 6 && NU <= 9,
                  "colour positions repeat every three rows and the loop is written for 6 or 9 ring rows");
    const int n = L.n;
    if ((int)blockIdx.x >= nblk) {
        // edge points (k = 0..n-1) and vertex blocks
        const int cb = blockIdx.x - nblk, ncb = gridDim.x - nblk;
        const int64_t ne = (int64_t)L.E * n, nv = (int64_t)L.V * L.vert_stride;
        for (int64_t t = (int64_t)cb * GS_SNT + threadIdx.x; t < ne + nv; t += (int64_t)ncb * GS_SNT) {
            const int64_t off = t < ne ? L.edge_base + (t / n) * L.edge_stride + (t % n) : L.vert_base + (t - ne);
            uout[off] = uin[off];
        }
        return;
    }
    const int lane = threadIdx.x & 63, wv = wave_id();
    // consecutive logical blocks on one XCD (hardware block b runs on XCD b mod 8)
    const int b = blockIdx.x, lb = (b & 7) * (nblk >> 3) + (b >> 3);
    const int ntl = L.n_gs_tl[0][0];
    const int task = lb * (GS_SNT / 64) + wv;
    if (task >= L.F * ntl) return;                      // the whole wave
    const int face = task / ntl;
    const FaceInfo& fi = L.faces[face];
    if (fi.ncolours != 3) return;
    const int2 tl = L.gs_tl[0][0][task % ntl];
    const int i0 = tl.x * TI, j0 = tl.y * TJ;
    const int s_end = min(j0 + TJ, n - i0);            // rows that hold a point of the strip
    const int64_t fb = face_base(L, face);
    const int xc = i0 - 3 + 3 * lane;                  // the lane's first column
    const W7<T> w = face_weights<T>(OP_LAPLACE, fi, L.inv4l, (const T*)nullptr, 0, 0, 0);
    const T invc = (T)1 / w.c;
    // face data the rows need, read once into registers (read in divergent
    // code they would be vector loads, and waiting for one waits for every
    // row load in flight)
    const T cot[3] = {(T)fi.cot[0], (T)fi.cot[1], (T)fi.cot[2]};
    int64_t gh[3];
    int ghr[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        gh[q] = fi.bside[q] ? -1 : edge_ghost(L, fi.edge[q], fi.slot[q]);
        ghr[q] = fi.rev[q];
    }

    // Row j of a field (j clamped into the face): the lane's three values in
    // one vector load.  A lane holding a point of the row loads from its own
    // first column (its last values may lie past the row's padding, inside
    // the next row of the face); any other lane loads the row's first three
    // slots.  Values outside the triangle are never read by an update or
    // stored.
    // The row starts of the three row streams (u and k loads, f loads,
    // stores) advance by one row per step; a stream's row is clamped to
    // 0 .. jm for its start, where jm is the last row the stream needs (the
    // loop runs whole rounds and loads ahead, so without the cap a tile
    // would fetch up to five rows of the next tile from memory; with it,
    // those steps reload the cap row, which the cache still holds).
    struct RowPos {
        int j, rs, jm;   // row, the start of clamp(j, 0, jm), the cap
    };
    auto row_at = [&](int j, int jm) { return RowPos{j, row_start(n, min(max(j, 0), jm)), jm}; };
    auto advance = [&](RowPos& r) {
        const int jn = r.j + 1;
        r.rs = jn <= 0 ? 0 : (jn > r.jm ? r.rs : r.rs + 16 * ((n - r.j + 15) >> 4));
        r.j = jn;
    };
    const T* ub = uin + fb;
    const T* kb = VARK ? kap + fb : nullptr;
    const T* fbp = f + fb;
    auto load_row = [&](const T* __restrict__ base, const RowPos& r, T* v) {
        const int st = (xc >= 0 && xc <= n - 1 - min(max(r.j, 0), r.jm)) ? xc : 0;
        const GsTrip<T> t = *reinterpret_cast<const GsTrip<T>*>(base + r.rs + st);
        v[0] = t.v[0];
        v[1] = t.v[1];
        v[2] = t.v[2];
    };
    // ring slot of row r: (r - s0 + 1) mod NU, for u, k and f alike
    const int s0 = j0 - 4;
    T ur[NU][3], kr[VARK ? NU : 1][3], fr[NU][3];
#pragma unroll
    for (int q = 0; q < NU; ++q)
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            ur[q][m] = fr[q][m] = (T)0;
            if (VARK) kr[q][m] = (T)0;
        }
    // the last rows read: stage 1 runs up to row s_end + 1, reading u of
    // the row above and f of its own row
    RowPos pu = row_at(s0 + 1, min(s_end + 2, n - 1)), pf = row_at(s0 + 2, min(s_end + 1, n - 1));
    RowPos ps = row_at(j0, n - 1);
#pragma unroll
    for (int q = 2; q <= NU - 2; ++q) {                 // u (k) rows s0 + 1 .. s0 + NU - 3
        load_row(ub, pu, ur[q]);
        if (VARK) load_row(kb, pu, kr[VARK ? q : 0]);
        advance(pu);
    }
#pragma unroll
    for (int q = 3; q <= NU - 1; ++q) {                 // f rows s0 + 2 .. s0 + NU - 2
        load_row(fbp, pf, fr[q]);
        advance(pf);
    }

    auto step = [&](auto phase, int s) {
        constexpr int P = decltype(phase)::value;
        constexpr int SL = (P + NU - 1) % NU;           // slot of u row s - 2 (free): row s + NU - 2
        load_row(ub, pu, ur[SL]);                       // row s + NU - 2
        if (VARK) load_row(kb, pu, kr[VARK ? SL : 0]);
        load_row(fbp, pf, fr[P]);                       // row s + NU - 1 into the slot of f row s - 1
        advance(pu);
        advance(pf);
        if (s >= s_end) return;
        constexpr int SM = (2 + P) % 3;                 // s mod 3 (s0 = 2 mod 3)
        constexpr int C0 = BACK ? 2 : 0, C1 = 1, C2 = BACK ? 0 : 2;
        auto stage = [&](auto col, auto dj) {
            // stage of colour C on row s + DJ
            constexpr int C = decltype(col)::value, DJ = decltype(dj)::value;
            constexpr int M = (C + SM + DJ) % 3;       // the lane's column of colour C in that row
            constexpr int RC = (P + DJ + 1) % NU, RS = (P + DJ) % NU, RN = (P + DJ + 2) % NU;
            const int j = s + DJ, x = xc + M;
            const T v = gs_stream_point<T, VARK, M>(cot, w, invc, fr[RC][M], ur[RS], ur[RC], ur[RN],
                                                    VARK ? kr[VARK ? RS : 0] : nullptr,
                                                    VARK ? kr[VARK ? RC : 0] : nullptr,
                                                    VARK ? kr[VARK ? RN : 0] : nullptr);
            // interior points only: 1 <= x <= n - 2 - j on rows 1 <= j <= n - 3
            // (cnt = number of interior points of the row, 0 on other rows)
            const int cnt = (j >= 1 && j <= n - 3) ? n - 2 - j : 0;
            ur[RC][M] = (unsigned)(x - 1) < (unsigned)cnt ? v : ur[RC][M];
        };
        stage(std::integral_constant<int, C0>(), std::integral_constant<int, 2>());
        if (s >= j0 - 2) stage(std::integral_constant<int, C1>(), std::integral_constant<int, 1>());
        if (s >= j0) {
            stage(std::integral_constant<int, C2>(), std::integral_constant<int, 0>());
            // row s is final: store the strip's columns (lanes 1 .. 62; one
            // vector store where all three lie in the triangle) and the
            // near-edge copies
            T* rp = uout + fb + ps.rs;
            advance(ps);
            T* row = ur[(P + 1) % NU];
            const int xe = n - 1 - s;                   // last column of row s
            GsTrip<T> t;
            t.v[0] = row[0];
            t.v[1] = row[1];
            t.v[2] = row[2];
            const bool mid = lane >= 1 && lane <= 62;
            if (xe >= i0 + TI - 1) {                    // the whole strip lies in the row
                if (mid) *reinterpret_cast<GsTrip<T>*>(rp + xc) = t;
            } else if (mid && xc <= xe) {
                if (xc + 2 <= xe) {
                    *reinterpret_cast<GsTrip<T>*>(rp + xc) = t;
                } else {
                    rp[xc] = row[0];
                    if (xc + 1 <= xe) rp[xc + 1] = row[1];
                }
            }
            // copies in the edge ghost rows (rows j = 1, i = 1, i + j = n - 2),
            // each behind a test that is uniform over the wave
            if (s == 1 && gh[0] >= 0) {
#pragma unroll
                for (int m = 0; m < 3; ++m) {
                    const int x = xc + m;
                    if (mid && x <= n - 2) uout[gh[0] + (ghr[0] ? n - 2 - x : x)] = row[m];
                }
            }
            if (i0 == 0 && s <= n - 2 && gh[1] >= 0) {
                if (lane == 1) uout[gh[1] + (ghr[1] ? n - 2 - s : s)] = row[1];   // x = 1
            }
            if (n - 2 - s >= i0 && n - 2 - s < i0 + TI && gh[2] >= 0) {
                const int m = n - 2 - s - xc;               // the lane holding x = n - 2 - s
                if (m >= 0 && m < 3) uout[gh[2] + (ghr[2] ? n - 2 - s : s)] = m == 0 ? row[0] : (m == 1 ? row[1] : row[2]);
            }
        }
    };
    const int rounds = (s_end - s0 + NU - 1) / NU;
    for (int k = 0; k < rounds; ++k) {
        const int s = s0 + k * NU;
        step(std::integral_constant<int, 0>(), s);
        step(std::integral_constant<int, 1>(), s + 1);
        step(std::integral_constant<int, 2>(), s + 2);
        step(std::integral_constant<int, 3 % NU>(), s + 3);
        step(std::integral_constant<int, 4 % NU>(), s + 4);
        step(std::integral_constant<int, 5 % NU>(), s + 5);
        if constexpr (NU == 9) {
            step(std::integral_constant<int, 6 % NU>(), s + 6);
            step(std::integral_constant<int, 7 % NU>(), s + 7);
            step(std::integral_constant<int, 8 % NU>(), s + 8);
        }
    }
}

// The point operator of k_apply_low extended to the face points, taken from LDS tiles:
// the smoother's TI x TJ tiles, each loaded with a one-point halo in one
// round of independent row loads (f of the block's points into registers
// alongside), then every interior point formed from LDS.  The blocks from gt
// on take the edge and vertex points.  Modes and outputs as k_apply_low; for the
// norm modes every block writes partials[blockIdx.x] (0 without work).
template <class T, bool VARK, int MODE, int TJ>
__global__ __launch_bounds__(GS_NT) void k_apply_tiled(LevelDev L, int op, const T* __restrict__ x,
                                                       const T* __restrict__ f, T* __restrict__ y,
                                                       const T* __restrict__ kap, int nblk_tiles, int gt,
                                                       double* __restrict__ partials) {
    constexpr int TI = GsTile<TJ, GS_H>::TI, RA = TJ + 2, TL = TJ == GS_TJ16 ? 1 : 0;
    constexpr int RPW = (RA + GS_NW - 1) / GS_NW, KR = TJ / GS_NW;
    static_assert(TJ % GS_NW == 0, "tile rows must split evenly over the waves");
    static_assert(TI + 2 <= GS_W, "tile with halo must fit an LDS row");
    constexpr bool NORM = MODE == 1 || MODE == 4;
    __shared__ T xs[RA][GS_W];
    __shared__ T ks[VARK ? RA : 1][GS_W];
    __shared__ double sm[GS_NW + 1];
    const int b = blockIdx.x, n = L.n;
    const int wv = wave_id(), lane = threadIdx.x & 63;
    double acc = 0.0;
    if (b >= gt) {
        const int64_t ne = (int64_t)L.E * (n - 2);
        for (int64_t t = (int64_t)(b - gt) * GS_NT + threadIdx.x; t < ne + L.V;
             t += (int64_t)(gridDim.x - gt) * GS_NT)
            apply_low_item<T, MODE>(L, op, x, f, y, kap, t, ne, acc);
    } else {
        const int logical = (b & 7) * (gt >> 3) + (b >> 3);   // contiguous tiles per XCD
        if (logical < nblk_tiles) {
            const int ntl = L.n_gs_tl[0][TL];
            const int face = logical / ntl;
            const FaceInfo& fi = L.faces[face];
            const FaceGhosts gh = face_ghosts(L, fi);
            const int2 tl = L.gs_tl[0][TL][logical % ntl];
            const int i0 = tl.x * TI - 1, j0 = tl.y * TJ - 1;   // LDS origin
            const int64_t fb = face_base(L, face);
            // all loads first (tile into registers, then f), LDS stores after,
            // so that the loads are in flight together
            T xr[RPW][3], kr[VARK ? RPW : 1][3];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int r = wv + GS_NW * q, j = j0 + r;
                const int64_t rb = fb + row_start(n, j < 0 ? 0 : (j > n ? n : j));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    const bool in = r < RA && tx < TI + 2 && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
                    xr[q][c] = in ? x[rb + i] : (T)0;
                    if (VARK) kr[q][c] = in ? kap[rb + i] : (T)0;
                }
            }
            T fr[KR][3];
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int r = 1 + wv + GS_NW * k, j = j0 + r;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    const bool pt = MODE >= 1 && MODE != 3 && tx >= 1 && tx <= TI && j >= 1 && i >= 1 &&
                                    i + j <= n - 2;
                    fr[k][c] = pt ? f[fb + row_start(n, pt ? j : 0) + i] : (T)0;
                }
            }
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int r = wv + GS_NW * q;
                if (r >= RA) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[r][lane + 64 * c] = xr[q][c];
                    if (VARK) ks[r][lane + 64 * c] = kr[q][c];
                }
            }
            const W7<T> wf = face_weights<T>(VARK ? OP_LAPLACE : op, fi, L.inv4l, (const T*)nullptr, 0, 0, 0);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int r = 1 + wv + GS_NW * k, j = j0 + r;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    if (!(tx >= 1 && tx <= TI && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
                    const W7<T> w = VARK ? gs_weights_lds<T>(fi, ks, r, tx) : wf;
                    T v;
                    if (MODE == 3) {
                        v = xs[r][tx] / w.c;
                    } else {
                        v = w.c * xs[r][tx] + w.e * xs[r][tx + 1] + w.w * xs[r][tx - 1] + w.n * xs[r + 1][tx] +
                            w.s * xs[r - 1][tx] + w.se * xs[r - 1][tx + 1] + w.nw * xs[r + 1][tx - 1];
                        if (MODE >= 1) v = fr[k][c] - v;
                        if (NORM) acc += (double)v * (double)v;
                        if (MODE == 2) v = v / w.c;
                    }
                    if (MODE == 4) continue;
                    y[fb + row_start(n, j) + i] = v;
                    push_face_near(gh, n, y, i, j, v);
                }
            }
        }
    }
    if (NORM && partials) {
        const double t = block_sum<GS_NT>(acc, sm);
        if (threadIdx.x == 0) partials[b] = t;
    }
}

// Outer step of mixed-precision refinement on FP64 x, FP32 correction e and
// FP64 f.  With UPD: v = x + e is the new iterate, written to xo with all
// copies (Dirichlet entries keep x); without: v = x and xo is untouched.
// The residual f - A v is formed in FP64, its squares summed per block in
// FP64 for the norm, and it is stored rounded to FP32 in r with all copies
// (0 on Dirichlet rows): the right-hand side of the next FP32 cycle.  Face
// points come from LDS tiles as in k_apply_tiled (the tile holds v with a
// one-point halo, loaded in one round of independent loads); the blocks from
// gt on take edges and vertices; every block writes partials[blockIdx.x].
template <bool UPD, bool VARK, int TJ>
__global__ __launch_bounds__(GS_NT) void k_mp_step_tiled(LevelDev L, int op, const double* __restrict__ x,
                                                         const float* __restrict__ e,
                                                         const double* __restrict__ f,
                                                         double* __restrict__ xo, float* __restrict__ r,
                                                         const double* __restrict__ kap, int nblk_tiles, int gt,
                                                         double* __restrict__ partials) {
    constexpr int TI = GsTile<TJ, GS_H>::TI, RA = TJ + 2, TL = TJ == GS_TJ16 ? 1 : 0;
    constexpr int RPW = (RA + GS_NW - 1) / GS_NW, KR = TJ / GS_NW;
    static_assert(TJ % GS_NW == 0, "tile rows must split evenly over the waves");
    __shared__ double vs[RA][GS_W];
    __shared__ double ks[VARK ? RA : 1][GS_W];
    __shared__ double sm[GS_NW + 1];
    const int b = blockIdx.x, n = L.n;
    const int wv = wave_id(), lane = threadIdx.x & 63;
    double acc = 0.0;
    if (b >= gt) {
        const int64_t ne = (int64_t)L.E * (n - 2);
        for (int64_t t = (int64_t)(b - gt) * GS_NT + threadIdx.x; t < ne + L.V;
             t += (int64_t)(gridDim.x - gt) * GS_NT)
            mp_low_item<UPD>(L, op, x, e, f, xo, r, kap, t, ne, acc);
    } else {
        const int logical = (b & 7) * (gt >> 3) + (b >> 3);
        if (logical < nblk_tiles) {
            const int ntl = L.n_gs_tl[0][TL];
            const int face = logical / ntl;
            const FaceInfo& fi = L.faces[face];
            const FaceGhosts gh = face_ghosts(L, fi);
            const int2 tl = L.gs_tl[0][TL][logical % ntl];
            const int i0 = tl.x * TI - 1, j0 = tl.y * TJ - 1;
            const int64_t fb = face_base(L, face);
            double vr[RPW][3], kr[VARK ? RPW : 1][3], fr[KR][3];
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int rr = wv + GS_NW * q, j = j0 + rr;
                const int64_t rb = fb + row_start(n, j < 0 ? 0 : (j > n ? n : j));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    const bool in = rr < RA && tx < TI + 2 && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
                    vr[q][c] = in ? (UPD ? x[rb + i] + (double)e[rb + i] : x[rb + i]) : 0.0;
                    if (VARK) kr[q][c] = in ? kap[rb + i] : 0.0;
                }
            }
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int rr = 1 + wv + GS_NW * k, j = j0 + rr;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    const bool pt = tx >= 1 && tx <= TI && j >= 1 && i >= 1 && i + j <= n - 2;
                    fr[k][c] = pt ? f[fb + row_start(n, pt ? j : 0) + i] : 0.0;
                }
            }
#pragma unroll
            for (int q = 0; q < RPW; ++q) {
                const int rr = wv + GS_NW * q;
                if (rr >= RA) continue;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    vs[rr][lane + 64 * c] = vr[q][c];
                    if (VARK) ks[rr][lane + 64 * c] = kr[q][c];
                }
            }
            const W7<double> wf = face_weights<double>(VARK ? OP_LAPLACE : op, fi, L.inv4l, (const double*)nullptr,
                                                       0, 0, 0);
            __syncthreads();
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const int rr = 1 + wv + GS_NW * k, j = j0 + rr;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    if (!(tx >= 1 && tx <= TI && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
                    const W7<double> w = VARK ? gs_weights_lds<double>(fi, ks, rr, tx) : wf;
                    const double v0 = vs[rr][tx];
                    const double v = fr[k][c] - (w.c * v0 + w.e * vs[rr][tx + 1] + w.w * vs[rr][tx - 1] +
                                                 w.n * vs[rr + 1][tx] + w.s * vs[rr - 1][tx] +
                                                 w.se * vs[rr - 1][tx + 1] + w.nw * vs[rr + 1][tx - 1]);
                    acc += v * v;
                    const int64_t p = fb + row_start(n, j) + i;
                    r[p] = (float)v;
                    push_face_near(gh, n, r, i, j, (float)v);
                    if (UPD) {
                        xo[p] = v0;
                        push_face_near(gh, n, xo, i, j, v0);
                    }
                }
            }
        }
    }
    const double t = block_sum<GS_NT>(acc, sm);
    if (threadIdx.x == 0) partials[b] = t;
}

// Squared residuals, one partial sum per block, of the points a backward
// sweep's face stage leaves out of its sum: the interior face points on the
// first row along each side (j = 1, i = 1, i + j = n - 2), enumerated per
// face as the row j = 1, the column i = 1 from j = 2, and the diagonal from
// j = 2 to n - 4; then the interior edge points and interior vertices.  Each
// interior unknown is in exactly one of the two sums.
template <class T>
__global__ __launch_bounds__(NT) void k_resnorm_rim(LevelDev L, int op, const T* __restrict__ x,
                                                    const T* __restrict__ f, const T* __restrict__ kap,
                                                    double* __restrict__ partials) {
    __shared__ double sm[NT / 64 + 1];
    const int n = L.n;
    const int64_t pf = n >= 5 ? 3 * (int64_t)n - 12 : 0;   // rim points per face
    const int64_t nfp = (int64_t)L.F * pf, ne = (int64_t)L.E * (n - 2);
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < nfp + ne + L.V; t += (int64_t)gridDim.x * NT) {
        T v = (T)0;
        if (t < nfp) {
            const int face = (int)(t / pf), q = (int)(t - face * pf);
            int i, j;
            if (q < n - 3) {
                i = q + 1;
                j = 1;
            } else if (q < 2 * n - 7) {
                i = 1;
                j = q - (n - 3) + 2;
            } else {
                j = q - (2 * n - 7) + 2;
                i = n - 2 - j;
            }
            const FaceInfo& fi = L.faces[face];
            const int64_t p = face_base(L, face) + row_start(n, j) + i;
            const int64_t up = row_start(n, j + 1) - row_start(n, j);
            const int64_t dn = row_start(n, j) - row_start(n, j - 1);
            const W7<T> w = face_weights<T>(op, fi, L.inv4l, kap, p, up, dn);
            v = f[p] - (w.c * x[p] + w.e * x[p + 1] + w.w * x[p - 1] + w.n * x[p + up] + w.s * x[p - dn] +
                        w.se * x[p - dn + 1] + w.nw * x[p + up - 1]);
        } else if (t < nfp + ne) {
            const int64_t te = t - nfp;
            const int e = (int)(te / (n - 2)), k = (int)(te % (n - 2)) + 1;
            const EdgeInfo& ei = L.edges[e];
            if (!ei.boundary) {
                const int64_t m = edge_main(L, e);
                v = f[m + k] - edge_apply<T>(op, L, ei, x, kap, m, edge_ghost(L, e, 0), edge_ghost(L, e, 1), k);
            }
        } else {
            const int vv = (int)(t - nfp - ne);
            const VertexInfo& vi = L.verts[vv];
            if (!vi.boundary) {
                const int64_t vb = vert_off(L, vv);
                v = f[vb] - vertex_apply<T>(op, L, vi, x, kap, vb);
            }
        }
        acc += (double)v * (double)v;
    }
    const double s = block_sum<NT>(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// Stage A (stage = 0): interior vertices and even-k points of interior
// edges; stage B (stage = 1): odd-k points.  The points of a stage are
// updated at once from the values before the stage; every update writes
// its copies.  Odd points next to a vertex of two edges of one face read
// each other in stage B, so stage B leaves those ghost-row copies alone and
// stage A (which reads none of them) refreshes them; stage = 2 only
// refreshes them.
template <class T>
__device__ __forceinline__ void low_gs_item(const LevelDev& L, int op, T* __restrict__ u, const T* __restrict__ f,
                                            const T* __restrict__ kap, int stage, int64_t t, int64_t ne) {
    const int n = L.n;
    if (t < ne) {
        // every edge, Dirichlet ones skipped: the values' addresses need only
        // the edge id, so they load together with the edge's metadata
        const int e = (int)(t / (n - 2)), k = (int)(t % (n - 2)) + 1;
        const EdgeInfo& ei = L.edges[e];
        const int64_t m = edge_main(L, e);
        if ((k & 1) != stage) {
            if (stage != 1 && (k & 1) && (k == 1 || k == n - 2)) {
                const T v = u[m + k];
                if (ei.boundary) return;
                push_corner_ghosts(L, u, ei, k, v);
            }
            return;
        }
        const int64_t g0 = edge_ghost(L, e, 0), g1 = edge_ghost(L, e, 1);
        const T um = u[m + k - 1], up = u[m + k + 1], a0 = u[g0 + k - 1], b0 = u[g0 + k];
        const T a1 = u[g1 + k - 1], b1 = u[g1 + k], fv = f[m + k];
        if (ei.boundary) return;
        const WE<T> w = edge_weights<T>(op, ei, L.inv4l, kap, m, g0, g1, k);
        const T off = w.al * um + w.ah * up + w.l0 * a0 + w.h0 * b0 + w.l1 * a1 + w.h1 * b1;
        const T v = (fv - off) / w.c;
        u[m + k] = v;
        push_edge(L, u, ei, k, v, false);
    } else {
        const int vv = (int)(t - ne);
        const VertexInfo& vi = L.verts[vv];
        const int64_t vb = vert_off(L, vv);
        const int2 db = *reinterpret_cast<const int2*>(&vi.deg);   // deg, boundary in one load
        const T fv = f[vb];
        if (db.y) return;
        T s = (T)0, c = (T)0;
        vertex_ring_sums<T>(op, vi, db.x, L.inv4l, kap, u, vb, s, c);
        c = (op == OP_MASS) ? c : -c;
        const T v = (fv - s) / c;
        u[vb] = v;
        push_vertex(L, u, vi, v);
    }
}

template <class T>
__global__ __launch_bounds__(NT) void k_low_gs(LevelDev L, int op, T* __restrict__ u,
                                               const T* __restrict__ f, const T* __restrict__ kap,
                                               int stage) {
    const int n = L.n;
    const int64_t ne = (int64_t)L.E * (n - 2);
    const int64_t nv = stage == 0 ? L.V : 0;
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < ne + nv; t += (int64_t)gridDim.x * NT)
        low_gs_item<T>(L, op, u, f, kap, stage, t, ne);
}

// Restriction, the transpose of linear interpolation: a coarse point gets
// the fine residual at its own position plus half of it at each fine
// neighbour; zero at coarse Dirichlet points.  r carries its ghost copies.
// Blocks [0, gf): coarse face points; [gf, gl): coarse edge and vertex
// points; [gl, gridDim.x): zero the coarse correction uc.
template <class T>
__global__ __launch_bounds__(NT) void k_restrict(LevelDev Lf, LevelDev Lc, const T* __restrict__ r,
                                                 T* __restrict__ fc, T* __restrict__ uc, int64_t uc_n,
                                                 int gf, int gl) {
    if ((int)blockIdx.x < gf) {
        FACE_ALL_LOOP(Lc, gf)
        (void)fi;
        if (!interior) continue;
        const int nf_ = Lf.n, jf = 2 * j;
        const int64_t q = face_base(Lf, face) + row_start(nf_, jf) + 2 * i;
        const int64_t upf = row_start(nf_, jf + 1) - row_start(nf_, jf);
        const int64_t dnf = row_start(nf_, jf) - row_start(nf_, jf - 1);
        const T nb = r[q + 1] + r[q - 1] + r[q + upf] + r[q - dnf] + r[q - dnf + 1] + r[q + upf - 1];
        fc[p] = r[q] + (T)0.5 * nb;
        }
    } else if ((int)blockIdx.x < gl) {
        const int nc = Lc.n;
        const int64_t ne = (int64_t)Lc.E * (nc - 2);
        for (int64_t t = (int64_t)(blockIdx.x - gf) * NT + threadIdx.x; t < ne + Lc.V;
             t += (int64_t)(gl - gf) * NT) {
            if (t < ne) {
                const int e = (int)(t / (nc - 2)), K = (int)(t % (nc - 2)) + 1;
                const int64_t mc = edge_main(Lc, e);
                if (Lc.edges[e].boundary) { fc[mc + K] = (T)0; continue; }
                const int64_t m = edge_main(Lf, e), g0 = edge_ghost(Lf, e, 0), g1 = edge_ghost(Lf, e, 1);
                const int k = 2 * K;
                const T nb = r[m + k - 1] + r[m + k + 1] + r[g0 + k - 1] + r[g0 + k] + r[g1 + k - 1] +
                             r[g1 + k];
                fc[mc + K] = r[m + k] + (T)0.5 * nb;
            } else {
                const int v = (int)(t - ne);
                const VertexInfo& vi = Lc.verts[v];
                const int64_t vc = vert_off(Lc, v);
                if (vi.boundary) { fc[vc] = (T)0; continue; }
                const int64_t vf = vert_off(Lf, v);
                const int deg = vi.deg;
                T nb = (T)0;
                for (int q0 = 0; q0 < deg; q0 += 4) {     // ring loads four at a time, summed in order
                    T rq[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) rq[k] = r[vf + 1 + (q0 + k < deg ? q0 + k : q0)];
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (q0 + k < deg) nb += rq[k];
                }
                fc[vc] = r[vf] + (T)0.5 * nb;
            }
        }
    } else {
        for (int64_t t = (int64_t)(blockIdx.x - gl) * NT + threadIdx.x; t < uc_n;
             t += (int64_t)(gridDim.x - gl) * NT)
            uc[t] = (T)0;
    }
}

// Restriction of the coarse edge and vertex points straight from the swept
// fine field x, after the sweep that restricts the face residuals (which
// leaves the edge and vertex residuals unformed): the fine residuals these
// points need (edge points k - 1, k, k + 1; a vertex and its ring, whose
// members are the first points of the incident edges) are formed here, with
// the arithmetic of k_apply_low's residual; the residuals of the face points
// next to the edges come from r's ghost rows.  The weights and the order of
// the sums are k_restrict's.  Blocks [gl, gridDim.x) zero the coarse
// correction uc.
template <class T>
__global__ __launch_bounds__(NT) void k_restrict_low(LevelDev Lf, LevelDev Lc, int op, const T* __restrict__ x,
                                                     const T* __restrict__ f, const T* __restrict__ kap,
                                                     const T* __restrict__ r, T* __restrict__ fc,
                                                     T* __restrict__ uc, int64_t uc_n, int gl) {
    if ((int)blockIdx.x < gl) {
        const int nc = Lc.n, n = Lf.n;
        const int64_t ne = (int64_t)Lc.E * (nc - 2);
        for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < ne + Lc.V; t += (int64_t)gl * NT) {
            if (t < ne) {
                const int e = (int)(t / (nc - 2)), K = (int)(t % (nc - 2)) + 1;
                const int64_t mc = edge_main(Lc, e);
                const EdgeInfo& ei = Lf.edges[e];
                // formed before the Dirichlet test (all reads stay inside the
                // edge block), so the loads go out with the edge's metadata
                const int64_t g0 = edge_ghost(Lf, e, 0), g1 = edge_ghost(Lf, e, 1);
                const int k = 2 * K;
                const T rm = edge_resid<T>(op, Lf, ei, e, x, f, kap, k - 1);
                const T rk = edge_resid<T>(op, Lf, ei, e, x, f, kap, k);
                const T rp = edge_resid<T>(op, Lf, ei, e, x, f, kap, k + 1);
                const T nb = rm + rp + r[g0 + k - 1] + r[g0 + k] + r[g1 + k - 1] + r[g1 + k];
                fc[mc + K] = ei.boundary ? (T)0 : rk + (T)0.5 * nb;
            } else {
                const int v = (int)(t - ne);
                const VertexInfo& vi = Lf.verts[v];
                const int64_t vc = vert_off(Lc, v);
                const int2 db = *reinterpret_cast<const int2*>(&vi.deg);   // deg, boundary in one load
                if (db.y) {
                    fc[vc] = (T)0;
                    continue;
                }
                const int64_t vf = vert_off(Lf, v);
                const int deg = db.x;
                const T rv = vertex_resid<T>(op, Lf, vi, deg, x, f, kap, vf);
                T nb = (T)0;
                for (int q0 = 0; q0 < deg; q0 += 4) {     // ring members four at a time, summed in order
                    // formed without a branch (an edge block always has both
                    // ghost rows, so the reads stay inside it), then masked:
                    // the four members' loads are in flight together
                    T rq[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int q = q0 + j < deg ? q0 + j : q0, e2 = vi.edge[q];
                        const EdgeInfo& e2i = Lf.edges[e2];
                        const T rr = edge_resid<T>(op, Lf, e2i, e2, x, f, kap, vi.at_a[q] ? 1 : n - 2);
                        rq[j] = e2i.boundary ? (T)0 : rr;
                    }
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (q0 + j < deg) nb += rq[j];
                }
                fc[vc] = rv + (T)0.5 * nb;
            }
        }
    } else {
        for (int64_t t = (int64_t)(blockIdx.x - gl) * NT + threadIdx.x; t < uc_n;
             t += (int64_t)(gridDim.x - gl) * NT)
            uc[t] = (T)0;
    }
}

// u += P uc.  A fine point coincides with a coarse point or is the midpoint
// of a coarse micro-edge.  Every holder of a copy updates it from its own
// coarse copies (same operands, so the copies stay identical): faces their
// whole triangle except Dirichlet points, pushing near-edge rows; edges
// their points and end slots; vertices their value and ghost copies (the
// ring copies of Dirichlet vertices too).
template <class T>
__global__ __launch_bounds__(NT) void k_prolong(LevelDev Lf, LevelDev Lc, const T* __restrict__ uc,
                                                T* __restrict__ u, int gf) {
    if ((int)blockIdx.x < gf) {
        FACE_ALL_LOOP(Lf, gf)
        (void)interior;
        T v = u[p];
        if (!face_dirichlet(fi, n, i, j)) {
            v += prol_face<T>(uc, face_base(Lc, face), Lc.n, i, j);
            u[p] = v;
        }
        push_face_near(Lf, u, fi, i, j, v);
        }
    } else {
        const int n = Lf.n;
        const int64_t ne = (int64_t)Lf.n_iedges * (n - 2);
        for (int64_t t = (int64_t)(blockIdx.x - gf) * NT + threadIdx.x; t < ne + Lf.V;
             t += (int64_t)(gridDim.x - gf) * NT) {
            if (t < ne) {
                const int e = Lf.iedges[t / (n - 2)], k = (int)(t % (n - 2)) + 1;
                const EdgeInfo& ei = Lf.edges[e];
                const int64_t m = edge_main(Lf, e), mc = edge_main(Lc, e);
                const T c = (k & 1) ? (T)0.5 * (uc[mc + (k >> 1)] + uc[mc + (k >> 1) + 1]) : uc[mc + (k >> 1)];
                u[m + k] += c;
                if (k == 1 && !Lf.verts[ei.a].boundary) u[m] += uc[mc];
                if (k == n - 2 && !Lf.verts[ei.b].boundary) u[m + n - 1] += uc[mc + Lc.n - 1];
            } else {
                // every vertex: an interior one updates its value and ring; a
                // Dirichlet one keeps its value but updates the ring copies of
                // the first points of its interior edges, which the edge
                // blocks update (same operands, so the copies stay identical)
                const int v = (int)(t - ne);
                const VertexInfo& vi = Lf.verts[v];
                const int64_t vf = vert_off(Lf, v), vc = vert_off(Lc, v);
                const T cv = uc[vc];
                if (!vi.boundary) u[vf] += cv;
                for (int q = 0; q < vi.deg; ++q)
                    if (!vi.boundary || !Lf.edges[vi.edge[q]].boundary) u[vf + 1 + q] += (T)0.5 * (cv + uc[vc + 1 + q]);
            }
        }
    }
}

// Canonical <-> layout.  to_canon = 0: field[owner] = canon; 1: reverse.
template <class T>
__global__ __launch_bounds__(NT) void k_face_canon(LevelDev L, const T* __restrict__ src,
                                                   T* __restrict__ dst, int to_canon) {
    FACE_TILE_LOOP(L, gridDim.x)
    (void)fi; (void)up; (void)dn;
    const int64_t nfi = (int64_t)(n - 2) * (n - 3) / 2;
    const int64_t before = (int64_t)(j - 1) * (n - 2) - (int64_t)(j - 1) * j / 2;
    const int64_t c = L.can_face_base + (int64_t)face * nfi + before + (i - 1);
    if (to_canon) dst[c] = src[p]; else dst[p] = src[c];
    FACE_TILE_END
}

template <class T>
__global__ __launch_bounds__(NT) void k_low_canon(LevelDev L, const T* __restrict__ src,
                                                  T* __restrict__ dst, int to_canon) {
    const int n = L.n;
    const int64_t ne = (int64_t)L.E * (n - 2);
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < ne + L.V; t += (int64_t)gridDim.x * NT) {
        int64_t p, c;
        if (t < ne) {
            const int e = (int)(t / (n - 2)), k = (int)(t % (n - 2)) + 1;
            p = edge_main(L, e) + k;
            c = L.can_edge_base + t;
        } else {
            const int v = (int)(t - ne);
            p = vert_off(L, v);
            c = v;
        }
        if (to_canon) dst[c] = src[p]; else dst[p] = src[c];
    }
}

// Injection of owned values: coarse point = coincident fine point.
template <class T>
__global__ __launch_bounds__(NT) void k_face_inject(LevelDev Lf, LevelDev Lc, const T* __restrict__ kf,
                                                    T* __restrict__ kc) {
    FACE_TILE_LOOP(Lc, gridDim.x)
    (void)fi; (void)up; (void)dn;
    kc[p] = kf[face_base(Lf, face) + row_start(Lf.n, 2 * j) + 2 * i];
    FACE_TILE_END
}

template <class T>
__global__ __launch_bounds__(NT) void k_low_inject(LevelDev Lf, LevelDev Lc, const T* __restrict__ kf,
                                                   T* __restrict__ kc) {
    const int nc = Lc.n;
    const int64_t ne = (int64_t)Lc.E * (nc - 2);
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < ne + Lc.V; t += (int64_t)gridDim.x * NT) {
        if (t < ne) {
            const int e = (int)(t / (nc - 2)), K = (int)(t % (nc - 2)) + 1;
            kc[edge_main(Lc, e) + K] = kf[edge_main(Lf, e) + 2 * K];
        } else {
            const int v = (int)(t - ne);
            kc[vert_off(Lc, v)] = kf[vert_off(Lf, v)];
        }
    }
}

// ELL values of the coarse operator, in the order [centre, neighbours...]
// used by the host-built column table.
__global__ __launch_bounds__(NT) void k_coarse_extract(LevelDev L, CoarseDev C, int op,
                                                       const double* __restrict__ kap,
                                                       double* __restrict__ vals) {
    const int n = L.n;
    for (int p = blockIdx.x * NT + threadIdx.x; p < C.N; p += gridDim.x * NT) {
        double* v = vals + (int64_t)p * C.W;
        for (int w = 0; w < C.W; ++w) v[w] = 0.0;
        const int kind = C.kind[p], prim = C.prim[p];
        if (kind == 2) {
            const int i = C.pa[p], j = C.pb[p];
            const int64_t q = face_base(L, prim) + row_start(n, j) + i;
            const int64_t up = row_start(n, j + 1) - row_start(n, j), dn = row_start(n, j) - row_start(n, j - 1);
            const W7<double> w = face_weights<double>(op, L.faces[prim], L.inv4l, kap, q, up, dn);
            v[0] = w.c; v[1] = w.e; v[2] = w.w; v[3] = w.n; v[4] = w.s; v[5] = w.se; v[6] = w.nw;
        } else if (kind == 1) {
            const int k = C.pa[p];
            const int64_t m = edge_main(L, prim), g0 = edge_ghost(L, prim, 0), g1 = edge_ghost(L, prim, 1);
            const WE<double> w = edge_weights<double>(op, L.edges[prim], L.inv4l, kap, m, g0, g1, k);
            v[0] = w.c; v[1] = w.al; v[2] = w.ah; v[3] = w.l0; v[4] = w.h0; v[5] = w.l1; v[6] = w.h1;
        } else {
            const VertexInfo& vi = L.verts[prim];
            const int64_t vb = vert_off(L, prim);
            double c = 0.0;
            for (int q = 0; q < vi.deg; ++q) {
                const double wq = vertex_weight<double>(op, vi, L.inv4l, kap, vb, q);
                v[1 + q] = wq;
                c += wq;
            }
            v[0] = (op == OP_MASS) ? c : -c;
        }
        (void)n;
    }
}

// Jacobi-preconditioned CG from zero on the coarse interior system (one
// workgroup); b is read from the residual field, u[owner] += x at the end.
template <class T>
__global__ __launch_bounds__(1024) void k_coarse_pcg(CoarseDev C, const double* __restrict__ vals,
                                                     const T* __restrict__ rf, T* __restrict__ uf,
                                                     double tol, int maxit) {
    __shared__ double sm[1024 / 64 + 1];
    const int N = C.N, W = C.W, tid = threadIdx.x;
    double* x = C.vec;
    double* r = x + N;
    double* z = r + N;
    double* p = z + N;
    double* q = p + N;
    double bb = 0.0;
    for (int a = tid; a < N; a += 1024) {
        const double b = (double)rf[C.owner[a]];
        x[a] = 0.0;
        r[a] = b;
        bb += b * b;
    }
    bb = block_sum<1024>(bb, sm);
    const double bn = sqrt(bb);
    if (bn == 0.0) return;
    double rz = 0.0;
    for (int a = tid; a < N; a += 1024) {
        z[a] = r[a] / vals[(int64_t)a * W];
        p[a] = z[a];
        rz += r[a] * z[a];
    }
    rz = block_sum<1024>(rz, sm);
    for (int it = 0; it < maxit; ++it) {
        double pq = 0.0;
        for (int a = tid; a < N; a += 1024) {
            double s = 0.0;
            for (int w = 0; w < W; ++w) {
                const int c = C.cols[(int64_t)a * W + w];
                if (c >= 0) s += vals[(int64_t)a * W + w] * p[c];
            }
            q[a] = s;
            pq += p[a] * s;
        }
        pq = block_sum<1024>(pq, sm);
        const double alpha = rz / pq;
        double rr = 0.0;
        for (int a = tid; a < N; a += 1024) {
            x[a] += alpha * p[a];
            r[a] -= alpha * q[a];
            rr += r[a] * r[a];
        }
        rr = block_sum<1024>(rr, sm);
        if (sqrt(rr) <= tol * bn) break;
        double rzn = 0.0;
        for (int a = tid; a < N; a += 1024) {
            z[a] = r[a] / vals[(int64_t)a * W];
            rzn += r[a] * z[a];
        }
        rzn = block_sum<1024>(rzn, sm);
        const double beta = rzn / rz;
        rz = rzn;
        for (int a = tid; a < N; a += 1024) p[a] = z[a] + beta * p[a];
        __syncthreads();
    }
    __syncthreads();
    for (int a = tid; a < N; a += 1024) uf[C.owner[a]] += (T)x[a];
}

// Block sum of two values at once (same fixed tree as block_sum).
template <int NTH>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* sm) {
    a = wave_sum(a);
    b = wave_sum(b);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const unsigned nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) { sm[w] = a; sm[NTH / 64 + w] = b; }
    __syncthreads();
    if (threadIdx.x < 64) {
        double ta = (threadIdx.x < nw) ? sm[threadIdx.x] : 0.0;
        double tb = (threadIdx.x < nw) ? sm[NTH / 64 + threadIdx.x] : 0.0;
        ta = wave_sum(ta);
        tb = wave_sum(tb);
        if (threadIdx.x == 0) { sm[2 * (NTH / 64)] = ta; sm[2 * (NTH / 64) + 1] = tb; }
    }
    __syncthreads();
    a = sm[2 * (NTH / 64)];
    b = sm[2 * (NTH / 64) + 1];
}

// Register-resident Jacobi-PCG for coarse systems with N <= CG_RPT * 1024
// rows and at most CG_W stencil entries per row.  Each thread owns rows
// tid + k * blockDim.x; only the search direction is shared (LDS).  Same
// recurrences and stopping rule as k_coarse_pcg.  rhs(a) gives b[a]; out(a,
// x) receives the solution row by row (not called when b = 0).
constexpr int CG_RPT = 2;
constexpr int CG_W = 8;
constexpr int CG_MAXN = CG_RPT * 1024;
static_assert(CG_MAXN == COARSE_DENSE_MAXN, "coarse inverse size bound");

template <class Rhs, class Out>
__device__ __forceinline__ void pcg_reg_core(const CoarseDev& C, const double* __restrict__ vals, Rhs rhs,
                                             Out out, double tol, int maxit, double* ps, double* sm) {
    const int N = C.N, W = C.W, nt = blockDim.x, tid = threadIdx.x;
    double x[CG_RPT], r[CG_RPT], z[CG_RPT], p[CG_RPT], dinv[CG_RPT], av[CG_RPT][CG_W];
    int ac[CG_RPT][CG_W];
    double bb = 0.0;
#pragma unroll
    for (int k = 0; k < CG_RPT; ++k) {
        const int a = tid + k * nt;
        const bool own = a < N;
        x[k] = 0.0;
        r[k] = own ? rhs(a) : 0.0;
        dinv[k] = own ? 1.0 / vals[(int64_t)a * W] : 0.0;
#pragma unroll
        for (int w = 0; w < CG_W; ++w) {
            const bool in = own && w < W;
            ac[k][w] = in ? C.cols[(int64_t)a * W + w] : -1;
            av[k][w] = in ? vals[(int64_t)a * W + w] : 0.0;
        }
        bb += r[k] * r[k];
    }
    double rz = 0.0;
#pragma unroll
    for (int k = 0; k < CG_RPT; ++k) {
        z[k] = dinv[k] * r[k];
        p[k] = z[k];
        rz += r[k] * z[k];
    }
    block_sum2<1024>(bb, rz, sm);
    const double bn = sqrt(bb);
    if (bn == 0.0) return;
    for (int it = 0; it < maxit; ++it) {
#pragma unroll
        for (int k = 0; k < CG_RPT; ++k)
            if (tid + k * nt < N) ps[tid + k * nt] = p[k];
        __syncthreads();
        double q[CG_RPT], pq = 0.0, dummy = 0.0;
#pragma unroll
        for (int k = 0; k < CG_RPT; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < CG_W; ++w)
                if (ac[k][w] >= 0) s += av[k][w] * ps[ac[k][w]];
            q[k] = s;
            pq += p[k] * s;
        }
        block_sum2<1024>(pq, dummy, sm);
        const double alpha = rz / pq;
        double rr = 0.0, rzn = 0.0;
#pragma unroll
        for (int k = 0; k < CG_RPT; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
            z[k] = dinv[k] * r[k];
            rr += r[k] * r[k];
            rzn += r[k] * z[k];
        }
        block_sum2<1024>(rr, rzn, sm);
        if (sqrt(rr) <= tol * bn) break;
        const double beta = rzn / rz;
        rz = rzn;
#pragma unroll
        for (int k = 0; k < CG_RPT; ++k) p[k] = z[k] + beta * p[k];
    }
#pragma unroll
    for (int k = 0; k < CG_RPT; ++k) {
        const int a = tid + k * nt;
        if (a < N) out(a, x[k]);
    }
}

template <class T>
__global__ __launch_bounds__(1024) void k_coarse_pcg_reg(CoarseDev C, const double* __restrict__ vals,
                                                         const T* __restrict__ rf, T* __restrict__ uf,
                                                         double tol, int maxit) {
    __shared__ double ps[CG_MAXN];
    __shared__ double sm[2 * (1024 / 64) + 2];
    pcg_reg_core(C, vals, [&](int a) { return (double)rf[C.owner[a]]; },
                 [&](int a, double x) { uf[C.owner[a]] += (T)x; }, tol, maxit, ps, sm);
}

// Row j of the coarse inverse (block j): PCG on A x = e_j; inv[j N + a] =
// x[a] = (A^-1)[a][j].
__global__ __launch_bounds__(1024) void k_coarse_inverse(CoarseDev C, const double* __restrict__ vals,
                                                         double* __restrict__ inv, double tol, int maxit) {
    __shared__ double ps[CG_MAXN];
    __shared__ double sm[2 * (1024 / 64) + 2];
    const int j = blockIdx.x;
    double* row = inv + (int64_t)j * C.N;
    pcg_reg_core(C, vals, [&](int a) { return a == j ? 1.0 : 0.0; },
                 [&](int a, double x) { row[a] = x; }, tol, maxit, ps, sm);
}

// Direct coarse solve with the stored inverse, in two launches: x = A^-1 b,
// then one refinement step x += A^-1 (b - A x) and u[owner] += x, with b
// read from the residual field.  The refinement makes the result exact to
// rounding although the inverse comes from an iterative solve.  One wave
// per row: it reads the row of the (symmetric) inverse coalesced, multiplies
// with the vector held in LDS and reduces in a fixed order.
constexpr int CD_NT = 256;

__device__ __forceinline__ double coarse_row_dot(const double* __restrict__ row, const double* v, int N) {
    // four independent partial sums keep four loads per lane in flight
    const int l = threadIdx.x & 63;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int j = l;
    for (; j + 192 < N; j += 256) {
        s0 += row[j] * v[j];
        s1 += row[j + 64] * v[j + 64];
        s2 += row[j + 128] * v[j + 128];
        s3 += row[j + 192] * v[j + 192];
    }
    for (; j < N; j += 64) s0 += row[j] * v[j];
    return wave_sum((s0 + s1) + (s2 + s3));
}

template <class T>
__global__ __launch_bounds__(CD_NT) void k_coarse_dense1(CoarseDev C, const double* __restrict__ inv,
                                                         const T* __restrict__ rf, double* __restrict__ xbuf) {
    __shared__ double bs[CG_MAXN];
    const int N = C.N;
    for (int a = threadIdx.x; a < N; a += CD_NT) bs[a] = (double)rf[C.owner[a]];
    __syncthreads();
    const int nw = gridDim.x * (CD_NT / 64);
    for (int a = blockIdx.x * (CD_NT / 64) + (threadIdx.x >> 6); a < N; a += nw) {
        const double s = coarse_row_dot(inv + (int64_t)a * N, bs, N);
        if ((threadIdx.x & 63) == 0) xbuf[a] = s;
    }
}

template <class T>
__global__ __launch_bounds__(CD_NT) void k_coarse_dense2(CoarseDev C, const double* __restrict__ vals,
                                                         const double* __restrict__ inv,
                                                         const T* __restrict__ rf,
                                                         const double* __restrict__ xbuf, T* __restrict__ uf) {
    __shared__ double rs[CG_MAXN];
    const int N = C.N, W = C.W;
    for (int a = threadIdx.x; a < N; a += CD_NT) {
        double s = (double)rf[C.owner[a]];
        for (int w = 0; w < W; ++w) {
            const int c = C.cols[(int64_t)a * W + w];
            if (c >= 0) s -= vals[(int64_t)a * W + w] * xbuf[c];
        }
        rs[a] = s;
    }
    __syncthreads();
    const int nw = gridDim.x * (CD_NT / 64);
    for (int a = blockIdx.x * (CD_NT / 64) + (threadIdx.x >> 6); a < N; a += nw) {
        const double s = coarse_row_dot(inv + (int64_t)a * N, rs, N);
        if ((threadIdx.x & 63) == 0) uf[C.owner[a]] += (T)(xbuf[a] + s);
    }
}

__global__ __launch_bounds__(NT) void k_f64_to_f32(const double* __restrict__ s, float* __restrict__ d,
                                                   int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        d[t] = (float)s[t];
}

__global__ __launch_bounds__(NT) void k_f32_to_f64(const float* __restrict__ s, double* __restrict__ d,
                                                   int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        d[t] = (double)s[t];
}

__global__ __launch_bounds__(NT) void k_add_f32_to_f64(double* __restrict__ u, const float* __restrict__ e,
                                                       int64_t n) {
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        u[t] += (double)e[t];
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int64_t items, int cap) {
    int64_t g = (items + NT - 1) / NT;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}
static inline int face_grid(const LevelDev& L) {
    int64_t g = (int64_t)L.F * L.ntiles;
    if (g < 1) g = 1;
    return (int)(g > MAX_FACE_BLOCKS ? MAX_FACE_BLOCKS : g);
}
static inline int64_t low_items(const LevelDev& L) { return (int64_t)L.E * (L.n - 2) + L.V; }

template <class T>
static const T* kap_of(const hhg_mesh* M, int level);
template <>
const double* kap_of<double>(const hhg_mesh* M, int level) { return M->kap64[level]; }
template <>
const float* kap_of<float>(const hhg_mesh* M, int level) { return M->kap32[level]; }

hipError_t launch_sync(const hhg_mesh* M, int level, int dtype, void* x, int mask, hipStream_t s) {
    const LevelDev L = M->dev(level);
    // classes are stored contiguously in the order VERT, EEVEN, EODD, FACE
    int c = 0;
    while (c < G_NCLS) {
        if (!(mask & (1 << c))) { ++c; continue; }
        int c2 = c;
        while (c2 < G_NCLS && (mask & (1 << c2))) ++c2;
        const int64_t lo = L.gcls[c], hi = L.gcls[c2];
        if (hi > lo) {
            const int g = grid_for(hi - lo, 4096);
            if (dtype == DT_F64)
                k_sync<double><<<g, NT, 0, s>>>((double*)x, L.gdst, L.gsrc, lo, hi);
            else
                k_sync<float><<<g, NT, 0, s>>>((float*)x, L.gdst, L.gsrc, lo, hi);
        }
        c = c2;
    }
    return hipGetLastError();
}

// Grid of the tiled point operator: tile blocks (a multiple of 8, for the
// XCD-contiguous order) followed by edge/vertex blocks.
struct TiledGrid {
    int tiles, gt, gl;
};
static inline TiledGrid tiled_grid(int64_t F, int64_t ntl, int64_t low) {
    TiledGrid g;
    g.tiles = (int)(F * ntl);
    g.gt = (g.tiles + 7) / 8 * 8;
    int64_t gl = (low + GS_NT - 1) / GS_NT;
    g.gl = (int)std::max<int64_t>(1, std::min<int64_t>(gl, MAX_LOW_BLOCKS / 2));
    return g;
}

// Point operator (k_apply_low's modes) over a whole level; returns the number of
// partial sums written (norm modes with partials).
template <class T, int MODE>
static int apply_tiled(const hhg_mesh* M, int level, int op, const T* x, const T* f, T* y,
                       double* partials, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const T* kap = kap_of<T>(M, level);
    const bool vk = op == OP_DIFFUSION;
    const int tl = vk && sizeof(T) == 8 ? 1 : 0;
    const TiledGrid g = tiled_grid(L.F, L.n_gs_tl[0][tl], low_items(L));
    const int grid = g.gt + g.gl;
    if (vk && sizeof(T) == 8)
        k_apply_tiled<T, true, MODE, GS_TJ16><<<grid, GS_NT, 0, s>>>(L, op, x, f, y, kap, g.tiles, g.gt, partials);
    else if (vk)
        k_apply_tiled<T, true, MODE, GS_TJ><<<grid, GS_NT, 0, s>>>(L, op, x, f, y, kap, g.tiles, g.gt, partials);
    else
        k_apply_tiled<T, false, MODE, GS_TJ><<<grid, GS_NT, 0, s>>>(L, op, x, f, y, kap, g.tiles, g.gt, partials);
    return grid;
}

template <class T>
static hipError_t apply_t(const hhg_mesh* M, int level, int op, const T* x, T* y, hipStream_t s) {
    apply_tiled<T, 0>(M, level, op, x, nullptr, y, nullptr, s);
    return hipGetLastError();
}

hipError_t launch_apply(const hhg_mesh* M, int level, int op, int dtype, const void* x, void* y,
                        hipStream_t s) {
    if (dtype == DT_F64) return apply_t<double>(M, level, op, (const double*)x, (double*)y, s);
    return apply_t<float>(M, level, op, (const float*)x, (float*)y, s);
}

template <class T>
static hipError_t residual_t(const hhg_mesh* M, int level, int op, const T* u, const T* f, T* r,
                             double* norm, hipStream_t s) {
    const int np = r ? apply_tiled<T, 1>(M, level, op, u, f, r, norm ? M->partials : nullptr, s)
                     : apply_tiled<T, 4>(M, level, op, u, f, r, M->partials, s);
    if (norm) k_reduce_final<<<1, 1024, 0, s>>>(M->partials, np, norm, 1);
    return hipGetLastError();
}

hipError_t launch_mp_step(const hhg_mesh* M, int level, int op, const double* x, const float* e,
                          const double* f, double* xo, float* r, double* norm, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const bool vk = op == OP_DIFFUSION;
    const TiledGrid g = tiled_grid(L.F, L.n_gs_tl[0][vk ? 1 : 0], low_items(L));
    const int grid = g.gt + g.gl;
    const double* kap = M->kap64[level];
#define HHG_MP_LAUNCH(UP)                                                                              \
    do {                                                                                               \
        if (vk)                                                                                        \
            k_mp_step_tiled<UP, true, GS_TJ16><<<grid, GS_NT, 0, s>>>(L, op, x, e, f, xo, r, kap, g.tiles, \
                                                                     g.gt, M->partials);               \
        else                                                                                           \
            k_mp_step_tiled<UP, false, GS_TJ><<<grid, GS_NT, 0, s>>>(L, op, x, e, f, xo, r, kap, g.tiles, \
                                                                     g.gt, M->partials);               \
    } while (0)
    if (e) HHG_MP_LAUNCH(true);
    else HHG_MP_LAUNCH(false);
#undef HHG_MP_LAUNCH
    k_reduce_final<<<1, 1024, 0, s>>>(M->partials, grid, norm, 1);
    return hipGetLastError();
}

hipError_t launch_residual(const hhg_mesh* M, int level, int op, int dtype, const void* u,
                           const void* f, void* r, double* norm, hipStream_t s) {
    if (dtype == DT_F64)
        return residual_t<double>(M, level, op, (const double*)u, (const double*)f, (double*)r, norm, s);
    return residual_t<float>(M, level, op, (const float*)u, (const float*)f, (float*)r, norm, s);
}

struct TimingScope {
    const hhg_mesh* M;
    hipStream_t s;
    bool on;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TimingScope(const hhg_mesh* m, hipStream_t st, bool enable) : M(m), s(st), on(enable) {
        if (!on) return;
        hhg_mesh* mm = const_cast<hhg_mesh*>(M);
        size_t idx = (size_t)mm->t_launches;
        if (idx >= mm->t_events.size()) {
            hipEvent_t a, b;
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            mm->t_events.emplace_back((void*)a, (void*)b);
        }
        e0 = (hipEvent_t)mm->t_events[idx].first;
        e1 = (hipEvent_t)mm->t_events[idx].second;
        (void)hipEventRecord(e0, s);
    }
    ~TimingScope() {
        if (!on) return;
        (void)hipEventRecord(e1, s);
        const_cast<hhg_mesh*>(M)->t_launches++;
    }
};

template <class T>
static hipError_t gs_t(const hhg_mesh* M, int level, int op, T* x, T* y, const T* f, int backward,
                       hipStream_t s, const T* uc = nullptr, T* rout = nullptr, double* norm = nullptr,
                       T* fcout = nullptr) {
    const LevelDev L = M->dev(level);
    const T* kap = kap_of<T>(M, level);
    const int gl = grid_for((int64_t)L.E * (L.n - 2) + L.V, MAX_LOW_BLOCKS);
    // 0: sweep; 1: forward sweep that also writes the residual; 2: backward
    // sweep that also forms the residual norm; 3: forward sweep that also
    // restricts the residual of the face points (three-colour faces only)
    const int res = fcout ? 3 : (rout ? 1 : (norm ? 2 : 0));
    const bool has2 = M->m.nfaces2 > 0;
    if (res == 3 && (has2 || !rout)) return hipErrorInvalidValue;
    const bool timed = M->timing && level == M->m.L && !uc && res == 0;
    const LevelDev Lc = (uc || fcout) ? M->dev(level - 1) : L;
    // the variable-coefficient FP64 tile (u and k in LDS) is 16 rows high so
    // that two blocks fit on a CU; the others are 24 rows high
    const bool t16 = op == OP_DIFFUSION && sizeof(T) == 8;
    const int ntile_blocks = L.F * L.n_gs_tl[gs_list(res)][t16 ? 1 : 0];
    const int g = (ntile_blocks + GS_COPY_BLOCKS + 7) / 8 * 8;
    const int g2 = has2 ? (ntile_blocks + 7) / 8 * 8 : 0;
    const int64_t nrim = (int64_t)L.F * (L.n >= 5 ? 3 * (int64_t)L.n - 12 : 0) + low_items(L);
    const int grim = grid_for(nrim, MAX_LOW_BLOCKS);
    double* part = M->partials;
    if (res == 2 && (int64_t)g + g2 + grim > M->n_partials) return hipErrorInvalidValue;
    auto faces = [&]() -> hipError_t {
        TimingScope ts(M, s, timed);
#define HHG_FACE_LAUNCH(VK, PR, TJ, RS)                                                             \
    do {                                                                                            \
        k_face_gs_fused<T, VK, 3, PR, TJ, RS><<<g, GS_NT, 0, s>>>(L, x, y, f, kap, backward,         \
                                                                  ntile_blocks, 1, Lc, uc, rout, part, \
                                                                  nullptr);                          \
        if (has2)                                                                                   \
            k_face_gs_fused<T, VK, 2, PR, TJ, RS><<<g2, GS_NT, 0, s>>>(L, x, y, f, kap, backward,    \
                                                                       ntile_blocks, 0, Lc, uc, rout, \
                                                                       part + g, nullptr);           \
    } while (0)
#define HHG_FACE_LAUNCH_R(VK, TJ)                                                                   \
    k_face_gs_fused<T, VK, 3, false, TJ, 3><<<g, GS_NT, 0, s>>>(L, x, y, f, kap, backward, ntile_blocks, 1, \
                                                               Lc, uc, rout, part, fcout)
        if constexpr (GS_STREAM && sizeof(T) == 4) if (res == 0 && !uc && L.F * L.n_gs_tl[0][0] >= GS_STREAM_MIN) {
            // plain FP32 sweep of a large level: streamed kernel on the
            // three-colour faces, tiles on the faces with a right angle (in
            // FP64 the rows take twice the registers and the tile sweep is
            // faster; on smaller levels a wave's chain of row steps is
            // longer than a tile's load-stage-store)
            const int ntask = L.F * L.n_gs_tl[0][0];
            const int nb = (int)pad_up((ntask + GS_SNT / 64 - 1) / (GS_SNT / 64), 8);
            const int gsb = nb + GS_COPY_BLOCKS;
#define HHG_STREAM_LAUNCH(VK)                                                                       \
    do {                                                                                            \
        if (backward) k_face_gs_stream<T, VK, true, GS_NU><<<gsb, GS_SNT, 0, s>>>(L, x, y, f, kap, nb);  \
        else k_face_gs_stream<T, VK, false, GS_NU><<<gsb, GS_SNT, 0, s>>>(L, x, y, f, kap, nb);          \
        if (has2)                                                                                   \
            k_face_gs_fused<T, VK, 2, false, (VK && sizeof(T) == 8) ? GS_TJ16 : GS_TJ, 0>             \
                <<<g2, GS_NT, 0, s>>>(L, x, y, f, kap, backward, ntile_blocks, 0, Lc, uc, rout, part, nullptr); \
    } while (0)
            if (op == OP_DIFFUSION) HHG_STREAM_LAUNCH(true);
            else HHG_STREAM_LAUNCH(false);
#undef HHG_STREAM_LAUNCH
            return hipGetLastError();
        }
        if (op == OP_DIFFUSION) {
            constexpr int TJV = sizeof(T) == 8 ? GS_TJ16 : GS_TJ;
            if (uc) HHG_FACE_LAUNCH(true, true, TJV, 0);
            else if (res == 3) HHG_FACE_LAUNCH_R(true, sizeof(T) == 8 ? GS_TJ16 : GS_TJR);
            else if (res == 1) HHG_FACE_LAUNCH(true, false, TJV, 1);
            else if (res == 2) HHG_FACE_LAUNCH(true, false, TJV, 2);
            else HHG_FACE_LAUNCH(true, false, TJV, 0);
        } else {
            if (uc) HHG_FACE_LAUNCH(false, true, GS_TJ, 0);
            else if (res == 3) HHG_FACE_LAUNCH_R(false, GS_TJR);
            else if (res == 1) HHG_FACE_LAUNCH(false, false, GS_TJ, 1);
            else if (res == 2) HHG_FACE_LAUNCH(false, false, GS_TJ, 2);
            else HHG_FACE_LAUNCH(false, false, GS_TJ, 0);
        }
#undef HHG_FACE_LAUNCH
#undef HHG_FACE_LAUNCH_R
        return hipGetLastError();
    };
    hipError_t e;
    if (!backward) {
        k_low_gs<T><<<gl, NT, 0, s>>>(L, op, x, f, kap, 0);
        k_low_gs<T><<<gl, NT, 0, s>>>(L, op, x, f, kap, 1);
        if ((e = faces()) != hipSuccess || res != 1) return e;
        // residual of the edge and vertex points (all copies) from the swept y
        k_apply_low<T, 1><<<grid_for(low_items(L), MAX_LOW_BLOCKS), NT, 0, s>>>(L, op, y, f, rout, kap, nullptr);
        return hipGetLastError();
    }
    if ((e = faces()) != hipSuccess) return e;
    k_low_gs<T><<<gl, NT, 0, s>>>(L, op, y, f, kap, 1);
    k_low_gs<T><<<gl, NT, 0, s>>>(L, op, y, f, kap, 0);
    if (res == 2) {
        // the rest of the residual norm, now that the edge stages are done
        k_resnorm_rim<T><<<grim, NT, 0, s>>>(L, op, y, f, kap, part + g + g2);
        k_reduce_final<<<1, 1024, 0, s>>>(part, g + g2 + grim, norm, 1);
    }
    return hipGetLastError();
}

int64_t face_loop_partials(const hhg_mesh* M, int level) {
    const LevelHost& H = M->m.lv[level];
    int64_t g = (int64_t)M->m.F * (int64_t)H.tiles.size();
    g = std::max<int64_t>(1, std::min<int64_t>(g, MAX_FACE_BLOCKS));
    const int n = H.n;
    const int64_t low = (int64_t)M->m.E * (n - 2) + M->m.V;
    int64_t most = g + grid_for(low, MAX_LOW_BLOCKS);
    for (int t = 0; t < 2; ++t) {
        const TiledGrid tg = tiled_grid(M->m.F, (int64_t)H.gs_tl[0][t].size(), low);
        most = std::max<int64_t>(most, (int64_t)tg.gt + tg.gl);
    }
    return most;
}

int64_t sweep_norm_partials(const hhg_mesh* M, int level) {
    const LevelHost& H = M->m.lv[level];
    const int n = H.n;
    const int64_t nrim = (int64_t)M->m.F * (n >= 5 ? 3 * (int64_t)n - 12 : 0) + (int64_t)M->m.E * (n - 2) + M->m.V;
    int64_t most = 0;
    for (int t = 0; t < 2; ++t) {
        const int64_t tiles = (int64_t)M->m.F * (int64_t)H.gs_tl[1][t].size();
        const int64_t g = (tiles + GS_COPY_BLOCKS + 7) / 8 * 8;
        const int64_t g2 = M->m.nfaces2 > 0 ? (tiles + 7) / 8 * 8 : 0;
        most = std::max(most, g + g2 + grid_for(nrim, MAX_LOW_BLOCKS));
    }
    return most;
}

hipError_t launch_gs_sweep(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                           const void* f, int backward, hipStream_t s) {
    if (dtype == DT_F64)
        return gs_t<double>(M, level, op, (double*)x, (double*)y, (const double*)f, backward, s);
    return gs_t<float>(M, level, op, (float*)x, (float*)y, (const float*)f, backward, s);
}

hipError_t launch_gs_sweep_norm(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                const void* f, double* norm, hipStream_t s) {
    if (dtype == DT_F64)
        return gs_t<double>(M, level, op, (double*)x, (double*)y, (const double*)f, 1, s, nullptr, nullptr, norm);
    return gs_t<float>(M, level, op, (float*)x, (float*)y, (const float*)f, 1, s, nullptr, nullptr, norm);
}

hipError_t launch_gs_sweep_prolong(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                   const void* f, const void* uc, hipStream_t s) {
    if (dtype == DT_F64)
        return gs_t<double>(M, level, op, (double*)x, (double*)y, (const double*)f, 1, s, (const double*)uc);
    return gs_t<float>(M, level, op, (float*)x, (float*)y, (const float*)f, 1, s, (const float*)uc);
}

template <class T>
static hipError_t restrict_t(const hhg_mesh* M, int level, const T* r, T* fc, T* uc, hipStream_t s) {
    const LevelDev Lf = M->dev(level), Lc = M->dev(level - 1);
    const int gf = face_grid(Lc), gl = gf + grid_for(low_items(Lc), MAX_LOW_BLOCKS);
    const int gz = uc ? grid_for(Lc.total, 2048) : 0;
    k_restrict<T><<<gl + gz, NT, 0, s>>>(Lf, Lc, r, fc, uc, Lc.total, gf, gl);
    return hipGetLastError();
}

hipError_t launch_restrict(const hhg_mesh* M, int level, int dtype, const void* r, void* fc, void* uc,
                           hipStream_t s) {
    if (dtype == DT_F64) return restrict_t<double>(M, level, (const double*)r, (double*)fc, (double*)uc, s);
    return restrict_t<float>(M, level, (const float*)r, (float*)fc, (float*)uc, s);
}

// The last pre-smoothing sweep with the restriction of its residual: on
// meshes of three-colour faces the coarse face points are restricted inside
// the sweep and the coarse edge and vertex points by k_restrict_low; with
// two-colour faces the residual is stored whole and restricted after.
template <class T>
static hipError_t gs_restrict_t(const hhg_mesh* M, int level, int op, T* x, T* y, const T* f, T* r, T* fc,
                                T* uc, hipStream_t s) {
    const bool fused = M->m.nfaces2 == 0;
    const hipError_t e = gs_t<T>(M, level, op, x, y, f, 0, s, nullptr, r, nullptr, fused ? fc : nullptr);
    if (e != hipSuccess) return e;
    if (!fused) return restrict_t<T>(M, level, r, fc, uc, s);
    const LevelDev Lf = M->dev(level), Lc = M->dev(level - 1);
    const int gl = grid_for(low_items(Lc), MAX_LOW_BLOCKS), gz = uc ? grid_for(Lc.total, 2048) : 0;
    k_restrict_low<T><<<gl + gz, NT, 0, s>>>(Lf, Lc, op, y, f, kap_of<T>(M, level), r, fc, uc, Lc.total, gl);
    return hipGetLastError();
}

hipError_t launch_gs_sweep_restrict(const hhg_mesh* M, int level, int op, int dtype, void* x, void* y,
                                    const void* f, void* r, void* fc, void* uc, hipStream_t s) {
    if (dtype == DT_F64)
        return gs_restrict_t<double>(M, level, op, (double*)x, (double*)y, (const double*)f, (double*)r,
                                     (double*)fc, (double*)uc, s);
    return gs_restrict_t<float>(M, level, op, (float*)x, (float*)y, (const float*)f, (float*)r, (float*)fc,
                                (float*)uc, s);
}

template <class T>
static hipError_t prolong_t(const hhg_mesh* M, int level, const T* uc, T* u, hipStream_t s) {
    const LevelDev Lf = M->dev(level), Lc = M->dev(level - 1);
    const int gf = face_grid(Lf);
    const int gl = grid_for((int64_t)Lf.n_iedges * (Lf.n - 2) + Lf.V, MAX_LOW_BLOCKS);
    k_prolong<T><<<gf + gl, NT, 0, s>>>(Lf, Lc, uc, u, gf);
    return hipGetLastError();
}

hipError_t launch_prolong_add(const hhg_mesh* M, int level, int dtype, const void* uc, void* u,
                              hipStream_t s) {
    if (dtype == DT_F64) return prolong_t<double>(M, level, (const double*)uc, (double*)u, s);
    return prolong_t<float>(M, level, (const float*)uc, (float*)u, s);
}

hipError_t launch_fill(void* x, int64_t n, int dtype, double v, hipStream_t s) {
    const int g = grid_for(n, 4096);
    if (dtype == DT_F64) k_fill<double><<<g, NT, 0, s>>>((double*)x, n, v);
    else k_fill<float><<<g, NT, 0, s>>>((float*)x, n, (float)v);
    return hipGetLastError();
}

hipError_t launch_coarse_extract(const hhg_mesh* M, int op, double* vals, hipStream_t s) {
    const LevelDev L = M->dev(M->m.lc);
    k_coarse_extract<<<grid_for(M->coarse.N, 64), NT, 0, s>>>(L, M->coarse, op, M->kap64[M->m.lc], vals);
    return hipGetLastError();
}

template <class T>
static hipError_t coarse_t(const hhg_mesh* M, int op, T* u, const T* f, const double* vals,
                           hipStream_t s, bool u_zero) {
    const int lc = M->m.lc;
    // with u = 0 the residual is f itself (the solvers read the owned points)
    T* r = u_zero ? const_cast<T*>(f) : (T*)(sizeof(T) == 8 ? M->r64[lc] : M->r32[lc]);
    if (!u_zero) {
        hipError_t e = residual_t<T>(M, lc, op, u, f, r, nullptr, s);
        if (e != hipSuccess) return e;
    }
    const int N = M->coarse.N;
    const int which = vals == M->coarse.vals ? 0 : 1;
    double* inv = M->coarse_inv[which];
    if (N > 0 && inv && N <= CG_MAXN && M->coarse.W <= CG_W) {
        int nt = (N + CG_RPT - 1) / CG_RPT;
        nt = (nt + 63) / 64 * 64;
        if (!M->inv_ok[which]) {
            k_coarse_inverse<<<N, nt, 0, s>>>(M->coarse, vals, inv, 1e-14, 4 * N);
            M->inv_ok[which] = true;
        }
        const int nb = std::min((N + CD_NT / 64 - 1) / (CD_NT / 64), 512);
        k_coarse_dense1<T><<<nb, CD_NT, 0, s>>>(M->coarse, inv, r, M->coarse.vec);
        k_coarse_dense2<T><<<nb, CD_NT, 0, s>>>(M->coarse, vals, inv, r, M->coarse.vec, u);
    } else if (N <= CG_MAXN && M->coarse.W <= CG_W) {
        int nt = (N + CG_RPT - 1) / CG_RPT;
        nt = (nt + 63) / 64 * 64;
        k_coarse_pcg_reg<T><<<1, nt, 0, s>>>(M->coarse, vals, r, u, 1e-14, 4 * N);
    } else {
        k_coarse_pcg<T><<<1, 1024, 0, s>>>(M->coarse, vals, r, u, 1e-14, 4 * N);
    }
    return launch_sync(M, lc, sizeof(T) == 8 ? DT_F64 : DT_F32, u, GM_ALL, s);
}

hipError_t launch_coarse_solve(const hhg_mesh* M, int op, int dtype, void* u, const void* f,
                               const double* vals, hipStream_t s, bool u_zero) {
    if (dtype == DT_F64) return coarse_t<double>(M, op, (double*)u, (const double*)f, vals, s, u_zero);
    return coarse_t<float>(M, op, (float*)u, (const float*)f, vals, s, u_zero);
}

template <class T>
static hipError_t canon_t(const hhg_mesh* M, int level, const T* src, T* dst, int to_canon,
                          hipStream_t s) {
    const LevelDev L = M->dev(level);
    k_face_canon<T><<<face_grid(L), NT, 0, s>>>(L, src, dst, to_canon);
    k_low_canon<T><<<grid_for(low_items(L), MAX_LOW_BLOCKS), NT, 0, s>>>(L, src, dst, to_canon);
    if (!to_canon) return launch_sync(M, level, sizeof(T) == 8 ? DT_F64 : DT_F32, dst, GM_ALL, s);
    return hipGetLastError();
}

hipError_t launch_canon(const hhg_mesh* M, int level, int dtype, const void* src, void* dst,
                        int to_canon, hipStream_t s) {
    if (dtype == DT_F64) return canon_t<double>(M, level, (const double*)src, (double*)dst, to_canon, s);
    return canon_t<float>(M, level, (const float*)src, (float*)dst, to_canon, s);
}

template <class T>
static hipError_t inject_t(const hhg_mesh* M, int level, const T* kf, T* kc, hipStream_t s) {
    const LevelDev Lf = M->dev(level), Lc = M->dev(level - 1);
    k_face_inject<T><<<face_grid(Lc), NT, 0, s>>>(Lf, Lc, kf, kc);
    k_low_inject<T><<<grid_for(low_items(Lc), MAX_LOW_BLOCKS), NT, 0, s>>>(Lf, Lc, kf, kc);
    return launch_sync(M, level - 1, sizeof(T) == 8 ? DT_F64 : DT_F32, kc, GM_ALL, s);
}

hipError_t launch_inject(const hhg_mesh* M, int level, int dtype, const void* kf, void* kc,
                         hipStream_t s) {
    if (dtype == DT_F64) return inject_t<double>(M, level, (const double*)kf, (double*)kc, s);
    return inject_t<float>(M, level, (const float*)kf, (float*)kc, s);
}

hipError_t launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t s) {
    k_f64_to_f32<<<grid_for(n, 4096), NT, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
    k_f32_to_f64<<<grid_for(n, 4096), NT, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_add_f32_to_f64(double* u, const float* e, int64_t n, hipStream_t s) {
    k_add_f32_to_f64<<<grid_for(n, 4096), NT, 0, s>>>(u, e, n);
    return hipGetLastError();
}

template <class T>
static hipError_t jacobi_t(const hhg_mesh* M, int level, int op, const T* u, const T* f, T* rho,
                           hipStream_t s) {
    if (f) apply_tiled<T, 2>(M, level, op, u, f, rho, nullptr, s);
    else apply_tiled<T, 3>(M, level, op, u, nullptr, rho, nullptr, s);
    return hipGetLastError();
}

hipError_t launch_jacobi_low(const hhg_mesh* M, int level, int op, const float* u, const float* f,
                             float* rho, hipStream_t s) {
    const LevelDev L = M->dev(level);
    k_apply_low<float, 2><<<grid_for(low_items(L), MAX_LOW_BLOCKS), NT, 0, s>>>(L, op, u, f, rho, M->kap32[level],
                                                                                nullptr);
    return hipGetLastError();
}

hipError_t launch_jacobi(const hhg_mesh* M, int level, int op, int dtype, const void* u, const void* f,
                         void* rho, hipStream_t s) {
    if (dtype == DT_F64) return jacobi_t<double>(M, level, op, (const double*)u, (const double*)f, (double*)rho, s);
    return jacobi_t<float>(M, level, op, (const float*)u, (const float*)f, (float*)rho, s);
}

hipError_t launch_dot(const hhg_mesh* M, int level, int dtype, const void* x, const void* y, double* out,
                      hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int gf = face_grid(L);
    const int gl = grid_for((int64_t)L.n_iedges * (L.n - 2) + L.n_iverts, MAX_LOW_BLOCKS);
    if (dtype == DT_F64) k_dot<double><<<gf + gl, NT, 0, s>>>(L, (const double*)x, (const double*)y, gf, M->partials);
    else k_dot<float><<<gf + gl, NT, 0, s>>>(L, (const float*)x, (const float*)y, gf, M->partials);
    k_reduce_final<<<1, 1024, 0, s>>>(M->partials, gf + gl, out, 0);
    return hipGetLastError();
}

// Scratch of the allocation-free dot product: one partial sum per block of
// k_dot (at most MAX_FACE_BLOCKS face blocks plus MAX_LOW_BLOCKS edge/vertex
// blocks), 72 KiB per device, held from the library's first use on that
// device until the process ends.  Host code reaches it only through the
// device address hipGetSymbolAddress returns on each device.
constexpr int64_t SCRATCH_PARTIALS = (int64_t)MAX_FACE_BLOCKS + MAX_LOW_BLOCKS;
static __device__ __align__(256) double scratch[SCRATCH_PARTIALS];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t scratch_init() {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
    return hipSuccess;
}

// Partial sums k_dot needs on `level`, and whether they fit the scratch.
static int64_t dot_partials(const LevelDev& L) {
    return (int64_t)face_grid(L) + grid_for((int64_t)L.n_iedges * (L.n - 2) + L.n_iverts, MAX_LOW_BLOCKS);
}
bool dot_noalloc_fits(const hhg_mesh* M, int level) { return dot_partials(M->dev(level)) <= SCRATCH_PARTIALS; }

hipError_t launch_dot_noalloc(const hhg_mesh* M, int level, int dtype, const void* x, const void* y,
                              double* out, hipStream_t s) {
    hipError_t e = scratch_init();
    if (e != hipSuccess) return e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        part = g_scratch_ptr[dev];
    }
    const LevelDev L = M->dev(level);
    const int gf = face_grid(L);
    const int gl = grid_for((int64_t)L.n_iedges * (L.n - 2) + L.n_iverts, MAX_LOW_BLOCKS);
    if ((int64_t)gf + gl > SCRATCH_PARTIALS) return hipErrorInvalidValue;   // callers check first
    if (dtype == DT_F64) k_dot<double><<<gf + gl, NT, 0, s>>>(L, (const double*)x, (const double*)y, gf, part);
    else k_dot<float><<<gf + gl, NT, 0, s>>>(L, (const float*)x, (const float*)y, gf, part);
    k_reduce_final<<<1, 1024, 0, s>>>(part, gf + gl, out, 0);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int64_t count, double* out, hipStream_t s) {
    k_reduce_final<<<1, 1024, 0, s>>>(partials, count, out, 0);
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, int dtype, double alpha, const void* x, double beta, const void* y,
                        void* z, hipStream_t s) {
    const int g = grid_for(n, 4096);
    if (dtype == DT_F64)
        k_axpby<double><<<g, NT, 0, s>>>(n, alpha, (const double*)x, beta, (const double*)y, (double*)z);
    else
        k_axpby<float><<<g, NT, 0, s>>>(n, (float)alpha, (const float*)x, (float)beta, (const float*)y, (float*)z);
    return hipGetLastError();
}

hipError_t launch_low_gs(const hhg_mesh* M, int level, int op, int dtype, void* u, const void* f,
                         int stage, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int gl = grid_for((int64_t)L.E * (L.n - 2) + L.V, MAX_LOW_BLOCKS);
    if (dtype == DT_F64)
        k_low_gs<double><<<gl, NT, 0, s>>>(L, op, (double*)u, (const double*)f, M->kap64[level], stage);
    else
        k_low_gs<float><<<gl, NT, 0, s>>>(L, op, (float*)u, (const float*)f, M->kap32[level], stage);
    return hipGetLastError();
}

}  // namespace hhg
