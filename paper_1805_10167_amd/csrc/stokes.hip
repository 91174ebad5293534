// HIP kernels (gfx950) of the equal-order P1-P1 Stokes system with pressure
// stabilisation (the monolithic saddle-point problem of the paper's
// energy-transport example, sec. 5.2) and of the preconditioned MINRES
// iteration that solves it (sec. 4.3).
//
// A Stokes vector is three fields of one level, u_x | u_y | p, each of
// `fs` elements in the level layout (owned values and ghost copies).  The
// operator
//   [ A    0    BX^T ] [u_x]
//   [ 0    A    BY^T ] [u_y]
//   [ BX   BY   -C   ] [ p ]
// is applied matrix-free from one constant stencil per primitive and block
// (StokesFace / StokesEdge / StokesVert, built on the host by P1 element
// assembly at the macro scale): the viscous block is level independent, the
// divergence and gradient blocks scale with the micro-step h = 2^-l, the
// stabilisation and the lumped pressure mass with h^2.  Velocity rows of
// Dirichlet points are zero (the velocity there is data, not an unknown);
// pressure rows exist at every point.
//
// Edge points read the near-row points of their faces straight from the
// face arrays (which own them), so no ghost row is needed for edges on the
// boundary; vertices read their ring from their own ghost slots.  Every
// kernel that writes a value also writes its ghost copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "hhg_device.hpp"

namespace hhg {

// face-local offsets of the 7 face-stencil neighbours C, E, W, N, S, SE, NW
struct FaceNbr {
    int64_t o[7];
};
__device__ __forceinline__ FaceNbr face_nbr(int64_t p, int64_t up, int64_t dn) {
    FaceNbr q;
    q.o[0] = p; q.o[1] = p + 1; q.o[2] = p - 1; q.o[3] = p + up; q.o[4] = p - dn;
    q.o[5] = p - dn + 1; q.o[6] = p + up - 1;
    return q;
}

// Near-row point g_s[m] of edge side s in its face's array (face-local
// point at distance 1 from the side, parameter t along the side).
__device__ __forceinline__ int64_t near_row(const LevelDev& L, const EdgeInfo& ei, int s, int m) {
    const int n = L.n;
    const int t = ei.rev[s] ? n - 2 - m : m;
    int i, j;
    if (ei.side[s] == 0) { i = t; j = 1; }
    else if (ei.side[s] == 1) { i = 1; j = t; }
    else { i = n - 2 - t; j = t; }
    return face_base(L, ei.face[s]) + row_start(n, j) + i;
}

// y = K x of the three blocks at one point from its neighbour values.
template <int W>
__device__ __forceinline__ void stokes_rows(const double (&w)[SB_N][W], int cnt, const double* ux,
                                            const double* uy, const double* pp, double hB, double hC,
                                            double& yx, double& yy, double& yp) {
    double ax = 0.0, ay = 0.0, gx = 0.0, gy = 0.0, dx = 0.0, dy = 0.0, cp = 0.0;
    for (int t = 0; t < cnt; ++t) {
        ax += w[SB_A][t] * ux[t];
        ay += w[SB_A][t] * uy[t];
        gx += w[SB_BXT][t] * pp[t];
        gy += w[SB_BYT][t] * pp[t];
        dx += w[SB_BX][t] * ux[t];
        dy += w[SB_BY][t] * uy[t];
        cp += w[SB_C][t] * pp[t];
    }
    yx = ax + hB * gx;
    yy = ay + hB * gy;
    yp = hB * (dx + dy) - hC * cp;
}

// Stokes operator over a whole level.
//   MODE 0: y = K x
//   MODE 1: y = K x and per-block sums of y . x over owned points
//   MODE 2: y = b - K x (velocity rows of Dirichlet points 0)
// k_stokes_apply takes the face-interior rows over the smoother's TI x TJ
// tiles (halo-3 tile list, grid-stride over gf blocks), each in three
// sub-tiles of ST_SJ rows whose three fields are staged with a one-point
// halo in LDS (one round of independent loads, LDS stores after); a wave
// forms one row of a sub-tile.  k_stokes_apply_low takes the edge points and
// vertices in a launch of its own (their ring arrays would otherwise size
// the face kernel's registers), its block sums after the face blocks'.
constexpr int ST_NT = 512, ST_NW = ST_NT / 64, ST_SJ = ST_NW;
constexpr int ST_TI = GS_W - 2 * GS_H, ST_TJ = GS_TJ, ST_RA = ST_SJ + 2;
constexpr int ST_RPW = (ST_RA + ST_NW - 1) / ST_NW;
static_assert(ST_TJ % ST_SJ == 0, "sub-tiles must split the tile rows");
static_assert(ST_TI + 2 <= GS_W, "tile with halo must fit an LDS row");

// LDS offsets of the neighbours C, E, W, N, S, SE, NW in a GS_W-wide tile
__constant__ int c_st_off[7] = {0, 1, -1, GS_W, -GS_W, -GS_W + 1, GS_W - 1};

template <int MODE>
__global__ __launch_bounds__(ST_NT) void k_stokes_apply(LevelDev L, const double* __restrict__ x,
                                                        const double* __restrict__ b, double* __restrict__ y,
                                                        int64_t fs, double hB, double hC, int gf,
                                                        double* __restrict__ partials) {
    __shared__ double xs[3][ST_RA][GS_W];
    __shared__ double ws[SB_N][7];                 // the face's stencils (broadcast reads)
    __shared__ double sm[ST_NW + 1];
    double acc = 0.0;
    const double* xx = x;
    const double* xy = x + fs;
    const double* xp = x + 2 * fs;
    double* yx_ = y;
    double* yy_ = y + fs;
    double* yp_ = y + 2 * fs;
    const int n = L.n;
    {
        const int wv = wave_id(), lane = threadIdx.x & 63;
        const int ntl = L.n_gs_tl[0][0];
        const int ntiles = L.F * ntl;
        for (int tile = blockIdx.x; tile < ntiles; tile += gf) {
            const int face = tile / ntl;
            const int2 tl = L.gs_tl[0][0][tile % ntl];
            const FaceInfo& fi = L.faces[face];
            const FaceGhosts gh = face_ghosts(L, fi);
            const int64_t fb = face_base(L, face);
            if (threadIdx.x < SB_N * 7) (&ws[0][0])[threadIdx.x] = (&L.sfaces[face].w[0][0])[threadIdx.x];
            for (int sub = 0; sub < ST_TJ / ST_SJ; ++sub) {
                const int i0 = tl.x * ST_TI - 1, j0 = tl.y * ST_TJ + sub * ST_SJ - 1;   // LDS origin
                if (j0 + 1 > n - 3) break;                 // no interior rows left (block-uniform)
                double xr[3][ST_RPW][3];
#pragma unroll
                for (int q = 0; q < ST_RPW; ++q) {
                    const int r = wv + ST_NW * q, j = j0 + r;
                    const int64_t rb = fb + row_start(n, j < 0 ? 0 : (j > n ? n : j));
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const int tx = lane + 64 * c, i = i0 + tx;
                        const bool in = r < ST_RA && tx < ST_TI + 2 && j >= 0 && j < n && i >= 0 && i <= n - 1 - j;
                        xr[0][q][c] = in ? xx[rb + i] : 0.0;
                        xr[1][q][c] = in ? xy[rb + i] : 0.0;
                        xr[2][q][c] = in ? xp[rb + i] : 0.0;
                    }
                }
                const int r = 1 + wv, j = j0 + r;           // this wave's output row
                double br[3][3];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    const bool pt = MODE == 2 && tx >= 1 && tx <= ST_TI && j >= 1 && i >= 1 && i + j <= n - 2;
                    const int64_t pb = fb + row_start(n, pt ? j : 0) + i;
                    br[0][c] = pt ? b[pb] : 0.0;
                    br[1][c] = pt ? b[fs + pb] : 0.0;
                    br[2][c] = pt ? b[2 * fs + pb] : 0.0;
                }
                __syncthreads();                           // the previous sub-tile's LDS reads are done
#pragma unroll
                for (int q = 0; q < ST_RPW; ++q) {
                    const int rr = wv + ST_NW * q;
                    if (rr >= ST_RA) continue;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        xs[0][rr][lane + 64 * c] = xr[0][q][c];
                        xs[1][rr][lane + 64 * c] = xr[1][q][c];
                        xs[2][rr][lane + 64 * c] = xr[2][q][c];
                    }
                }
                __syncthreads();
                const int64_t rowb = fb + row_start(n, j >= 1 && j <= n - 3 ? j : 1);
                // one column at a time: unrolled, the three columns' 63 LDS
                // reads are hoisted together and the registers triple
#pragma unroll 1
                for (int c = 0; c < 3; ++c) {
                    const int tx = lane + 64 * c, i = i0 + tx;
                    if (!(tx >= 1 && tx <= ST_TI && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
                    // the seven sums of stokes_rows, tap by tap (neighbours C, E,
                    // W, N, S, SE, NW): few values live at a time
                    const double* x0 = &xs[0][r][tx];
                    const double* x1 = &xs[1][r][tx];
                    const double* x2 = &xs[2][r][tx];
                    double ax = 0.0, ay = 0.0, gx = 0.0, gy = 0.0, dx = 0.0, dy = 0.0, cp = 0.0;
                    double u0 = 0.0, v0 = 0.0, p0 = 0.0;
#pragma unroll 1
                    for (int t = 0; t < 7; ++t) {
                        const int o = c_st_off[t];
                        const double a = x0[o], bq = x1[o], pq = x2[o];
                        if (t == 0) { u0 = a; v0 = bq; p0 = pq; }
                        ax += ws[SB_A][t] * a;
                        ay += ws[SB_A][t] * bq;
                        gx += ws[SB_BXT][t] * pq;
                        gy += ws[SB_BYT][t] * pq;
                        dx += ws[SB_BX][t] * a;
                        dy += ws[SB_BY][t] * bq;
                        cp += ws[SB_C][t] * pq;
                    }
                    double vx = ax + hB * gx, vy = ay + hB * gy, vp = hB * (dx + dy) - hC * cp;
                    if (MODE == 2) {
                        vx = (c == 0 ? br[0][0] : c == 1 ? br[0][1] : br[0][2]) - vx;
                        vy = (c == 0 ? br[1][0] : c == 1 ? br[1][1] : br[1][2]) - vy;
                        vp = (c == 0 ? br[2][0] : c == 1 ? br[2][1] : br[2][2]) - vp;
                    }
                    if (MODE == 1) acc += vx * u0 + vy * v0 + vp * p0;
                    const int64_t p = rowb + i;
                    yx_[p] = vx;
                    yy_[p] = vy;
                    yp_[p] = vp;
                    push_face_near(gh, n, yx_, i, j, vx);
                    push_face_near(gh, n, yy_, i, j, vy);
                    push_face_near(gh, n, yp_, i, j, vp);
                }
            }
            __syncthreads();                               // LDS free for the next tile
        }
    }
    if (MODE == 1) {
        const double sblk = block_sum<ST_NT>(acc, sm);
        if (threadIdx.x == 0) partials[blockIdx.x] = sblk;
    }
}

template <int MODE>
__global__ __launch_bounds__(NT) void k_stokes_apply_low(LevelDev L, const double* __restrict__ x,
                                                        const double* __restrict__ b, double* __restrict__ y,
                                                        int64_t fs, double hB, double hC,
                                                        double* __restrict__ partials) {
    __shared__ double sm[NT / 64 + 1];
    double acc = 0.0;
    const double* xx = x;
    const double* xy = x + fs;
    const double* xp = x + 2 * fs;
    double* yx_ = y;
    double* yy_ = y + fs;
    double* yp_ = y + 2 * fs;
    const int n = L.n;
    {
        const int64_t ne = (int64_t)L.E * (n - 2);
        for (int64_t t = (int64_t)blockIdx.x * NT + threadIdx.x; t < ne + L.V; t += (int64_t)gridDim.x * NT) {
            double ux[1 + MAXDEG], uy[1 + MAXDEG], pp[1 + MAXDEG];
            double vx, vy, vp;
            if (t < ne) {
                const int e = (int)(t / (n - 2)), k = (int)(t % (n - 2)) + 1;
                const EdgeInfo& ei = L.edges[e];
                const StokesEdge& se = L.sedges[e];
                const int64_t m = edge_main(L, e) + k;
                int64_t o[7];
                o[0] = m; o[1] = m - 1; o[2] = m + 1;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const bool has = s < ei.nf;
                    o[3 + 2 * s] = has ? near_row(L, ei, s, k - 1) : m;
                    o[4 + 2 * s] = has ? near_row(L, ei, s, k) : m;
                }
#pragma unroll
                for (int u = 0; u < 7; ++u) {
                    ux[u] = xx[o[u]];
                    uy[u] = xy[o[u]];
                    pp[u] = xp[o[u]];
                }
                stokes_rows<7>(se.w, 7, ux, uy, pp, hB, hC, vx, vy, vp);
                if (MODE == 2) {
                    vx = b[m] - vx;
                    vy = b[fs + m] - vy;
                    vp = b[2 * fs + m] - vp;
                }
                if (ei.boundary) vx = vy = 0.0;
                if (MODE == 1) acc += vx * ux[0] + vy * uy[0] + vp * pp[0];
                yx_[m] = vx;
                yy_[m] = vy;
                yp_[m] = vp;
                push_edge(L, yx_, ei, k, vx, true);
                push_edge(L, yy_, ei, k, vy, true);
                push_edge(L, yp_, ei, k, vp, true);
            } else {
                const int v = (int)(t - ne);
                const VertexInfo& vi = L.verts[v];
                const StokesVert& sv = L.sverts[v];
                const int64_t vb = vert_off(L, v);
                const int deg = vi.deg;
                for (int u = 0; u <= deg; ++u) {
                    ux[u] = xx[vb + u];
                    uy[u] = xy[vb + u];
                    pp[u] = xp[vb + u];
                }
                stokes_rows<1 + MAXDEG>(sv.w, deg + 1, ux, uy, pp, hB, hC, vx, vy, vp);
                if (MODE == 2) {
                    vx = b[vb] - vx;
                    vy = b[fs + vb] - vy;
                    vp = b[2 * fs + vb] - vp;
                }
                if (vi.boundary) vx = vy = 0.0;
                if (MODE == 1) acc += vx * ux[0] + vy * uy[0] + vp * pp[0];
                yx_[vb] = vx;
                yy_[vb] = vy;
                yp_[vb] = vp;
                push_vertex(L, yx_, vi, vx);
                push_vertex(L, yy_, vi, vy);
                push_vertex(L, yp_, vi, vp);
            }
        }
    }
    if (MODE == 1) {
        const double sblk = block_sum<NT>(acc, sm);
        if (threadIdx.x == 0) partials[blockIdx.x] = sblk;
    }
}

// Pressure block of the preconditioner, z_p = r_p / m (m: lumped mass
// weighted with 1/mu plus 4 times the centre weight of the stabilisation C,
// at level scale hC), with every copy of z_p, and
// per-block sums of r . z over owned points of all three fields (the
// velocity parts of z are already in place).
__global__ __launch_bounds__(NT) void k_stokes_pscale_dot(LevelDev L, const double* __restrict__ r,
                                                          double* __restrict__ z, int64_t fs, double hC, int gf,
                                                          double* __restrict__ partials) {
    __shared__ double sm[NT / 64 + 1];
    double acc = 0.0;
    const double* rp = r + 2 * fs;
    double* zp = z + 2 * fs;
    if ((int)blockIdx.x < gf) {
        FACE_TILE_LOOP(L, gf)
        (void)up;
        (void)dn;
        const double v = rp[p] / (hC * L.sfaces[face].m);
        zp[p] = v;
        push_face_near(L, zp, fi, i, j, v);
        acc += r[p] * z[p] + r[fs + p] * z[fs + p] + rp[p] * v;
        FACE_TILE_END
    } else {
        LOW_LOOP(L, gf) {
            int64_t q;
            double v;
            if (t < ne_) {
                const int e = (int)(t / (nl_ - 2)), k = (int)(t % (nl_ - 2)) + 1;
                q = edge_main(L, e) + k;
                v = rp[q] / (hC * L.sedges[e].m);
                zp[q] = v;
                push_edge(L, zp, L.edges[e], k, v, true);
            } else {
                const int vv = (int)(t - ne_);
                q = vert_off(L, vv);
                v = rp[q] / (hC * L.sverts[vv].m);
                zp[q] = v;
                push_vertex(L, zp, L.verts[vv], v);
            }
            acc += r[q] * z[q] + r[fs + q] * z[fs + q] + rp[q] * v;
        }
    }
    const double sblk = block_sum<NT>(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = sblk;
}

// Per-block sums of a . b over the owned points of the three fields.
__global__ __launch_bounds__(NT) void k_stokes_dot(LevelDev L, const double* __restrict__ a,
                                                   const double* __restrict__ b, int64_t fs, int gf,
                                                   double* __restrict__ partials) {
    __shared__ double sm[NT / 64 + 1];
    double acc = 0.0;
    if ((int)blockIdx.x < gf) {
        FACE_TILE_LOOP(L, gf)
        (void)fi;
        (void)up;
        (void)dn;
        acc += a[p] * b[p] + a[fs + p] * b[fs + p] + a[2 * fs + p] * b[2 * fs + p];
        FACE_TILE_END
    } else {
        LOW_LOOP(L, gf) {
            int64_t q;
            if (t < ne_) q = edge_main(L, (int)(t / (nl_ - 2))) + (t % (nl_ - 2)) + 1;
            else q = vert_off(L, (int)(t - ne_));
            acc += a[q] * b[q] + a[fs + q] * b[fs + q] + a[2 * fs + q] * b[2 * fs + q];
        }
    }
    const double sblk = block_sum<NT>(acc, sm);
    if (threadIdx.x == 0) partials[blockIdx.x] = sblk;
}

// MINRES scalar state (device memory), see launch_minres_scalars.
enum {
    MS_BNORM = 0,   // beta_k: norm of the current Lanczos vector (z_k = y_k / beta_k, v_k = r_k / beta_k)
    MS_BPREV,       // beta_{k-1}
    MS_BSUB,        // sub-diagonal entry of column k of the Lanczos matrix (0 at k = 1)
    MS_ALPHA,
    MS_COLD, MS_SOLD, MS_C, MS_S,   // rotations k-2 and k-1
    MS_ETA,         // rotated right-hand side entry: |eta| = P^-1-norm of the residual
    MS_ETA0,
    MS_A1, MS_A2, MS_A3,            // r_{k+1} = a1 K y_k - a2 r_k - a3 r_{k-1}
    MS_W1, MS_W2, MS_W3, MS_TAU,    // w = w1 y_k - w2 w_{k-1} - w3 w_{k-2}; x += tau w
    MS_K,           // Lanczos step
    MS_NSTATE
};

// Fixed-order sum of the partials, then the scalar part of one MINRES stage
// by thread 0:
//   STAGE 0 (after the first preconditioned residual): beta_1 and the start
//           state;
//   STAGE 1 (after y = K y_k with the sums of y . y_k): alpha_k and the
//           coefficients of the Lanczos recurrence;
//   STAGE 2 (after the new preconditioned vector with the sums of r . z):
//           beta_{k+1}, one Givens rotation, the update coefficients of the
//           direction and the iterate, and the residual norm |eta| into
//           slot[0] (slot[1] = beta_{k+1}, slot[2] = beta_1).
template <int STAGE>
__global__ __launch_bounds__(1024) void k_minres_scalars(const double* __restrict__ partials, int64_t count,
                                                         double* __restrict__ st, double* __restrict__ slot) {
    __shared__ double sm[1024 / 64 + 1];
    double a = 0.0;
    for (int64_t t = threadIdx.x; t < count; t += 1024) a += partials[t];
    const double sum = block_sum<1024>(a, sm);
    if (threadIdx.x != 0) return;
    // a sum that rounding left slightly negative counts as 0; a NaN stays NaN
    // (fmax would drop it), so the host sees a broken start or breakdown
    const double root = sum >= 0.0 ? sqrt(sum) : (sum < 0.0 ? 0.0 : sum);
    if (STAGE == 0) {
        const double beta = root;
        st[MS_BNORM] = beta;
        st[MS_BPREV] = 0.0;
        st[MS_BSUB] = 0.0;
        st[MS_COLD] = st[MS_C] = 1.0;
        st[MS_SOLD] = st[MS_S] = 0.0;
        st[MS_ETA] = st[MS_ETA0] = beta;
        st[MS_K] = 1.0;
        slot[0] = beta;
        slot[1] = beta;
        slot[2] = beta;
    } else if (STAGE == 1) {
        const double bn = st[MS_BNORM];
        const double alpha = sum / (bn * bn);
        st[MS_ALPHA] = alpha;
        st[MS_A1] = 1.0 / bn;
        st[MS_A2] = alpha / bn;
        st[MS_A3] = st[MS_BPREV] > 0.0 ? st[MS_BSUB] / st[MS_BPREV] : 0.0;
    } else {
        const double bnext = root;
        const double bsub = st[MS_BSUB], alpha = st[MS_ALPHA];
        const double c_old = st[MS_COLD], s_old = st[MS_SOLD], c = st[MS_C], s = st[MS_S];
        const double eps = s_old * bsub;
        const double dbar = c_old * bsub;
        const double delta = c * dbar + s * alpha;
        const double gbar = -s * dbar + c * alpha;
        const double gamma = hypot(gbar, bnext);
        const double c_new = gamma > 0.0 ? gbar / gamma : 1.0;
        const double s_new = gamma > 0.0 ? bnext / gamma : 0.0;
        const double eta = st[MS_ETA];
        const double ig = gamma > 0.0 ? 1.0 / gamma : 0.0;
        st[MS_W1] = ig / st[MS_BNORM];
        st[MS_W2] = delta * ig;
        st[MS_W3] = eps * ig;
        st[MS_TAU] = c_new * eta;
        st[MS_ETA] = -s_new * eta;
        st[MS_COLD] = c;
        st[MS_SOLD] = s;
        st[MS_C] = c_new;
        st[MS_S] = s_new;
        st[MS_BPREV] = st[MS_BNORM];
        st[MS_BNORM] = bnext;
        st[MS_BSUB] = bnext;
        st[MS_K] += 1.0;
        slot[0] = fabs(-s_new * eta);
        slot[1] = bnext;
    }
}

// r_old <- a1 y - a2 r - a3 r_old over whole fields (copies included).
__global__ __launch_bounds__(NT) void k_minres_rupdate(int64_t n, const double* __restrict__ y,
                                                       const double* __restrict__ r, double* __restrict__ r_old,
                                                       const double* __restrict__ st) {
    const double a1 = st[MS_A1], a2 = st[MS_A2], a3 = st[MS_A3];
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT)
        r_old[t] = a1 * y[t] - a2 * r[t] - a3 * r_old[t];
}

// w_older <- w1 y - w2 w_old - w3 w_older, x += tau w_older.
__global__ __launch_bounds__(NT) void k_minres_wupdate(int64_t n, const double* __restrict__ yk,
                                                       const double* __restrict__ w_old,
                                                       double* __restrict__ w_older, double* __restrict__ x,
                                                       const double* __restrict__ st) {
    const double w1 = st[MS_W1], w2 = st[MS_W2], w3 = st[MS_W3], tau = st[MS_TAU];
    for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n; t += (int64_t)gridDim.x * NT) {
        const double w = w1 * yk[t] - w2 * w_old[t] - w3 * w_older[t];
        w_older[t] = w;
        x[t] += tau * w;
    }
}

// ------------------------------------------------------------------ launchers

static inline int st_grid_for(int64_t items, int cap) {
    int64_t g = (items + NT - 1) / NT;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}
struct StGrid {
    int gf, gl;
};
static inline StGrid st_grid(const LevelDev& L) {
    StGrid g;
    g.gf = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)L.F * L.ntiles, MAX_FACE_BLOCKS));
    g.gl = st_grid_for((int64_t)L.E * (L.n - 2) + L.V, MAX_LOW_BLOCKS);
    return g;
}

int64_t stokes_partials() { return (int64_t)MAX_FACE_BLOCKS + MAX_LOW_BLOCKS; }

hipError_t launch_stokes_apply(const hhg_mesh* M, int level, int mode, const double* x, const double* b,
                               double* y, double* partials, int64_t* nparts, hipStream_t s) {
    const LevelDev L = M->dev(level);
    StGrid g;
    g.gf = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)L.F * L.n_gs_tl[0][0], MAX_FACE_BLOCKS));
    g.gl = st_grid_for((int64_t)L.E * (L.n - 2) + L.V, MAX_LOW_BLOCKS);
    double* lp = partials ? partials + g.gf : nullptr;
    const int64_t fs = L.total;
    const double hB = std::ldexp(1.0, -level), hC = L.inv4l;
    if (mode == 0) {
        k_stokes_apply<0><<<g.gf, ST_NT, 0, s>>>(L, x, b, y, fs, hB, hC, g.gf, partials);
        k_stokes_apply_low<0><<<g.gl, NT, 0, s>>>(L, x, b, y, fs, hB, hC, lp);
    } else if (mode == 1) {
        k_stokes_apply<1><<<g.gf, ST_NT, 0, s>>>(L, x, b, y, fs, hB, hC, g.gf, partials);
        k_stokes_apply_low<1><<<g.gl, NT, 0, s>>>(L, x, b, y, fs, hB, hC, lp);
    } else {
        k_stokes_apply<2><<<g.gf, ST_NT, 0, s>>>(L, x, b, y, fs, hB, hC, g.gf, partials);
        k_stokes_apply_low<2><<<g.gl, NT, 0, s>>>(L, x, b, y, fs, hB, hC, lp);
    }
    if (nparts) *nparts = g.gf + g.gl;
    return hipGetLastError();
}

hipError_t launch_stokes_pscale_dot(const hhg_mesh* M, int level, const double* r, double* z,
                                    double* partials, int64_t* nparts, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const StGrid g = st_grid(L);
    k_stokes_pscale_dot<<<g.gf + g.gl, NT, 0, s>>>(L, r, z, L.total, L.inv4l, g.gf, partials);
    if (nparts) *nparts = g.gf + g.gl;
    return hipGetLastError();
}

hipError_t launch_stokes_dot(const hhg_mesh* M, int level, const double* a, const double* b,
                             double* partials, int64_t* nparts, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const StGrid g = st_grid(L);
    k_stokes_dot<<<g.gf + g.gl, NT, 0, s>>>(L, a, b, L.total, g.gf, partials);
    if (nparts) *nparts = g.gf + g.gl;
    return hipGetLastError();
}

hipError_t launch_minres_scalars(int stage, const double* partials, int64_t count, double* st, double* slot,
                                 hipStream_t s) {
    if (stage == 0) k_minres_scalars<0><<<1, 1024, 0, s>>>(partials, count, st, slot);
    else if (stage == 1) k_minres_scalars<1><<<1, 1024, 0, s>>>(partials, count, st, slot);
    else k_minres_scalars<2><<<1, 1024, 0, s>>>(partials, count, st, slot);
    return hipGetLastError();
}

hipError_t launch_minres_rupdate(int64_t n, const double* y, const double* r, double* r_old, const double* st,
                                 hipStream_t s) {
    k_minres_rupdate<<<st_grid_for(n, 8192), NT, 0, s>>>(n, y, r, r_old, st);
    return hipGetLastError();
}

hipError_t launch_minres_wupdate(int64_t n, const double* yk, const double* w_old, double* w_older, double* x,
                                 const double* st, hipStream_t s) {
    k_minres_wupdate<<<st_grid_for(n, 8192), NT, 0, s>>>(n, yk, w_old, w_older, x, st);
    return hipGetLastError();
}

}  // namespace hhg
