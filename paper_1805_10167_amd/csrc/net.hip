// Learned face smoother: a two-layer hexagonal CNN on the refined
// macro-faces (not part of the paper; a smoother variant layered on the
// multigrid method).  out = N(rho) with
//   a_c(q)  = sum_t W1[c][t] rho(q + d_t)            (16 hidden channels)
//   h_c(q)  = ReLU(a_c(q)) on face-interior q, 0 elsewhere
//   out(p)  = sum_t sum_c W2[c][t] h_c(p + d_t)     (face-interior p)
// over the 7 offsets d_t = C, E, W, N, S, SE, NW of face-local (i, j).
//
// Forward on MFMA (BF16 operands, FP32 accumulation), per 16 pixels:
//   layer 1 as a^T = W1 (16 ch x 16 taps) * R^T (16 taps x 16 px), so that
//   the output registers hold h in exactly the A-operand layout of
//   layer 2: z = h (16 px x 16 ch) * W2 (16 ch x 16 taps), then
//   out(p) = sum_t z_t(p + d_t) from LDS.
// Lane layout of v_mfma_f32_16x16x16_bf16 (64 lanes): A[m][k] in lane
// m + 16 (k / 4) element k % 4; B[k][n] in lane n + 16 (k / 4) element
// k % 4; D[m][n] in lane n + 16 (m / 4) element m % 4.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhg_kernels.hpp"

namespace hhg {

constexpr int NET_NT = 256;
constexpr int NZ = NET_TI + 2, NZR = NET_TJ + 2;      // hidden/z region (tile + 1)
constexpr int NRW = NET_TI + 4, NRR = NET_TJ + 4;     // rho region (tile + 2)
constexpr int NPX = NZ * NZR;                          // pixels of the hidden region

__constant__ int c_di[7] = {0, 1, -1, 0, 0, 1, -1};
__constant__ int c_dj[7] = {0, 0, 0, 1, -1, -1, 1};

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// Round to nearest even BF16 (the hardware conversion).
__device__ __forceinline__ short4v to_bf16x4(float a, float b, float c, float d) {
    const bf16x2 lo = __builtin_convertvector((float2v){a, b}, bf16x2);
    const bf16x2 hi = __builtin_convertvector((float2v){c, d}, bf16x2);
    const bf16x4 v = {lo[0], lo[1], hi[0], hi[1]};
    return __builtin_bit_cast(short4v, v);
}
__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

__device__ __forceinline__ int nrow_start(int n, int j) {
    const auto S = [](int N) { const int q = N >> 4, t = N & 15; return 8 * q * (q + 1) + t * (q + 1); };
    return 16 * (S(n) - S(n - j));
}

__device__ __forceinline__ int64_t nface_base(const LevelDev& L, int f) {
    return L.face_base + (int64_t)f * L.face_stride;
}
__device__ __forceinline__ int64_t nedge_ghost(const LevelDev& L, int e, int s) {
    return L.edge_base + (int64_t)e * L.edge_stride + L.ghost_off + (int64_t)s * L.ghost_stride;
}

// z_t over the tile grown by 1: MFMA (BF16) or FP32 arithmetic.  Each wave
// takes groups of 16 hidden pixels; two groups per trip give the scheduler
// independent MFMA chains to interleave.
constexpr int NGRP = (NPX + 15) / 16;
constexpr int NWV = NET_NT / 64;
constexpr int GPW = (NGRP + NWV - 1) / NWV;

template <bool MFMA>
__device__ __forceinline__ void net_hidden(int n, int i0, int j0, const float* __restrict__ W,
                                           float (*rs)[NRW], float (*zs)[NPX]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (MFMA) {
        const int q4 = lane >> 4, l16 = lane & 15;
        float a1[4], a2[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = 4 * q4 + e;
            a1[e] = t < 7 ? W[l16 * 7 + t] : 0.f;            // A[c = l16][k = t]
            a2[e] = l16 < 7 ? W[112 + t * 7 + l16] : 0.f;     // B[k = c = t][n = tap l16]
        }
        const short4v w1op = to_bf16x4(a1[0], a1[1], a1[2], a1[3]);
        const short4v w2op = to_bf16x4(a2[0], a2[1], a2[2], a2[3]);
        int di[4], dj[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = 4 * q4 + e;
            di[e] = t < 7 ? c_di[t] : 0;
            dj[e] = t < 7 ? c_dj[t] : 0;
        }
#pragma unroll 2
        for (int it = 0; it < GPW; ++it) {
            const int g = wv + NWV * it;
            if (g >= NGRP) break;
            const int px = g * 16 + l16;
            const int pxc = px < NPX ? px : NPX - 1;
            const int rr = pxc / NZ, cc = pxc - rr * NZ;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float x = rs[rr + 1 + dj[e]][cc + 1 + di[e]];
                v[e] = (4 * q4 + e < 7) ? x : 0.f;
            }
            float4v acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1op, to_bf16x4(v[0], v[1], v[2], v[3]),
                                                            acc, 0, 0, 0);
            // lane holds a for channels 4 q4 + e of pixel l16: ReLU on interior
            const int j = j0 - 1 + rr, i = i0 - 1 + cc;
            const bool inner = px < NPX && j >= 1 && i >= 1 && i + j <= n - 2;
            const short4v hop = to_bf16x4(inner ? fmaxf(acc[0], 0.f) : 0.f, inner ? fmaxf(acc[1], 0.f) : 0.f,
                                          inner ? fmaxf(acc[2], 0.f) : 0.f, inner ? fmaxf(acc[3], 0.f) : 0.f);
            float4v z = {0.f, 0.f, 0.f, 0.f};
            z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hop, w2op, z, 0, 0, 0);
            // lane holds z for tap l16 of pixels 4 q4 + e
            if (l16 < 7)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int p2 = g * 16 + 4 * q4 + e;
                    if (p2 < NPX) zs[l16][p2] = z[e];
                }
        }
    } else {
        for (int px = threadIdx.x; px < NPX; px += NET_NT) {
            const int rr = px / NZ, cc = px - rr * NZ;
            const int j = j0 - 1 + rr, i = i0 - 1 + cc;
            const bool inner = j >= 1 && i >= 1 && i + j <= n - 2;
            float rt[7];
            for (int t = 0; t < 7; ++t) rt[t] = rs[rr + 1 + c_dj[t]][cc + 1 + c_di[t]];
            float z[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int c = 0; c < 16; ++c) {
                float a = 0.f;
                for (int t = 0; t < 7; ++t) a += W[c * 7 + t] * rt[t];
                const float h = inner ? fmaxf(a, 0.f) : 0.f;
                for (int t = 0; t < 7; ++t) z[t] += W[112 + c * 7 + t] * h;
            }
            for (int t = 0; t < 7; ++t) zs[t][px] = z[t];
        }
    }
}

// out = N(rho) on face-interior points (mode 0: write out, whose other
// entries the caller has zeroed; mode 1: u += N(rho) in place).  Both write
// the near-edge-row copies of what they change.  All global loads of a
// thread are issued together: rho for the LDS tile, then (mode 1) the
// outputs' old values, which arrive while the MFMA phase runs.
constexpr int NLD = (NRR * NRW + NET_NT - 1) / NET_NT;
constexpr int NOUT = (NET_TI * NET_TJ + NET_NT - 1) / NET_NT;

template <class T, bool MFMA>
__global__ __launch_bounds__(NET_NT) void k_net_forward(LevelDev L, const T* __restrict__ rho,
                                                        T* __restrict__ y, const float* __restrict__ W,
                                                        int mode) {
    __shared__ float rs[NRR][NRW];
    __shared__ float zs[7][NPX];
    const int n = L.n;
    const int face = blockIdx.x / L.n_net_tiles;
    const int2 tl = L.net_tiles[blockIdx.x % L.n_net_tiles];
    const int i0 = tl.x * NET_TI, j0 = tl.y * NET_TJ;
    const FaceInfo& fi = L.faces[face];
    const int64_t fb = nface_base(L, face);
    float v[NLD];
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int idx = threadIdx.x + k * NET_NT;
        const int r = idx / NRW, c = idx - r * NRW;
        const int j = j0 - 2 + r, i = i0 - 2 + c;
        v[k] = 0.f;
        if (idx < NRR * NRW && j >= 0 && j < n && i >= 0 && i <= n - 1 - j)
            v[k] = (float)rho[fb + nrow_start(n, j) + i];
    }
    int64_t po[NOUT];
    float yo[NOUT];
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        const int idx = threadIdx.x + k * NET_NT;
        const int rr = idx / NET_TI, cc = idx - rr * NET_TI;
        const int j = j0 + rr, i = i0 + cc;
        const bool ok = idx < NET_TI * NET_TJ && j >= 1 && i >= 1 && i + j <= n - 2;
        po[k] = ok ? fb + nrow_start(n, j) + i : -1;
        yo[k] = 0.f;
        if (ok && mode == 1) yo[k] = (float)y[po[k]];
    }
#pragma unroll
    for (int k = 0; k < NLD; ++k) {
        const int idx = threadIdx.x + k * NET_NT;
        if (idx < NRR * NRW) rs[idx / NRW][idx % NRW] = v[k];
    }
    __syncthreads();
    net_hidden<MFMA>(n, i0, j0, W, rs, zs);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NOUT; ++k) {
        if (po[k] < 0) continue;
        const int idx = threadIdx.x + k * NET_NT;
        const int rr = idx / NET_TI, cc = idx - rr * NET_TI;
        const int j = j0 + rr, i = i0 + cc;
        float o = 0.f;
#pragma unroll
        for (int t = 0; t < 7; ++t) o += zs[t][(rr + 1 + c_dj[t]) * NZ + (cc + 1 + c_di[t])];
        const T val = (T)(yo[k] + o);
        y[po[k]] = val;
        if (j == 1 && i <= n - 2 && !fi.bside[0])
            y[nedge_ghost(L, fi.edge[0], fi.slot[0]) + (fi.rev[0] ? n - 2 - i : i)] = val;
        if (i == 1 && j <= n - 2 && !fi.bside[1])
            y[nedge_ghost(L, fi.edge[1], fi.slot[1]) + (fi.rev[1] ? n - 2 - j : j)] = val;
        if (i + j == n - 2 && !fi.bside[2])
            y[nedge_ghost(L, fi.edge[2], fi.slot[2]) + (fi.rev[2] ? n - 2 - j : j)] = val;
    }
}

// Weight gradients of sum_p g(p) out(p) over the face-interior points of
// one tile; thread w < 112 owns dW1[w / 7][w % 7], 112 <= w < 224 owns
// dW2.  With BF16 the inputs and weights are rounded as in the forward.
//   dW2[c][t] = sum_q h_c(q) g(q - d_t)
//   dW1[c][t] = sum_q [a_c(q) > 0] (sum_s W2[c][s] g(q - d_s)) rho(q + d_t)
template <class T, bool BF16>
__global__ __launch_bounds__(NET_NT) void k_net_backward(LevelDev L, const T* __restrict__ rho,
                                                         const T* __restrict__ g,
                                                         const float* __restrict__ W,
                                                         float* __restrict__ partials) {
    __shared__ float rs[NRR][NRW];
    __shared__ float gs[NRR][NRW];
    __shared__ float ws[224];
    const int n = L.n;
    const int face = blockIdx.x / L.n_net_tiles;
    const int2 tl = L.net_tiles[blockIdx.x % L.n_net_tiles];
    const int i0 = tl.x * NET_TI, j0 = tl.y * NET_TJ;
    const int64_t fb = nface_base(L, face);
    for (int idx = threadIdx.x; idx < NRR * NRW; idx += NET_NT) {
        const int r = idx / NRW, c = idx - r * NRW;
        const int j = j0 - 2 + r, i = i0 - 2 + c;
        float v = 0.f, gv = 0.f;
        if (j >= 0 && j < n && i >= 0 && i <= n - 1 - j) {
            const int64_t p = fb + nrow_start(n, j) + i;
            v = (float)rho[p];
            if (j >= 1 && i >= 1 && i + j <= n - 2) gv = (float)g[p];
        }
        rs[r][c] = BF16 ? bf16_round(v) : v;
        gs[r][c] = gv;
    }
    for (int w = threadIdx.x; w < 224; w += NET_NT) ws[w] = BF16 ? bf16_round(W[w]) : W[w];
    __syncthreads();
    const int w = threadIdx.x;
    float acc = 0.f;
    if (w < 224) {
        const bool second = w >= 112;
        const int c = (second ? w - 112 : w) / 7, t = (second ? w - 112 : w) % 7;
        for (int rr = 0; rr < NET_TJ; ++rr) {
            const int j = j0 + rr;
            for (int cc = 0; cc < NET_TI; ++cc) {
                const int i = i0 + cc;
                if (!(j >= 1 && i >= 1 && i + j <= n - 2)) continue;
                const int R = rr + 2, C = cc + 2;
                float a = 0.f;
                for (int s = 0; s < 7; ++s) a += ws[c * 7 + s] * rs[R + c_dj[s]][C + c_di[s]];
                if (second) {
                    const float h = fmaxf(a, 0.f);
                    acc += (BF16 ? bf16_round(h) : h) * gs[R - c_dj[t]][C - c_di[t]];
                } else if (a > 0.f) {
                    float dh = 0.f;
                    for (int s = 0; s < 7; ++s) dh += ws[112 + c * 7 + s] * gs[R - c_dj[s]][C - c_di[s]];
                    acc += dh * rs[R + c_dj[t]][C + c_di[t]];
                }
            }
        }
        partials[(int64_t)blockIdx.x * 224 + w] = acc;
    }
}

// dW[w] += sum over blocks of partials (fixed order, FP64 accumulation).
__global__ __launch_bounds__(256) void k_net_reduce(const float* __restrict__ partials, int nblocks,
                                                    float* __restrict__ dW) {
    const int w = threadIdx.x;
    if (w >= 224) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)partials[(int64_t)b * 224 + w];
    dW[w] += (float)s;
}

// Adam on the FP32 master weights (bias-corrected, step counted from 1).
__global__ __launch_bounds__(256) void k_net_adam(float* __restrict__ W, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ grad,
                                                  float lr, float b1, float b2, float eps, int step) {
    const int w = threadIdx.x;
    if (w >= 224) return;
    const float gr = grad[w];
    const float mw = b1 * m[w] + (1.f - b1) * gr;
    const float vw = b2 * v[w] + (1.f - b2) * gr * gr;
    m[w] = mw;
    v[w] = vw;
    const float mh = mw / (1.f - powf(b1, (float)step));
    const float vh = vw / (1.f - powf(b2, (float)step));
    W[w] -= lr * mh / (sqrtf(vh) + eps);
}

hipError_t launch_net_forward(const hhg_mesh* M, int level, const float* rho, float* y, int mode,
                              bool mfma, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int g = L.F * L.n_net_tiles;
    if (g == 0) return hipSuccess;
    if (mfma) k_net_forward<float, true><<<g, NET_NT, 0, s>>>(L, rho, y, M->net_w, mode);
    else k_net_forward<float, false><<<g, NET_NT, 0, s>>>(L, rho, y, M->net_w, mode);
    return hipGetLastError();
}

hipError_t launch_net_backward(const hhg_mesh* M, int level, const float* rho, const float* g,
                               float* dW, bool bf16, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int nb = L.F * L.n_net_tiles;
    if (nb == 0) return hipSuccess;
    if (bf16) k_net_backward<float, true><<<nb, NET_NT, 0, s>>>(L, rho, g, M->net_w, M->net_partials);
    else k_net_backward<float, false><<<nb, NET_NT, 0, s>>>(L, rho, g, M->net_w, M->net_partials);
    k_net_reduce<<<1, 256, 0, s>>>(M->net_partials, nb, dW);
    return hipGetLastError();
}

hipError_t launch_net_adam(const hhg_mesh* M, const float* grad, float lr, int step, hipStream_t s) {
    k_net_adam<<<1, 256, 0, s>>>(M->net_w, M->net_m, M->net_v, grad, lr, 0.9f, 0.999f, 1e-8f, step);
    return hipGetLastError();
}

}  // namespace hhg
