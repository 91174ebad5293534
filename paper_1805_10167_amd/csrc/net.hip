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

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "hhg_kernels.hpp"

namespace hhg {

constexpr int NET_NT = 256;
constexpr int NWV = NET_NT / 64;                      // waves per block
constexpr int NZ = NET_TI + 2, NZR = NET_TJ + 2;      // hidden/z region (tile + 1)
constexpr int NRW = NET_TI + 4, NRR = NET_TJ + 4;     // rho region (tile + 2)
constexpr int NXW = NET_TI + 6;                       // x columns of a fused-step strip (tile + 3)
// LDS rows of every region are 64 values: one per lane of a wave, so a wave
// works on whole rows with wave-uniform row offsets.  The hidden row of 60
// pixels is four MFMA groups of 16 (4 slots unused).
constexpr int RW = 64;
static_assert(NXW == RW, "x row of a strip = one wave");
// The z planes (one per tap) are NZR rows of RW values, RW * NZR = 0 mod 64
// dwords; padded to 8 mod 64, the 16-byte stores of the seven tap lanes of an
// MFMA result land in disjoint banks (unpadded they all hit one bank).
constexpr int ZPS = NZR * RW + 8;
static_assert((NZR * RW) % 64 == 0 && ZPS % 4 == 0, "z plane padding assumes rows of whole banks");

__constant__ int c_di[7] = {0, 1, -1, 0, 0, 1, -1};
__constant__ int c_dj[7] = {0, 0, 0, 1, -1, -1, 1};

typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float4v __attribute__((ext_vector_type(4)));
typedef float float2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef unsigned uint2v __attribute__((ext_vector_type(2)));

// Round to nearest even BF16 (the hardware conversion), packed in pairs so
// that each pair is one v_cvt_pk_bf16_f32.
__device__ __forceinline__ short4v to_bf16x4(float a, float b, float c, float d) {
    const float2v f0 = {a, b}, f1 = {c, d};
    const uint2v u = {__builtin_bit_cast(unsigned, __builtin_convertvector(f0, bf16x2)),
                      __builtin_bit_cast(unsigned, __builtin_convertvector(f1, bf16x2))};
    return __builtin_bit_cast(short4v, u);
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

// z_t over the hidden region (tile grown by 1): MFMA (BF16) or FP32.
// rs[r][c]: rho at (i0 - 2 + c, j0 - 2 + r); zs[t][r * RW + c]: z_t at hidden
// pixel (i0 - 1 + c, j0 - 1 + r).  A wave takes whole hidden rows; in an
// MFMA group lane l16 is pixel 16 q + l16 of the row and lane group q4
// holds taps (layer 1) or channels (layer 2) 4 q4 .. 4 q4 + 3.
template <bool MFMA>
__device__ __forceinline__ void net_hidden(int n, int i0, int j0, const float* __restrict__ W,
                                           float (*rs)[RW], float (*zs)[ZPS]) {
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (MFMA) {
        const int q4 = lane >> 4, l16 = lane & 15;
        float a1[4], a2[4];
        int toff[4];
        bool tval[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = 4 * q4 + e;
            a1[e] = t < 7 ? W[l16 * 7 + t] : 0.f;            // A[c = l16][k = t]
            a2[e] = l16 < 7 ? W[112 + t * 7 + l16] : 0.f;     // B[k = c = t][n = tap l16]
            tval[e] = t < 7;
            toff[e] = t < 7 ? (1 + c_dj[t]) * RW + (1 + c_di[t]) : RW + 1;
        }
        const short4v w1op = to_bf16x4(a1[0], a1[1], a1[2], a1[3]);
        const short4v w2op = to_bf16x4(a2[0], a2[1], a2[2], a2[3]);
        for (int row = wv; row < NZR; row += NWV) {
            const int j = j0 - 1 + row;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int cc = 16 * q + l16;
                const float* base = &rs[row][cc];
                // the hidden layer exists on interior pixels only: zero taps there
                // give a = 0 exactly, so ReLU needs no mask afterwards
                const int i = i0 - 1 + cc;
                const bool inner = cc < NZ && j >= 1 && i >= 1 && i + j <= n - 2;
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float xv = base[toff[e]];
                    v[e] = (tval[e] && inner) ? xv : 0.f;
                }
                float4v acc = {0.f, 0.f, 0.f, 0.f};
                acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w1op, to_bf16x4(v[0], v[1], v[2], v[3]),
                                                                acc, 0, 0, 0);
                // lane holds a for channels 4 q4 + e of pixel cc
                const short4v hop = to_bf16x4(fmaxf(acc[0], 0.f), fmaxf(acc[1], 0.f), fmaxf(acc[2], 0.f),
                                              fmaxf(acc[3], 0.f));
                float4v z = {0.f, 0.f, 0.f, 0.f};
                z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hop, w2op, z, 0, 0, 0);
                // lane holds z for tap l16 of pixels 16 q + 4 q4 + e
                if (l16 < 7) *reinterpret_cast<float4v*>(&zs[l16][row * RW + 16 * q + 4 * q4]) = z;
            }
        }
    } else {
        for (int row = wv; row < NZR; row += NWV) {
            const int cc = lane, j = j0 - 1 + row, i = i0 - 1 + cc;
            const bool inner = cc < NZ && j >= 1 && i >= 1 && i + j <= n - 2;
            float z[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (cc < NZ) {
                float rt[7];
                for (int t = 0; t < 7; ++t) rt[t] = rs[row + 1 + c_dj[t]][cc + 1 + c_di[t]];
                for (int c = 0; c < 16; ++c) {
                    float a = 0.f;
                    for (int t = 0; t < 7; ++t) a += W[c * 7 + t] * rt[t];
                    const float h = inner ? fmaxf(a, 0.f) : 0.f;
                    for (int t = 0; t < 7; ++t) z[t] += W[112 + c * 7 + t] * h;
                }
            }
            for (int t = 0; t < 7; ++t) zs[t][row * RW + cc] = z[t];
        }
    }
}

// Per-tile constants of the face: FP32 cotangents (and the constant-k
// centre weight), and for each side the start of the ghost row that holds
// copies of the face's near-side row (-1 on a Dirichlet side) with its
// direction.  Loaded once per tile, outside divergent code.
struct NetFace {
    float c0, c1, c2, wc;
    int64_t g[3];
    int rev[3];
};
__device__ __forceinline__ NetFace net_face(const LevelDev& L, const FaceInfo& fi) {
    NetFace t;
    t.c0 = (float)fi.cot[0];
    t.c1 = (float)fi.cot[1];
    t.c2 = (float)fi.cot[2];
    t.wc = (float)(2.0 * (fi.cot[0] + fi.cot[1] + fi.cot[2]));
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        t.g[s] = fi.bside[s] ? -1 : nedge_ghost(L, fi.edge[s], fi.slot[s]);
        t.rev[s] = fi.rev[s];
    }
    return t;
}

// out at output pixel (i0 + c, j0 + r) from the z planes.
__device__ __forceinline__ float net_out(float (*zs)[ZPS], int r, int c) {
    float o = 0.f;
#pragma unroll
    for (int t = 0; t < 7; ++t) o += zs[t][(r + 1 + c_dj[t]) * RW + c + 1 + c_di[t]];
    return o;
}

// out = N(rho) on face-interior points (mode 0: write out, whose other
// entries the caller has zeroed; mode 1: u += N(rho) in place).  Both write
// the near-edge-row copies of what they change.  Waves take whole rows of
// each region; a thread issues its global loads (rho, then the outputs' old
// values) before any of them is used.
constexpr int NLR = (NRR + NWV - 1) / NWV;      // rho rows per wave
constexpr int NOR = (NET_TJ + NWV - 1) / NWV;   // output rows per wave

template <class T, bool MFMA>
__global__ __launch_bounds__(NET_NT) void k_net_forward(LevelDev L, const T* __restrict__ rho,
                                                        T* __restrict__ y, const float* __restrict__ W,
                                                        int mode) {
    __shared__ float rs[NRR + 1][RW];
    __shared__ __align__(16) float zs[7][ZPS];
    const int n = L.n;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ntile = L.F * L.n_net_tiles;
    for (int tile = blockIdx.x; tile < ntile; tile += gridDim.x) {
    __syncthreads();                                   // LDS of the previous tile is free
    const int face = tile / L.n_net_tiles;
    const int2 tl = L.net_tiles[tile % L.n_net_tiles];
    const int i0 = tl.x * NET_TI, j0 = tl.y * NET_TJ;
    const NetFace nf = net_face(L, L.faces[face]);
    const int64_t fb = nface_base(L, face);
    float v[NLR];
#pragma unroll
    for (int k = 0; k < NLR; ++k) {
        const int r = wv + NWV * k, j = j0 - 2 + r, i = i0 - 2 + lane;
        const bool row_ok = r < NRR && j >= 0 && j < n;
        const bool in = row_ok && lane < NRW && i >= 0 && i <= n - 1 - j;
        v[k] = in ? (float)rho[fb + nrow_start(n, row_ok ? j : 0) + i] : 0.f;
    }
    float yo[NOR];
#pragma unroll
    for (int k = 0; k < NOR; ++k) {
        const int r = wv + NWV * k, j = j0 + r, i = i0 + lane;
        const bool row_ok = r < NET_TJ && j >= 1;
        const bool ok = row_ok && lane < NET_TI && i >= 1 && i + j <= n - 2;
        yo[k] = (ok && mode == 1) ? (float)y[fb + nrow_start(n, row_ok ? j : 0) + i] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < NLR; ++k) {
        const int r = wv + NWV * k;
        if (r < NRR) rs[r][lane] = v[k];
    }
    if (wv == 0) rs[NRR][lane] = 0.f;
    __syncthreads();
    net_hidden<MFMA>(n, i0, j0, W, rs, zs);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NOR; ++k) {
        const int r = wv + NWV * k, j = j0 + r, i = i0 + lane;
        if (!(r < NET_TJ && lane < NET_TI && j >= 1 && i >= 1 && i + j <= n - 2)) continue;
        const T val = (T)(yo[k] + net_out(zs, r, lane));
        const int64_t p = fb + nrow_start(n, j) + i;
        y[p] = val;
        if (j == 1 && i <= n - 2 && nf.g[0] >= 0) y[nf.g[0] + (nf.rev[0] ? n - 2 - i : i)] = val;
        if (i == 1 && j <= n - 2 && nf.g[1] >= 0) y[nf.g[1] + (nf.rev[1] ? n - 2 - j : j)] = val;
        if (i + j == n - 2 && nf.g[2] >= 0) y[nf.g[2] + (nf.rev[2] ? n - 2 - j : j)] = val;
    }
    }
}

// Face step of the learned sweep, from x to y:
//   rho = D^-1 (f - A x) on face-interior points (ring points take rho_ring,
//   written beforehand by the edge/vertex Jacobi pass; 0 outside the
//   triangle), y = x + N(rho) on face-interior points, with their near-row
//   copies in y's ghost rows.
// One wave per strip piece: output columns i0 <= i < i0 + NET_TI and rows
// j0 <= j < j0 + net_sr of one face, lane c standing for column
// i = i0 - 3 + c.  The wave walks up the rows; at row s it
//   - takes x of row s + 3 and f (or rho_ring) of row s + 2 from register
//     rings loaded NS_U - 4 rows ahead,
//   - forms rho of row s + 2 from the x rows s + 1 .. s + 3 held in
//     registers (east and west neighbours by whole-wave lane shifts),
//   - forms the hidden layer and z of row s + 1 from rho rows s .. s + 2,
//   - forms out of row s from z rows s - 1 .. s + 1 and writes y = x + out.
// rho and z live in rings of three rows in the wave's own LDS: a wave never
// waits for another, and every row of every stage is formed once.
// Extra blocks copy what the face step leaves unchanged from x to y: edge
// and vertex blocks, face rings and the ghost-row corner entries, so y is a
// complete field.  Reading x and writing y keeps the rows that neighbouring
// pieces read free of updated values.
constexpr int NS_COPY_BLOCKS = 32;
constexpr int NS_U = 6;                // register ring rows (a multiple of 3); loads NS_U - 4 rows ahead
static_assert(NS_U % 3 == 0 && (NS_U == 6 || NS_U == 9), "the step loop is written for 6 or 9 ring rows");
constexpr int NS_RW = 72;              // rho ring row: pixel p at p + 4
constexpr int NS_ZP = 3 * RW + 4;      // z ring of one tap: three rows of RW pixels, planes 4 mod 64 banks apart
struct NetRing {
    float rho[3][NS_RW];
    float z[7][NS_ZP];
};
static_assert((3 * NS_RW) % 4 == 0 && NS_ZP % 4 == 0 && RW % 4 == 0, "16-byte aligned z stores");

__host__ __device__ constexpr int tap_di(int t) { return (t == 1 || t == 5) ? 1 : ((t == 2 || t == 6) ? -1 : 0); }
__host__ __device__ constexpr int tap_dj(int t) { return (t == 3 || t == 6) ? 1 : ((t == 4 || t == 5) ? -1 : 0); }
// Layer-1 contraction index k -> tap (-1: unused): C E N S | W - NW SE, so
// that k and k + 4 have the same row offset k_dj(k % 4).
__host__ __device__ constexpr int k_tap(int k) {
    return k == 0 ? 0 : k == 1 ? 1 : k == 2 ? 3 : k == 3 ? 4 : k == 4 ? 2 : k == 6 ? 6 : k == 7 ? 5 : -1;
}
__host__ __device__ constexpr int k_dj(int e) { return e == 2 ? 1 : (e == 3 ? -1 : 0); }
static_assert(tap_dj(k_tap(0)) == k_dj(0) && tap_dj(k_tap(4)) == k_dj(0) && tap_dj(k_tap(1)) == k_dj(1) &&
                  tap_dj(k_tap(2)) == k_dj(2) && tap_dj(k_tap(6)) == k_dj(2) && tap_dj(k_tap(3)) == k_dj(3) &&
                  tap_dj(k_tap(7)) == k_dj(3),
              "one row offset per slot");

// Value held by lane c + 1 (lane_next) or c - 1 (lane_prev) of the wave, 0
// where that lane does not exist.
__device__ __forceinline__ float lane_next(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}

// LDS written by some lanes of a wave and read by others of the same wave:
// the DS instructions of one wave execute in order, so only the compiler has
// to keep them in program order.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// rho at the lane's point of the middle row from x (and k) of the rows
// below (S), at (0) and above (N) it.
template <bool VARK>
__device__ __forceinline__ float net_rho_rows(const NetFace& nf, float xS, float x0, float xN, float kS_,
                                              float k0_, float kN_, float fv) {
    const float uE = lane_next(x0), uW = lane_prev(x0), uN = xN, uS = xS;
    const float uSE = lane_next(xS), uNW = lane_prev(xN), u0 = x0;
    const float c0 = nf.c0, c1 = nf.c1, c2 = nf.c2;
    float we, ww, wn, ws, wse, wnw, wc;
    if (!VARK) {
        wc = nf.wc;
        we = ww = -c2;
        wn = ws = -c1;
        wse = wnw = -c0;
    } else {
        const float k0 = k0_, kE = lane_next(k0_), kW = lane_prev(k0_), kN = kN_;
        const float kS = kS_, kSE = lane_next(kS_), kNW = lane_prev(kN_);
        const float third = 1.0f / 3.0f, h = 0.5f;
        const float t1 = (k0 + kE + kN) * third, t2 = (kSE + kE + k0) * third;
        const float t3 = (kW + k0 + kNW) * third, t4 = (kS + k0 + kW) * third;
        const float t5 = (k0 + kN + kNW) * third, t6 = (kS + kSE + k0) * third;
        we = -h * c2 * (t1 + t2);
        ww = -h * c2 * (t3 + t4);
        wn = -h * c1 * (t1 + t5);
        ws = -h * c1 * (t6 + t4);
        wse = -h * c0 * (t6 + t2);
        wnw = -h * c0 * (t3 + t5);
        wc = -(we + ww + wn + ws + wse + wnw);
    }
    const float ax = wc * u0 + we * uE + ww * uW + wn * uN + ws * uS + wse * uSE + wnw * uNW;
    // FP32 Jacobi scaling by the hardware reciprocal (1 ulp): the learned
    // step's rounding is set by its BF16 operands, far coarser
    return (fv - ax) * __builtin_amdgcn_rcpf(wc);
}

template <bool VARK, bool MFMA>
__global__ __launch_bounds__(NET_NT) void k_net_step(LevelDev L, const float* __restrict__ x,
                                                     float* __restrict__ y, const float* __restrict__ f,
                                                     const float* __restrict__ kap,
                                                     const float* __restrict__ rho_ring,
                                                     const float* __restrict__ W, int nblk) {
    __shared__ __align__(16) NetRing rings[NWV];
    const int n = L.n;
    if ((int)blockIdx.x >= nblk) {
        // copies x -> y: edge main (k = 0..n-1), vertex blocks, face rings,
        // ghost-row corner entries
        const int cb = blockIdx.x - nblk, ncb = gridDim.x - nblk;
        const int64_t ne = (int64_t)L.E * n, nv = (int64_t)L.V * L.vert_stride;
        const int64_t nr = (int64_t)L.F * 3 * (n - 1), ng = (int64_t)L.E * 4;
        for (int64_t t = (int64_t)cb * NET_NT + threadIdx.x; t < ne + nv + nr + ng; t += (int64_t)ncb * NET_NT) {
            int64_t off;
            if (t < ne) {
                off = L.edge_base + (t / n) * L.edge_stride + (t % n);
            } else if (t < ne + nv) {
                off = L.vert_base + (t - ne);
            } else if (t < ne + nv + nr) {
                const int64_t q = t - ne - nv;
                const int face = (int)(q / (3 * (n - 1))), m = (int)(q % (3 * (n - 1)));
                const int sd = m / (n - 1), tt = m % (n - 1);
                int i, j;
                if (sd == 0) { i = tt; j = 0; }
                else if (sd == 1) { i = n - 1 - tt; j = tt; }
                else { i = 0; j = n - 1 - tt; }
                off = nface_base(L, face) + nrow_start(n, j) + i;
            } else {
                const int64_t q = t - ne - nv - nr;
                const int e = (int)(q >> 2), sl = (int)((q >> 1) & 1), end = (int)(q & 1);
                if (L.edges[e].boundary) continue;
                off = nedge_ghost(L, e, sl) + (end ? n - 2 : 0);
            }
            y[off] = x[off];
        }
        return;
    }
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // consecutive logical blocks (neighbouring pieces, which share halo rows)
    // on one XCD: hardware block b runs on XCD b mod 8
    const int b = blockIdx.x, lb = (b & 7) * (nblk >> 3) + (b >> 3);
    const int task = lb * NWV + wv;
    if (task >= L.F * L.n_net_strips) return;          // the whole wave
    NetRing& R = rings[wv];
    const int face = task / L.n_net_strips;
    const int2 st = L.net_strips[task % L.n_net_strips];
    const int i0 = st.x * NET_TI, j0 = st.y * L.net_sr;
    const int s_end = min(j0 + L.net_sr, n - 1 - max(i0, 1));   // last output row + 1
    const NetFace nf = net_face(L, L.faces[face]);
    const int64_t fb = nface_base(L, face);
    const int ic = i0 - 3 + lane;
    const int q4 = lane >> 4, l16 = lane & 15;
    if (lane < 24) R.rho[lane >> 3][(lane & 7) < 4 ? (lane & 7) : NS_RW - 8 + (lane & 7)] = 0.f;

    // Loads from addresses clamped into the face's triangle are always
    // issued, so no register ever waits on a load it does not need: x (and
    // k) outside the triangle reach only rho of non-interior points, which
    // is replaced, and f is zeroed where it is consumed.
    auto row_addr = [&](int j) {
        const int jj = min(max(j, 0), n - 1);
        return fb + nrow_start(n, jj) + min(max(ic, 0), n - 1 - jj);
    };
    auto load_x = [&](int j, float& xv, float& kv) {
        const int64_t p = row_addr(j);
        xv = x[p];
        if (VARK) kv = kap[p];
    };
    auto load_f = [&](int j) {
        const float* src = (j >= 1 && ic >= 1 && ic + j <= n - 2) ? f : rho_ring;
        return src[row_addr(j)];
    };

    // Weights as MFMA operands.  Layer 1 contracts over k = 4 q4 + e with
    // the taps ordered C E N S | W - NW SE (k_tap), so that slot e of every
    // lane reads rho of one row offset: lane bases differ only in the column
    // and the row of a ring phase is an instruction offset.  Lanes of unused
    // k (weight 0) read the q4 = 0 tap of their slot.
    short4v w1op = {0, 0, 0, 0}, w2op = {0, 0, 0, 0};
    int tbase[4];
    if (MFMA) {
        float a1[4], a2[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t = k_tap(4 * q4 + e), tt = t >= 0 ? t : k_tap(e);
            a1[e] = t >= 0 ? W[l16 * 7 + t] : 0.f;            // A[c = l16][k]
            a2[e] = l16 < 7 ? W[112 + (4 * q4 + e) * 7 + l16] : 0.f;   // B[c = 4 q4 + e][tap l16]
            tbase[e] = 4 + l16 + tap_di(tt);
        }
        w1op = to_bf16x4(a1[0], a1[1], a1[2], a1[3]);
        w2op = to_bf16x4(a2[0], a2[1], a2[2], a2[3]);
    }
    const float* rho_flat = &R.rho[0][0];
    float* z_flat = &R.z[0][0];

    // Register rings of NS_U rows: x (k) of row r in xr[(r - s0) % NS_U], f of
    // row r in fr[(r - s0) % NS_U].  At step s the window is x rows s .. s + 3
    // and f row s + 2; x row s + NS_U - 1 and f row s + NS_U - 2 are loaded
    // into the slots that just fell out of use, NS_U - 4 steps ahead.  The
    // loop is unrolled NS_U times so that every slot stays one register, and
    // runs whole rounds (steps past the piece's last row skip their work):
    // a loop exit between steps would make the compiler copy ring registers
    // whose loads are still in flight.
    const int s0 = j0 - 4;
    float xr[NS_U], kr[NS_U], fr[NS_U];
#pragma unroll
    for (int q = 1; q < NS_U - 1; ++q) load_x(s0 + q, xr[q], kr[q]);
    xr[0] = kr[0] = xr[NS_U - 1] = kr[NS_U - 1] = 0.f;
#pragma unroll
    for (int q = 0; q < NS_U; ++q) fr[q] = 0.f;
#pragma unroll
    for (int q = 2; q < NS_U - 2; ++q) fr[q] = load_f(s0 + q);

    auto step = [&](auto phase, int s) {
        constexpr int P = decltype(phase)::value;
        load_x(s + NS_U - 1, xr[(P + NS_U - 1) % NS_U], kr[(P + NS_U - 1) % NS_U]);
        fr[(P + NS_U - 2) % NS_U] = load_f(s + NS_U - 2);
        if (s >= s_end) return;
        const float X0 = xr[P], X1 = xr[(P + 1) % NS_U], X2 = xr[(P + 2) % NS_U], X3 = xr[(P + 3) % NS_U];
        const float K1 = kr[(P + 1) % NS_U], K2 = kr[(P + 2) % NS_U], K3 = kr[(P + 3) % NS_U];
        constexpr int PH = P % 3;   // ring row of row s in the LDS rings (NS_U is a multiple of 3)
        {   // rho of row s + 2
            const int j = s + 2;
            const bool in = j >= 0 && j < n && ic >= 0 && ic <= n - 1 - j;
            const float F2 = in ? fr[(P + 2) % NS_U] : 0.f;
            const float r = net_rho_rows<VARK>(nf, X1, X2, X3, K1, K2, K3, F2);
            const bool interior = j >= 1 && ic >= 1 && ic + j <= n - 2;
            R.rho[(PH + 2) % 3][lane + 4] = interior ? r : F2;
        }
        wave_lds_order();
        if (s >= j0 - 2) {   // hidden layer and z of row s + 1
            const int j = s + 1;
            float* zrow = z_flat + ((PH + 1) % 3) * RW;
            if (MFMA) {
                float* zdst = zrow + l16 * NS_ZP + 4 * q4;
                if (j >= 1 && j <= n - 3) {
                    const unsigned lim = (unsigned)(n - 3 - j);
                    float v[4][4];
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            v[q][e] = rho_flat[tbase[e] + ((PH + 1 + k_dj(e) + 3) % 3) * NS_RW + 16 * q];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        float4v acc = {0.f, 0.f, 0.f, 0.f};
                        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                            w1op, to_bf16x4(v[q][0], v[q][1], v[q][2], v[q][3]), acc, 0, 0, 0);
                        // lane holds a for channels 4 q4 + e of pixel 16 q + l16; the
                        // hidden layer exists on interior pixels only
                        const float cap = (unsigned)(i0 - 4 + l16 + 16 * q) <= lim ? __builtin_inff() : 0.f;
                        const short4v hop = to_bf16x4(__builtin_amdgcn_fmed3f(acc[0], 0.f, cap),
                                                      __builtin_amdgcn_fmed3f(acc[1], 0.f, cap),
                                                      __builtin_amdgcn_fmed3f(acc[2], 0.f, cap),
                                                      __builtin_amdgcn_fmed3f(acc[3], 0.f, cap));
                        float4v z = {0.f, 0.f, 0.f, 0.f};
                        z = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hop, w2op, z, 0, 0, 0);
                        // lane holds z for tap l16 of pixels 16 q + 4 q4 + e
                        if (l16 < 7) *reinterpret_cast<float4v*>(zdst + 16 * q) = z;
                    }
                } else {
                    const float4v zero = {0.f, 0.f, 0.f, 0.f};
                    if (l16 < 7) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) *reinterpret_cast<float4v*>(zdst + 16 * q) = zero;
                    }
                }
            } else {
                float z[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (j >= 1 && ic >= 1 && ic + j <= n - 2) {
                    float rt[7];
#pragma unroll
                    for (int t = 0; t < 7; ++t)
                        rt[t] = rho_flat[((PH + 1 + tap_dj(t) + 3) % 3) * NS_RW + lane + 4 + tap_di(t)];
                    for (int c = 0; c < 16; ++c) {
                        float a = 0.f;
#pragma unroll
                        for (int t = 0; t < 7; ++t) a += W[c * 7 + t] * rt[t];
                        const float h = fmaxf(a, 0.f);
#pragma unroll
                        for (int t = 0; t < 7; ++t) z[t] += W[112 + c * 7 + t] * h;
                    }
                }
#pragma unroll
                for (int t = 0; t < 7; ++t) zrow[t * NS_ZP + lane] = z[t];
            }
            wave_lds_order();
        }
        if (s >= j0 && s >= 1 && s <= n - 3) {
            // out of row s (a row with interior points) from z rows s - 1 .. s + 1;
            // every lane forms it (its z reads stay inside the wave's rings),
            // the interior ones store it
            const float* zb = z_flat + lane;
            float o = 0.f;
#pragma unroll
            for (int t = 0; t < 7; ++t) o += zb[t * NS_ZP + ((PH + tap_dj(t) + 3) % 3) * RW + tap_di(t)];
            const float val = X0 + o;
            const bool ok = lane >= 3 && lane < 3 + NET_TI && (unsigned)(ic - 1) < (unsigned)(n - 2 - s);
            if (ok) y[fb + nrow_start(n, s) + ic] = val;
            // copies in the ghost rows of the face's edges (rows j = 1, i = 1,
            // i + j = n - 2), each behind a test that is uniform over the wave
            if (s == 1 && nf.g[0] >= 0) {
                if (ok) y[nf.g[0] + (nf.rev[0] ? n - 2 - ic : ic)] = val;
            }
            if (i0 == 0 && nf.g[1] >= 0) {
                if (lane == 4) y[nf.g[1] + (nf.rev[1] ? n - 2 - s : s)] = val;   // i = 1
            }
            const int ld = n - 2 - s - i0 + 3;           // lane of i = n - 2 - s
            if (ld >= 3 && ld < 3 + NET_TI && nf.g[2] >= 0) {
                if (lane == ld) y[nf.g[2] + (nf.rev[2] ? n - 2 - s : s)] = val;
            }
        }
    };
    const int rounds = (s_end - s0 + NS_U - 1) / NS_U;
    for (int k = 0; k < rounds; ++k) {
        const int s = s0 + k * NS_U;
        step(std::integral_constant<int, 0>(), s);
        step(std::integral_constant<int, 1>(), s + 1);
        step(std::integral_constant<int, 2>(), s + 2);
        step(std::integral_constant<int, 3>(), s + 3);
        step(std::integral_constant<int, 4>(), s + 4);
        step(std::integral_constant<int, 5>(), s + 5);
        if (NS_U > 6) {
            step(std::integral_constant<int, 6 % NS_U>(), s + 6);
            step(std::integral_constant<int, 7 % NS_U>(), s + 7);
            step(std::integral_constant<int, 8 % NS_U>(), s + 8);
        }
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

hipError_t launch_net_step(const hhg_mesh* M, int level, int op, const float* x, float* y, const float* f,
                           const float* rho_ring, bool mfma, hipStream_t s) {
    const LevelDev L = M->dev(level);
    const int nt = L.F * L.n_net_strips;
    const int nblk = (int)pad_up((nt + NWV - 1) / NWV, 8);   // whole XCD rounds
    const int g = nblk + NS_COPY_BLOCKS;
    const float* kap = M->kap32[level];
    if (op == OP_DIFFUSION) {
        if (mfma) k_net_step<true, true><<<g, NET_NT, 0, s>>>(L, x, y, f, kap, rho_ring, M->net_w, nblk);
        else k_net_step<true, false><<<g, NET_NT, 0, s>>>(L, x, y, f, kap, rho_ring, M->net_w, nblk);
    } else {
        if (mfma) k_net_step<false, true><<<g, NET_NT, 0, s>>>(L, x, y, f, kap, rho_ring, M->net_w, nblk);
        else k_net_step<false, false><<<g, NET_NT, 0, s>>>(L, x, y, f, kap, rho_ring, M->net_w, nblk);
    }
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
