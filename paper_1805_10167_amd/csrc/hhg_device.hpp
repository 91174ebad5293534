// Device helpers shared by the HIP kernels of the library: field indexing
// of the level layout, wave/block reductions, the loops over face tiles
// and edge/vertex points, and the ghost-copy pushes of a producing kernel
// (the process-local direct copy of the communication layer, sec. 2.4 and
// 3.3 of the paper: the writer of a value also writes its copies, in the
// receiver's order).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hhg_kernels.hpp"

namespace hhg {

constexpr int NT = 256;              // threads per block of the point kernels
constexpr int MAX_FACE_BLOCKS = 8192;
constexpr int MAX_LOW_BLOCKS = 1024;

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int64_t face_base(const LevelDev& L, int f) {
    return L.face_base + (int64_t)f * L.face_stride;
}
__device__ __forceinline__ int64_t edge_main(const LevelDev& L, int e) {
    return L.edge_base + (int64_t)e * L.edge_stride;
}
__device__ __forceinline__ int64_t edge_ghost(const LevelDev& L, int e, int s) {
    return L.edge_base + (int64_t)e * L.edge_stride + L.ghost_off + (int64_t)s * L.ghost_stride;
}
__device__ __forceinline__ int64_t vert_off(const LevelDev& L, int v) {
    return L.vert_base + (int64_t)v * L.vert_stride;
}

// Start of face-local row j: rows hold n - j values padded to 16, so the
// offset is 16 * sum_{m = n-j+1}^{n} ceil(m / 16); with
// S(N) = sum_{m=1}^{N} ceil(m/16) = 8 q (q+1) + t (q+1), N = 16 q + t.
__device__ __forceinline__ int ceil16_sum(int N) {
    const int q = N >> 4, t = N & 15;
    return 8 * q * (q + 1) + t * (q + 1);
}
__device__ __forceinline__ int row_start(int n, int j) {
    return 16 * (ceil16_sum(n) - ceil16_sum(n - j));
}

// Wave index inside the block, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ int face_colour(int rule, int i, int j) {
    switch (rule) {
        case 1: return (i + j) & 1;
        case 2: return i & 1;
        case 3: return j & 1;
        default: return ((i - j) % 3 + 3) % 3;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum (fixed reduction tree); every thread gets lane 0's
// value of the final wave.
template <int NTH>
__device__ __forceinline__ double block_sum(double v, double* sm) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[w] = v;
    __syncthreads();
    if (threadIdx.x < 64) {
        double t = (threadIdx.x < NTH / 64) ? sm[threadIdx.x] : 0.0;
        t = wave_sum(t);
        if (threadIdx.x == 0) sm[NTH / 64] = t;
    }
    __syncthreads();
    return sm[NTH / 64];
}

// Generic loop over face-interior points in 64 x 4 tiles, grid-stride over
// the first GF blocks (the face blocks of the launch: a launch that also has
// edge/vertex blocks passes its face-block count, a face-only launch
// gridDim.x).
#define FACE_TILE_LOOP(L, GF)                                                               \
    const int n = (L).n;                                                                    \
    const int ti_ = threadIdx.x & (TILE_I - 1), tj_ = wave_id();                          \
    const int64_t nitems_ = (int64_t)(L).F * (L).ntiles;                                    \
    for (int64_t it_ = blockIdx.x; it_ < nitems_; it_ += (GF)) {                           \
        const int face = (int)(it_ / (L).ntiles);                                           \
        const int2 tl_ = (L).tiles[it_ % (L).ntiles];                                       \
        const int i = tl_.x * TILE_I + ti_, j = tl_.y * TILE_J + tj_;                       \
        if (!(i >= 1 && j >= 1 && i + j <= n - 2)) continue;                                \
        const FaceInfo& fi = (L).faces[face];                                               \
        const int64_t p = face_base((L), face) + row_start(n, j) + i;                        \
        const int64_t up = row_start(n, j + 1) - row_start(n, j);                             \
        const int64_t dn = row_start(n, j) - row_start(n, j - 1);

#define FACE_TILE_END }

// ------------------------------------------------------------------ pushes
// A kernel that writes an owned value also writes its ghost copies (the
// process-local direct copy of the communication layer; the writer takes
// care of the receiver's order).

// Face-local (i, j) of parameter t along side `side` (0: j = 0, 1: i = 0,
// 2: i + j = n - 1).  Written with selects: as a divergent three-way branch
// the compiler (ROCm 7.2, -O3) dropped the side-2 assignment of j in one
// kernel, leaving j = 0 for those lanes.
__device__ __forceinline__ void side_point0(int side, int t, int n, int& i, int& j) {
    j = side == 0 ? 0 : t;
    i = side == 0 ? t : (side == 1 ? 0 : n - 1 - t);
}

// Copies of edge point k = 1 or n-2 in the first/last ghost-row entry of the
// neighbouring edges of each adjacent face (the entries next to the shared
// vertex).  Both faces' targets are read before either store, so their
// metadata loads are in flight together.
template <class T>
__device__ __forceinline__ void push_corner_ghosts(const LevelDev& L, T* x, const EdgeInfo& ei, int k, T val) {
    const int n = L.n, nf = ei.nf;
    for (int end = 0; end < 2; ++end) {
        if (k != (end == 0 ? 1 : n - 2)) continue;
        int64_t a[2];
        bool ok[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int ss = s < nf ? s : 0, e2 = ei.cg_edge[ss][end];
            ok[s] = s < nf && e2 >= 0;
            a[s] = ok[s] ? edge_ghost(L, e2, ei.cg_slot[ss][end]) + (ei.cg_first[ss][end] ? 0 : n - 2) : 0;
        }
#pragma unroll
        for (int s = 0; s < 2; ++s)
            if (ok[s]) x[a[s]] = val;
    }
}

// Copies of edge point k: face rings, the vertex ghost (k = 1 or n-2) and,
// with `corners`, the first/last ghost-row entry of the neighbouring edges.
template <class T>
__device__ __forceinline__ void push_edge(const LevelDev& L, T* x, const EdgeInfo& ei, int k, T val,
                                          bool corners) {
    const int n = L.n, nf = ei.nf;
    // both faces' targets first (the second clamped to the first when the
    // edge has one face), so their metadata loads are in flight together
    int64_t a[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int ss = s < nf ? s : 0;
        int i, j;
        side_point0(ei.side[ss], ei.rev[ss] ? n - 1 - k : k, n, i, j);
        a[s] = face_base(L, ei.face[ss]) + row_start(n, j) + i;
    }
    x[a[0]] = val;
    if (nf > 1) x[a[1]] = val;
    if (k == 1) x[vert_off(L, ei.a) + 1 + ei.vslot[0]] = val;
    if (k == n - 2) x[vert_off(L, ei.b) + 1 + ei.vslot[1]] = val;
    if (corners) push_corner_ghosts(L, x, ei, k, val);
}

// Copies of a vertex value: edge end slots and face ring corners.
// The targets are read four at a time (indices clamped into the lists), so
// that a group's metadata loads are in flight together.
template <class T>
__device__ __forceinline__ void push_vertex(const LevelDev& L, T* x, const VertexInfo& vi, T val) {
    const int n = L.n, deg = vi.deg, nfc = vi.nfc;
    for (int q0 = 0; q0 < deg; q0 += 4) {
        int64_t a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = q0 + k < deg ? q0 + k : q0;
            a[k] = edge_main(L, vi.edge[q]) + (vi.at_a[q] ? 0 : n - 1);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (q0 + k < deg) x[a[k]] = val;
    }
    for (int c0 = 0; c0 < nfc; c0 += 4) {
        int64_t a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int c = c0 + k < nfc ? c0 + k : c0, cr = vi.fc_corner[c];
            a[k] = face_base(L, vi.fc_face[c]) + row_start(n, cr == 2 ? n - 1 : 0) + (cr == 1 ? n - 1 : 0);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < nfc) x[a[k]] = val;
    }
}

// Where a face's near-edge rows are copied: for each side the start of the
// edge's ghost row that holds them (-1 on a Dirichlet side) and whether the
// edge runs against the side.  Read once per face in wave-uniform code, so
// the pushes of lane-divergent code use registers: a per-lane load of the
// face record there would be waited on together with every load in flight.
struct FaceGhosts {
    int64_t g[3];
    int rev[3];
};
__device__ __forceinline__ FaceGhosts face_ghosts(const LevelDev& L, const FaceInfo& fi) {
    FaceGhosts t;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        t.g[s] = fi.bside[s] ? -1 : edge_ghost(L, fi.edge[s], fi.slot[s]);
        t.rev[s] = fi.rev[s];
    }
    return t;
}

// Copies of face point (i, j) in the ghost rows of the face's edges, from
// the face record (point loops, where most lanes never get here) ...
template <class T>
__device__ __forceinline__ void push_face_near(const LevelDev& L, T* x, const FaceInfo& fi, int i, int j,
                                               T val) {
    const int n = L.n;
    if (j == 1 && i <= n - 2 && !fi.bside[0])
        x[edge_ghost(L, fi.edge[0], fi.slot[0]) + (fi.rev[0] ? n - 2 - i : i)] = val;
    if (i == 1 && j <= n - 2 && !fi.bside[1])
        x[edge_ghost(L, fi.edge[1], fi.slot[1]) + (fi.rev[1] ? n - 2 - j : j)] = val;
    if (i + j == n - 2 && !fi.bside[2])
        x[edge_ghost(L, fi.edge[2], fi.slot[2]) + (fi.rev[2] ? n - 2 - j : j)] = val;
}

// ... or from the registers of FaceGhosts (tile kernels, which read it once
// per tile)
template <class T>
__device__ __forceinline__ void push_face_near(const FaceGhosts& gh, int n, T* x, int i, int j, T val) {
    if (j == 1 && i <= n - 2 && gh.g[0] >= 0) x[gh.g[0] + (gh.rev[0] ? n - 2 - i : i)] = val;
    if (i == 1 && j <= n - 2 && gh.g[1] >= 0) x[gh.g[1] + (gh.rev[1] ? n - 2 - j : j)] = val;
    if (i + j == n - 2 && gh.g[2] >= 0) x[gh.g[2] + (gh.rev[2] ? n - 2 - j : j)] = val;
}

// Face-point loop over the 64 x 4 tiles of every face, grid-stride over the
// first gf blocks; yields all points of the triangle.
#define FACE_ALL_LOOP(L, GF)                                                                \
    const int n = (L).n;                                                                    \
    const int ti_ = threadIdx.x & (TILE_I - 1), tj_ = wave_id();                          \
    const int64_t nitems_ = (int64_t)(L).F * (L).ntiles;                                    \
    for (int64_t it_ = blockIdx.x; it_ < nitems_; it_ += (GF)) {                           \
        const int face = (int)(it_ / (L).ntiles);                                           \
        const int2 tl_ = (L).tiles[it_ % (L).ntiles];                                       \
        const int i = tl_.x * TILE_I + ti_, j = tl_.y * TILE_J + tj_;                       \
        if (j >= n || i > n - 1 - j) continue;                                              \
        const bool interior = i >= 1 && j >= 1 && i + j <= n - 2;                           \
        const FaceInfo& fi = (L).faces[face];                                               \
        const int64_t p = face_base((L), face) + row_start(n, j) + i;

// Edge points (every edge, k = 1..n-2) then vertices, grid-stride over the
// blocks [B0, gridDim.x).
#define LOW_LOOP(L, B0)                                                                      \
    const int nl_ = (L).n;                                                                   \
    const int64_t ne_ = (int64_t)(L).E * (nl_ - 2);                                          \
    const int64_t stride_ = (int64_t)(gridDim.x - (B0)) * NT;                                \
    for (int64_t t = (int64_t)(blockIdx.x - (B0)) * NT + threadIdx.x; t < ne_ + (L).V; t += stride_)

}  // namespace hhg
