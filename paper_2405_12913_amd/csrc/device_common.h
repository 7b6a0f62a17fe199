// Device helpers shared by the HIP kernels of the HRT library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "hrt_internal.h"

namespace hrt {

template <typename T>
using c2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
template <typename T>
using v4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;

template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
    return c2<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__host__ __device__ inline int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

// Cell index and fraction of particle i along one axis: u = i_lattice * 2^lratio + s / cell
// (2^lratio mesh cells per lattice spacing). The integer part of t = s / cell is split off
// first so the fraction keeps the precision of the displacement rather than of the absolute
// coordinate. The fraction is the hardware fract of t: t - floor(t), exact, except where t
// lies so little below an integer that t - floor(t) rounds to 1, and there the largest value
// below 1 (the particle keeps its cell floor(t) and puts all but 2^-24 (FP32) of its weight
// on the upper node, where it lies to that precision). So the fraction is always in [0, 1)
// and the CIC weights f and 1 - f are never negative (the paint's unsigned fixed-point sums
// rely on it). Contraction is off: t is the rounded product, as in every other use.
__device__ __forceinline__ float fract_of(float t) { return __builtin_amdgcn_fractf(t); }
__device__ __forceinline__ double fract_of(double t) { return __builtin_amdgcn_fract(t); }

template <typename T>
__device__ __forceinline__ void axis_cell(T s, int lattice, int lratio, T inv_cell, int nmask,
                                          int &c, T &f) {
#pragma clang fp contract(off)
    const T t = s * inv_cell;
    f = fract_of(t);
    c = ((lattice << lratio) + (int)floor(t)) & nmask;
}

__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Fourth-order central difference of phi along one axis from its values at -2, -1, +1, +2
// nodes, divided by the cell (inv12cell = 1 / (12 cell)). No contraction: every kernel
// that forms G (whole mesh, lens planes only, or one tile in LDS) gets the same bits.
template <typename T>
__device__ __forceinline__ T fd4(T m2, T m1, T p1, T p2, T inv12cell) {
#pragma clang fp contract(off)
    return (T(8) * (p1 - m1) - (p2 - m2)) * inv12cell;
}

// One particle's CIC readout of G from the 8 corner values g[k] (corner k is offset
// (k & 1, (k >> 1) & 1, k >> 2) from the particle's cell, f its fractions), then the kick
// p += K G and the drift s += D p. Explicit FMAs in a fixed order, so the kick-drift
// kernels of both particle orders move a particle to the same bits.
template <typename T>
__device__ __forceinline__ void cic_kick_drift(const T f[3], const v4<T> g[8], T K, T D, T s[3],
                                               T p[3]) {
#pragma clang fp contract(off)
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const T wz = (k >> 2) ? f[2] : T(1) - f[2];
        const T wyz = wz * (((k >> 1) & 1) ? f[1] : T(1) - f[1]);
        const T w = wyz * ((k & 1) ? f[0] : T(1) - f[0]);
        gx = fmadd(w, g[k].x, gx);
        gy = fmadd(w, g[k].y, gy);
        gz = fmadd(w, g[k].z, gz);
    }
    const T gg[3] = {gx, gy, gz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p[d] = fmadd(K, gg[d], p[d]);
        s[d] = fmadd(D, p[d], s[d]);
    }
}

// Cell and fraction of a ray on a lens plane along one axis: u = (obs + chi theta) / cell
// in FP64, fraction u - floor(u) formed without contraction, so it lies in [0, 1).
__device__ __forceinline__ void plane_cell(double obs, double chi, double th, double inv_cell,
                                           double &fl, double &frac) {
#pragma clang fp contract(off)
    const double u = (obs + chi * th) * inv_cell;
    fl = floor(u);
    frac = u - fl;
}

// Wave-aggregated atomic increment of counter[key] for every lane with key >= 0.
// The loop only groups equal keys (ballot per distinct key); afterwards the group
// leaders issue their atomics together in one instruction, so a wave pays one atomic
// round trip whatever the number of distinct keys. Returns the lane's slot (old counter
// value + rank among the lanes with the same key) when WANT_SLOT, else -1.
// All 64 lanes of the wave must call it (lanes without work pass key = -1).
template <bool WANT_SLOT>
__device__ __forceinline__ int wave_aggregated_increment(unsigned int *counter, int key) {
    const int lane = __lane_id();
    unsigned long long remaining = __ballot(key >= 0);
    int leader_of_mine = lane, rank = 0;
    unsigned int count = 0;
    while (remaining) {
        const int leader = __ffsll((long long)remaining) - 1;             // wave-uniform
        const int lkey = __builtin_amdgcn_readlane(key, leader);         // no LDS round trip
        const unsigned long long grp = __ballot(key == lkey);
        if (key == lkey) {
            leader_of_mine = leader;
            rank = __popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == leader) count = (unsigned int)__popcll(grp);
        remaining &= ~grp;
    }
    if (!WANT_SLOT) {
        if (count) atomicAdd(&counter[key], count);
        return -1;
    }
    unsigned int base = 0;
    if (count) base = atomicAdd(&counter[key], count);
    base = __shfl(base, leader_of_mine);
    return key >= 0 ? (int)base + rank : -1;
}

// wave_aggregated_increment<true> in two halves, so that a lane can have several such
// reservations in flight: wave_reserve groups the keys and issues the leaders' atomic (its
// old value is not waited for), wave_reserved_slot then returns the lane's slot.
struct WaveReservation {
    unsigned int old;        // the leader's atomic result (leader lanes)
    int leader, rank;
};
__device__ __forceinline__ WaveReservation wave_reserve(unsigned int *counter, int key) {
    const int lane = __lane_id();
    unsigned long long remaining = __ballot(key >= 0);
    WaveReservation w{0u, lane, 0};
    unsigned int count = 0;
    while (remaining) {
        const int leader = __ffsll((long long)remaining) - 1;
        const int lkey = __builtin_amdgcn_readlane(key, leader);
        const unsigned long long grp = __ballot(key == lkey);
        if (key == lkey) {
            w.leader = leader;
            w.rank = __popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == leader) count = (unsigned int)__popcll(grp);
        remaining &= ~grp;
    }
    if (count) w.old = atomicAdd(&counter[key], count);
    return w;
}
__device__ __forceinline__ int wave_reserved_slot(const WaveReservation &w, int key) {
    const unsigned int base = __shfl(w.old, w.leader);
    return key >= 0 ? (int)base + w.rank : -1;
}

// Streaming accesses that are touched once per kernel use non-temporal loads and stores so
// they do not evict gathered data (mesh nodes) from L2.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_stream(T v, T *p) { __builtin_nontemporal_store(v, p); }

// Particle handled by (logical block b, thread t) of a 256-thread block. With np >= 16 a
// block covers a 16 x 16 patch of one Lagrangian plane and a wave a 16 x 4 strip, so a
// wave's particles fall into few mesh tiles and read few mesh rows; smaller lattices use
// plain linear order.
// Launch-shape variants (chosen by the autotuner; every map covers each particle exactly
// once and the per-particle arithmetic does not depend on it, so results are identical):
// map 0 = the 16 x 16 patches above, 1 = linear order, 2 = 32 x 8 patches (wave 32 x 2,
// needs np >= 32), 3 = 64 x 4 patches (a wave is one contiguous run of 64 particles, the
// block's four waves four neighbouring rows; needs np >= 64). A map a lattice is too small
// for falls back to linear order.
__device__ __forceinline__ int particle_of(int b, int t, int lnp, int map = 0) {
    if (map == 3 && lnp >= 6) {
        const int pbx = 1 << (lnp - 6), pby = 1 << (lnp - 2);
        const int bx = b & (pbx - 1), by = (b >> (lnp - 6)) & (pby - 1), z = b >> (2 * lnp - 8);
        return (((z << lnp) + (by << 2) + (t >> 6)) << lnp) + (bx << 6) + (t & 63);
    }
    if (map == 2 && lnp >= 5) {
        const int pbx = 1 << (lnp - 5), pby = 1 << (lnp - 3);
        const int bx = b & (pbx - 1), by = (b >> (lnp - 5)) & (pby - 1), z = b >> (2 * lnp - 8);
        return (((z << lnp) + (by << 3) + (t >> 5)) << lnp) + (bx << 5) + (t & 31);
    }
    if (map == 1 || lnp < 4) return b * 256 + t;
    const int pb = 1 << (lnp - 4);
    const int bx = b & (pb - 1), by = (b >> (lnp - 4)) & (pb - 1), z = b >> (2 * (lnp - 4));
    return (((z << lnp) + (by << 4) + (t >> 4)) << lnp) + (bx << 4) + (t & 15);
}

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup w runs on XCD w % 8).
// Kernels whose neighbouring blocks share data remap w so that each XCD processes one
// contiguous range of logical blocks and the shared data stays in that XCD's L2.
__device__ __forceinline__ int xcd_block(int nblocks) {
    const int w = blockIdx.x, x = w & 7, k = w >> 3;
    const int per = nblocks >> 3, rem = nblocks & 7;
    return x * per + (x < rem ? x : rem) + k;
}

// Reverse mode: the force-mesh cotangent is summed in 64-bit fixed point. With m the
// largest single contribution (its double bits in *maxbits) and 2^h the most contributions
// one node can receive, one unit is 2^-(62-h) of 2^ceil(log2 m): no partial sum reaches
// 2^62, and integer sums are exact in any order.
__device__ __forceinline__ double adj_fixed_scale(const unsigned long long *maxbits, int hbits) {
    const double m = __longlong_as_double((long long)*maxbits);
    if (!(m > 0.0)) return 1.0;
    int e;
    frexp(m, &e);                                   // m < 2^e
    return ldexp(1.0, 62 - hbits - e);
}

// Block-wide maximum of v >= 0 (every thread of a 256-thread block calls), folded into
// *slot with an integer atomicMax (non-negative doubles order as their bits), issued only when
// the block's maximum exceeds the value already there: the slot only grows, so a stale read
// skips nothing that matters, and most blocks of a launch skip their atomic (same-address
// atomics serialise in L2, a few ns each).
__device__ __forceinline__ void block_max_to(unsigned long long *slot, double v) {
    __shared__ double wmax[4];
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    if (__lane_id() == 0) wmax[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        if (m > 0.0 && mb > __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMax(slot, mb);
    }
}

// Logical block of this workgroup: XCD-grouped (xcd_block) or in dispatch order.
__device__ __forceinline__ int logical_block(int xcd) {
    return xcd ? xcd_block(gridDim.x) : (int)blockIdx.x;
}

// Realisation owning logical block blk (uniform over the block).
__device__ __forceinline__ int real_of(const BlockMap &m, int blk) {
    int r = 0;
    while (r + 1 < m.R && blk >= m.start[r + 1]) ++r;
    return r;
}

}  // namespace hrt
