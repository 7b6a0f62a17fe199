// Device helpers shared by the HIP kernels of the HRT library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace hrt {

template <typename T>
using c2 = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
template <typename T>
using v4 = typename std::conditional<sizeof(T) == 4, float4, double4>::type;

template <typename T>
__device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
    return c2<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Cell index and fraction of particle i along one axis: u = i_lattice * ratio + s / cell.
// The integer part of s / cell is split off first so the fraction keeps the precision
// of the displacement rather than of the absolute coordinate.
template <typename T>
__device__ __forceinline__ void axis_cell(T s, int lattice, int ratio, T inv_cell, int nmask,
                                          int &c, T &f) {
    T t = s * inv_cell;
    T fl = floor(t);
    f = t - fl;
    c = (lattice * ratio + (int)fl) & nmask;
    if (f >= T(1)) {          // t just below an integer rounds up: same point, next cell
        f = T(0);
        c = (c + 1) & nmask;
    }
}

// Wave-aggregated atomic add of 1 on counter[key] for every active lane with key >= 0.
// Returns the lane's slot (old counter value + its rank among lanes with equal key).
// All 64 lanes of the wave must call it (inactive lanes pass key = -1).
__device__ __forceinline__ int wave_aggregated_increment(unsigned int *counter, int key) {
    const int lane = __lane_id();
    unsigned long long remaining = __ballot(key >= 0);
    int slot = -1;
    while (remaining) {
        const int leader = __ffsll((long long)remaining) - 1;
        const int lkey = __shfl(key, leader);
        const unsigned long long grp = __ballot(key == lkey);
        unsigned int base = 0;
        if (lane == leader) base = atomicAdd(&counter[lkey], (unsigned int)__popcll(grp));
        base = __shfl(base, leader);
        if (key == lkey) slot = (int)base + __popcll(grp & ((1ull << lane) - 1ull));
        remaining &= ~grp;
    }
    return slot;
}

}  // namespace hrt
