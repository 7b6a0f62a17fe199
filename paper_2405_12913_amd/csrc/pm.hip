// Particle side of the PM step: deterministic cloud-in-cell paint and the fused
// CIC readout + matter kick + drift.
//
// Paint (paper Sec. 4.2, CIC onto the 3D particle mesh), in four kernels:
//   1. bin_count   particles -> bin key (8^3-cell tile, and which of the tile's upper
//                  faces the particle's cell touches), wave-aggregated integer counts
//   2. scan        exclusive prefix sum of the counts (bin offsets, scatter cursors)
//   3. bin_scatter write (cell fraction, local cell) of every particle into its bin
//   4. paint_tiles one workgroup per tile pulls the particles of its own bins and of the
//                  upper-face bins of its 7 lower neighbours, and sums their CIC weights
//                  into the tile's 8^3 nodes in LDS as 64-bit fixed point.
// Integer sums are exact and order-independent, so the mesh is bit-identical across
// runs whatever the atomics' interleaving; each node is written by exactly one
// workgroup with a plain store. The result is delta = rho / rho_bar - 1.
#include "device_common.h"
#include "hrt_internal.h"

namespace hrt {
namespace {

constexpr int kTile = 8;
constexpr int kThreads = 256;

// np is a power of two (it divides the power-of-two mesh size): lattice indices by shifts.
template <typename T>
__device__ __forceinline__ void particle_cell(const T *__restrict__ sx, const T *__restrict__ sy,
                                              const T *__restrict__ sz, int i, int lnp,
                                              int ratio, T inv_cell, int nmask, int c[3], T f[3]) {
    const int pm = (1 << lnp) - 1;
    const int ix = i & pm;
    const int iy = (i >> lnp) & pm;
    const int iz = i >> (2 * lnp);
    axis_cell<T>(ld_stream(sx + i), ix, ratio, inv_cell, nmask, c[0], f[0]);
    axis_cell<T>(ld_stream(sy + i), iy, ratio, inv_cell, nmask, c[1], f[1]);
    axis_cell<T>(ld_stream(sz + i), iz, ratio, inv_cell, nmask, c[2], f[2]);
}

__device__ __forceinline__ int bin_key(const int c[3], int nt) {
    const int mask = ((c[0] & 7) == 7) | (((c[1] & 7) == 7) << 1) | (((c[2] & 7) == 7) << 2);
    return (((c[2] >> 3) * nt + (c[1] >> 3)) * nt + (c[0] >> 3)) * 8 + mask;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void bin_count_kernel(
    const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz, int P, int lnp,
    int ratio, T inv_cell, int n, unsigned int *__restrict__ count) {
    const int i = particle_of(blockIdx.x, threadIdx.x, lnp);
    int key = -1;
    if (i < P) {
        int c[3];
        T f[3];
        particle_cell<T>(sx, sy, sz, i, lnp, ratio, inv_cell, n - 1, c, f);
        key = bin_key(c, n / kTile);
    }
    wave_aggregated_increment<false>(count, key);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void bin_scatter_kernel(
    const T *__restrict__ sx, const T *__restrict__ sy, const T *__restrict__ sz, int P, int lnp,
    int ratio, T inv_cell, int n, unsigned int *__restrict__ cursor, v4<T> *__restrict__ sorted) {
    const int i = particle_of(blockIdx.x, threadIdx.x, lnp);
    int key = -1;
    int c[3] = {0, 0, 0};
    T f[3] = {0, 0, 0};
    if (i < P) {
        particle_cell<T>(sx, sy, sz, i, lnp, ratio, inv_cell, n - 1, c, f);
        key = bin_key(c, n / kTile);
    }
    const int slot = wave_aggregated_increment<true>(cursor, key);
    if (i < P) {
        const int lcell = ((c[2] & 7) * 8 + (c[1] & 7)) * 8 + (c[0] & 7);
        v4<T> e;
        e.x = f[0];
        e.y = f[1];
        e.z = f[2];
        if constexpr (sizeof(T) == 4) e.w = __int_as_float(lcell);
        else e.w = (double)lcell;
        sorted[slot] = e;
    }
}

__global__ void fill_u32_kernel(unsigned int *p, int64_t n, unsigned int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan, 1024 elements per block: local scan + block totals.
__global__ __launch_bounds__(256) void scan_local_kernel(const unsigned int *__restrict__ in,
                                                         int64_t n, unsigned int *__restrict__ out,
                                                         unsigned int *__restrict__ block_sums) {
    __shared__ unsigned int s[256];
    const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x * 4;
    unsigned int v[4], t = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0u;
        t += v[k];
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        unsigned int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned int run = s[threadIdx.x] - t;   // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) block_sums[blockIdx.x] = s[255];
}

// Exclusive scan of the block totals in one block of 1024 threads.
__global__ __launch_bounds__(1024) void scan_sums_kernel(unsigned int *__restrict__ sums, int nb) {
    __shared__ unsigned int s[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    unsigned int t = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) t += sums[b0 + k];
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned int x = threadIdx.x >= off ? s[threadIdx.x - off] : 0u;
        __syncthreads();
        s[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned int run = s[threadIdx.x] - t;
    for (int k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            unsigned int v = sums[b0 + k];
            sums[b0 + k] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) sums[nb] = s[1023];
}

__global__ __launch_bounds__(256) void scan_add_kernel(unsigned int *__restrict__ offs, int64_t n,
                                                       const unsigned int *__restrict__ sums, int nb,
                                                       unsigned int *__restrict__ cursor) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const unsigned int v = offs[i] + sums[i / 1024];
        offs[i] = v;
        cursor[i] = v;
    }
    if (i == 0) offs[n] = sums[nb];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void paint_tiles_kernel(
    const v4<T> *__restrict__ sorted, const unsigned int *__restrict__ offs, int n,
    double scale, double inv_scale_rho, T *__restrict__ delta) {
    __shared__ unsigned long long acc[512];
    __shared__ int rstart[27], rpre[28];
    __shared__ signed char rd[27][3];
    const int nt = n / kTile;
    const int t = xcd_block(nt * nt * nt);
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    for (int k = threadIdx.x; k < 512; k += kThreads) acc[k] = 0ull;
    if (threadIdx.x == 0) {
        int r = 0;
        rpre[0] = 0;
        for (int dz = 0; dz >= -1; --dz)
            for (int dy = 0; dy >= -1; --dy)
                for (int dx = 0; dx >= -1; --dx) {
                    const int req = (dx ? 1 : 0) | (dy ? 2 : 0) | (dz ? 4 : 0);
                    const int tn = ((((tz + dz) & (nt - 1)) * nt + ((ty + dy) & (nt - 1))) * nt +
                                    ((tx + dx) & (nt - 1)));
                    for (int m = 0; m < 8; ++m) {
                        if ((m & req) != req) continue;
                        const int b = tn * 8 + m;
                        rstart[r] = (int)offs[b];
                        rpre[r + 1] = rpre[r] + (int)(offs[b + 1] - offs[b]);
                        rd[r][0] = (signed char)dx;
                        rd[r][1] = (signed char)dy;
                        rd[r][2] = (signed char)dz;
                        ++r;
                    }
                }
    }
    __syncthreads();
    const int total = rpre[27];
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        int r = 0;
        while (idx >= rpre[r + 1]) ++r;
        const v4<T> e = sorted[rstart[r] + (idx - rpre[r])];
        int lcell;
        if constexpr (sizeof(T) == 4) lcell = __float_as_int(e.w);
        else lcell = (int)e.w;
        const int bx = kTile * rd[r][0] + (lcell & 7);
        const int by = kTile * rd[r][1] + ((lcell >> 3) & 7);
        const int bz = kTile * rd[r][2] + (lcell >> 6);
#pragma unroll
        for (int cz = 0; cz < 2; ++cz) {
            const int nz = bz + cz;
            if (nz < 0 || nz >= kTile) continue;
            const T wz = cz ? e.z : T(1) - e.z;
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
                const int ny = by + cy;
                if (ny < 0 || ny >= kTile) continue;
                const T wyz = wz * (cy ? e.y : T(1) - e.y);
#pragma unroll
                for (int cx = 0; cx < 2; ++cx) {
                    const int nx = bx + cx;
                    if (nx < 0 || nx >= kTile) continue;
                    const T w = wyz * (cx ? e.x : T(1) - e.x);
                    const unsigned long long q = (unsigned long long)llrint((double)w * scale);
                    atomicAdd(&acc[(nz * kTile + ny) * kTile + nx], q);
                }
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 512; k += kThreads) {
        const int x = tx * kTile + (k & 7), y = ty * kTile + ((k >> 3) & 7), z = tz * kTile + (k >> 6);
        st_stream((T)((double)acc[k] * inv_scale_rho - 1.0), delta + ((size_t)z * n + y) * n + x);
    }
}

// One lane per particle, particles in Lagrangian order; blocks are XCD-remapped so
// neighbouring particle rows (which read the same mesh rows) share one L2.
template <typename T>
__global__ __launch_bounds__(kThreads) void matter_kd_kernel(
    T *__restrict__ sx, T *__restrict__ sy, T *__restrict__ sz, T *__restrict__ px,
    T *__restrict__ py, T *__restrict__ pz, const v4<T> *__restrict__ g, int P, int lnp, int ratio,
    T inv_cell, int n, T K, T D) {
    const int i = particle_of(xcd_block(gridDim.x), threadIdx.x, lnp);
    if (i >= P) return;
    int c[3];
    T f[3];
    const T s0 = ld_stream(sx + i), s1 = ld_stream(sy + i), s2 = ld_stream(sz + i);
    {
        const int pm = (1 << lnp) - 1;
        axis_cell<T>(s0, i & pm, ratio, inv_cell, n - 1, c[0], f[0]);
        axis_cell<T>(s1, (i >> lnp) & pm, ratio, inv_cell, n - 1, c[1], f[1]);
        axis_cell<T>(s2, i >> (2 * lnp), ratio, inv_cell, n - 1, c[2], f[2]);
    }
    T gx = 0, gy = 0, gzz = 0;
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const int z = (c[2] + cz) & (n - 1);
        const T wz = cz ? f[2] : T(1) - f[2];
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int y = (c[1] + cy) & (n - 1);
            const T wyz = wz * (cy ? f[1] : T(1) - f[1]);
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int x = (c[0] + cx) & (n - 1);
                const T w = wyz * (cx ? f[0] : T(1) - f[0]);
                const v4<T> gv = g[((size_t)z * n + y) * n + x];
                gx += w * gv.x;
                gy += w * gv.y;
                gzz += w * gv.z;
            }
        }
    }
    const T npx = ld_stream(px + i) + K * gx;
    const T npy = ld_stream(py + i) + K * gy;
    const T npz = ld_stream(pz + i) + K * gzz;
    st_stream(npx, px + i);
    st_stream(npy, py + i);
    st_stream(npz, pz + i);
    st_stream(s0 + D * npx, sx + i);
    st_stream(s1 + D * npy, sy + i);
    st_stream(s2 + D * npz, sz + i);
}

template <typename T>
hipError_t paint_impl(hrt_ctx *c, const hrt_matter *m) {
    const int n = c->n, np = c->np;
    const int P = np * np * np;
    const int lnp = ilog2(np);
    const int ratio = n / np;
    const T inv_cell = (T)(1.0 / c->cell);
    const int64_t nbins = c->lay.nbins;
    unsigned int *count = reinterpret_cast<unsigned int *>(c->ws + c->lay.bins);
    unsigned int *offs = count + nbins;                 // nbins + 1
    unsigned int *sums = offs + nbins + 1;              // nblk + 1
    unsigned int *cursor = reinterpret_cast<unsigned int *>(c->ws + c->lay.cursor);
    v4<T> *sorted = reinterpret_cast<v4<T> *>(c->ws + c->lay.sorted);
    T *delta = reinterpret_cast<T *>(c->ws + c->lay.mesh_r);
    const T *sx = static_cast<const T *>(m->s[0]);
    const T *sy = static_cast<const T *>(m->s[1]);
    const T *sz = static_cast<const T *>(m->s[2]);
    hipStream_t st = c->stream;
    const int pblocks = (P + kThreads - 1) / kThreads;
    prof_begin(c);
    fill_u32_kernel<<<(int)((nbins + 255) / 256), 256, 0, st>>>(count, nbins, 0u);
    bin_count_kernel<T><<<pblocks, kThreads, 0, st>>>(sx, sy, sz, P, lnp, ratio, inv_cell, n, count);
    prof_end(c, K_BIN_COUNT);
    const int nblk = (int)((nbins + 1023) / 1024);
    prof_begin(c);
    scan_local_kernel<<<nblk, 256, 0, st>>>(count, nbins, offs, sums);
    scan_sums_kernel<<<1, 1024, 0, st>>>(sums, nblk);
    scan_add_kernel<<<(int)((nbins + 255) / 256), 256, 0, st>>>(offs, nbins, sums, nblk, cursor);
    prof_end(c, K_BIN_SCAN);
    prof_begin(c);
    bin_scatter_kernel<T><<<pblocks, kThreads, 0, st>>>(sx, sy, sz, P, lnp, ratio, inv_cell, n,
                                                         cursor, sorted);
    prof_end(c, K_BIN_SCATTER);
    const double scale = std::ldexp(1.0, c->fixed_bits);
    const double rho_bar = (double)P / ((double)n * n * n);
    const int ntiles = (n / kTile) * (n / kTile) * (n / kTile);
    prof_begin(c);
    paint_tiles_kernel<T><<<ntiles, kThreads, 0, st>>>(sorted, offs, n, scale, 1.0 / (scale * rho_bar),
                                                        delta);
    prof_end(c, K_PAINT);
    return hipGetLastError();
}

template <typename T>
hipError_t matter_impl(hrt_ctx *c, const hrt_matter *m, double K, double D) {
    const int n = c->n, np = c->np;
    const int P = np * np * np;
    const v4<T> *g = reinterpret_cast<const v4<T> *>(c->ws + c->lay.grad);
    prof_begin(c);
    matter_kd_kernel<T><<<(P + kThreads - 1) / kThreads, kThreads, 0, c->stream>>>(
        static_cast<T *>(m->s[0]), static_cast<T *>(m->s[1]), static_cast<T *>(m->s[2]),
        static_cast<T *>(m->p[0]), static_cast<T *>(m->p[1]), static_cast<T *>(m->p[2]), g, P,
        ilog2(np), n / np, (T)(1.0 / c->cell), n, (T)K, (T)D);
    prof_end(c, K_MATTER_KD);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_paint(hrt_ctx *c, const hrt_matter *m) {
    return c->f64 ? paint_impl<double>(c, m) : paint_impl<float>(c, m);
}

hipError_t launch_matter_kd(hrt_ctx *c, const hrt_matter *m, double K, double D) {
    return c->f64 ? matter_impl<double>(c, m, K, D) : matter_impl<float>(c, m, K, D);
}

}  // namespace hrt
