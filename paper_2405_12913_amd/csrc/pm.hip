// Particle side of the PM step: deterministic cloud-in-cell paint and the fused
// CIC readout + matter kick + drift. Every kernel covers all realisations of a context
// in one launch; realisation r owns the blocks [map.start[r], map.start[r+1]).
//
// Paint (paper Sec. 5.2, CIC onto the 3D particle mesh), in four kernels:
//   1. bin_count   particles -> bin key (8^3-cell tile, and which of the tile's upper
//                  faces the particle's cell touches), wave-aggregated integer counts
//   2. scan        exclusive prefix sum of the counts (bin offsets, scatter cursors)
//   3. bin_scatter write (cell fraction, local cell) of every particle into its bin
//   4. paint_tiles each tile (one, two or four per workgroup) pulls the particles of its
//                  own bins and of the upper-face bins of its 7 lower neighbours, and sums
//                  their CIC weights into the tile's 8^3 nodes in LDS as fixed point (FP32:
//                  32-bit sums of x-pairs of nodes at the scale 2^20, folded into 64-bit
//                  sums; FP64: 64-bit sums at the global scale).
// Integer sums are exact and order-independent, so the mesh is bit-identical across
// runs whatever the atomics' interleaving; each node is written by exactly one
// workgroup with a plain store. The result is delta = rho / rho_bar - 1.
// hrt_run can keep the particles in bin order for a whole sequence of steps (the
// sorted-state kernels further down: state_scatter, kd_tiles, state_gather).
#include "device_common.h"

namespace hrt {
namespace {

constexpr int kTile = 8;
constexpr int kThreads = 256;

template <typename T>
struct Particles {             // one realisation, as the particle kernels see it
    T *s[3], *p[3];
    unsigned int *count, *offs, *sums, *cursor;
    v4<T> *sorted;
    const v4<T> *grad;
    T *delta;
    v4<T> *rec[2];             // sorted-state run: records (s_x, s_y, s_z, lattice index)
    T *mom[2];                 //   and momenta (3 x P, axis-major), two buffers in turn
    const T *phi;
    int n, lnp, lratio, lnt, P, nbins, nblk;   // lnt = log2(n / 8)
    T inv_cell, K, D, inv12cell;
    double scale, inv_scale_rho;
    int fixed_bits;            // scale = 2^fixed_bits
    char *lbase;               // mover-list region (FP32 moving particles), else NULL
    int par;                   // mover-list run: the step's parity (its control words)
};

// CIC weight w in [0, 1] as a fixed-point integer round(w 2^F). For float the product is
// formed from w's bits (mantissa shifted by its exponent): exact whenever w 2^F is an
// integer (every w >= 2^(23-F)), rounded half up below that; for double by llrint.
__device__ __forceinline__ unsigned long long to_fixed(float w, double, int F) {
    // branch-free: shift left by max(sh, 0), round and shift right by min(max(-sh, 0), 63)
    const unsigned int bits = __float_as_uint(w);
    const int e = (int)((bits >> 23) & 0xffu);                 // sign dropped: -0 gives 0
    const unsigned long long m = (bits & 0x7fffffu) | 0x800000u;
    const int sh = e - 150 + F;                                // w 2^F = m 2^sh
    const int ls = sh > 0 ? sh : 0;
    const int rs = sh < 0 ? (-sh < 63 ? -sh : 63) : 0;
    const unsigned long long r = ((m << ls) + ((1ull << rs) >> 1)) >> rs;
    return e == 0 ? 0ull : r;                                  // zero (and denormals)
}
__device__ __forceinline__ unsigned long long to_fixed(double w, double scale, int) {
    return (unsigned long long)llrint(w * scale);
}

template <typename T>
struct PartBatch {
    BlockMap map;
    Particles<T> r[kMaxBatch];
    int pmap, xcd;             // launch-shape variant: particle map, XCD block grouping
};
static_assert(sizeof(PartBatch<double>) <= 4096, "kernel argument block over 4 KB");

// Mover-list run (kd_tiles variants 5 and 6): the control region at lbase, carved as
// list_offsets says; the particle data are indexed from rec0 = rec[0] and mom0 = mom[0]:
// records [rec0 | S | rec1 | U] (fronts of buffer cur from 2P cur, S from P, U from 3P),
// momenta [mom0 | S | mom1 | U] (axis d of a front slot at 6P cur + d P + slot, of S at
// 3P + d P + j, of U at 9P + 2P d + u).
template <typename T>
struct ListBufs {
    ListCtl *ctl;              // ctl[0], ctl[1]: control words per step parity
    unsigned int *lcount, *lcursor, *loffs, *lsums;   // histogram / cursors / offsets of S
    unsigned int *ubase, *ucnt;   // extent of each kick-drift workgroup's entries of U
};
template <typename T>
__device__ __forceinline__ ListBufs<T> list_bufs(const Particles<T> &a) {
    const ListOffsets o = list_offsets((size_t)a.nbins);
    char *const b = a.lbase;
    auto u32 = [&](size_t off) { return reinterpret_cast<unsigned int *>(b + off); };
    return ListBufs<T>{reinterpret_cast<ListCtl *>(b + o.ctl), u32(o.lcount), u32(o.lcursor), u32(o.loffs),
                       u32(o.lsums), u32(o.ubase), u32(o.ucnt)};
}

// Load of a value that is the same for the whole wave and that no kernel running alongside
// writes (the bin offsets, written by an earlier launch), through the constant address space,
// so it is a scalar load: it is not counted with the vector memory operations, and waiting
// for it does not wait for the stores the wave has issued.
__device__ __forceinline__ unsigned int uniform_load(const unsigned int *p) {
    return *(const __attribute__((address_space(4))) unsigned int *)p;
}

// A step that starts with more entries in S than the run's limit (P/16 by default) ends with
// a re-binning instead of the sort of U into S; it is known before the step's kick-drift,
// which then counts every particle into the full histogram (else only U's entries into the
// mover histogram). The list holds about one step's movers per step since the last
// re-binning (1-2 % of the particles per step on an evolved field at 256^3).
__device__ __forceinline__ bool list_rebuild(const ListCtl &q, int) { return q.nlist > q.limit; }

// np is a power of two (it divides the power-of-two mesh size): lattice indices by shifts.
template <typename T>
__device__ __forceinline__ void particle_cell(const Particles<T> &a, int i, int c[3], T f[3],
                                              T sv[3]) {
    const int pm = (1 << a.lnp) - 1;
    const int lat[3] = {i & pm, (i >> a.lnp) & pm, i >> (2 * a.lnp)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        sv[d] = ld_stream(a.s[d] + i);
        axis_cell<T>(sv[d], lat[d], a.lratio, a.inv_cell, a.n - 1, c[d], f[d]);
    }
}

// Sorted-state records (hrt_run): (s_x, s_y, s_z, lattice index), the index stored as the
// float's bits (FP32) or as an exact double (FP64).
template <typename T>
__device__ __forceinline__ int rec_index(const v4<T> &r) {
    if constexpr (sizeof(T) == 4) return __float_as_int(r.w);
    else return (int)r.w;
}

template <typename T>
__device__ __forceinline__ T index_field(int i) {
    if constexpr (sizeof(T) == 4) return __int_as_float(i);
    else return (T)i;
}

// What a particle's cell needs, copied out of the kernel arguments once so that loops keep
// it in registers (the compiler reloads argument fields after every global store).
template <typename T>
struct CellGeom {
    int lnp, lratio, nmask;
    T inv_cell;
};
template <typename T>
__device__ __forceinline__ CellGeom<T> geom_of(const Particles<T> &a) {
    return CellGeom<T>{a.lnp, a.lratio, a.n - 1, a.inv_cell};
}

// Cell and fraction of a record, exactly as particle_cell forms them from s and i.
template <typename T>
__device__ __forceinline__ void record_cell(const CellGeom<T> &g, const v4<T> &rec, int c[3], T f[3]) {
    const int i = rec_index<T>(rec), pm = (1 << g.lnp) - 1;
    const int lat[3] = {i & pm, (i >> g.lnp) & pm, i >> (2 * g.lnp)};
    axis_cell<T>(rec.x, lat[0], g.lratio, g.inv_cell, g.nmask, c[0], f[0]);
    axis_cell<T>(rec.y, lat[1], g.lratio, g.inv_cell, g.nmask, c[1], f[1]);
    axis_cell<T>(rec.z, lat[2], g.lratio, g.inv_cell, g.nmask, c[2], f[2]);
}

// Bin of a particle in cell c: its 8^3 tile ((n/8)^3 = 2^(3 lnt) tiles, x fastest) times 8
// plus the mask of the tile's upper faces that its cell touches.
__device__ __forceinline__ int bin_key(const int c[3], int lnt) {
    const int mask = ((c[0] & 7) == 7) | (((c[1] & 7) == 7) << 1) | (((c[2] & 7) == 7) << 2);
    return (((((c[2] >> 3) << lnt) + (c[1] >> 3)) << lnt) + (c[0] >> 3)) * 8 + mask;
}

template <typename T>
__global__ __launch_bounds__(256) void fill_counts_kernel(PartBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const int i = (blockIdx.x - b.map.start[r]) * 256 + threadIdx.x;
    if (i < a.nbins) a.count[i] = 0u;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void bin_count_kernel(PartBatch<T> b) {
    const int blk = logical_block(b.xcd);
    const int r = real_of(b.map, blk);
    const Particles<T> &a = b.r[r];
    const int i = particle_of(blk - b.map.start[r], threadIdx.x, a.lnp, b.pmap);
    int key = -1;
    if (i < a.P) {
        int c[3];
        T f[3], sv[3];
        particle_cell<T>(a, i, c, f, sv);
        key = bin_key(c, a.lnt);
    }
    wave_aggregated_increment<false>(a.count, key);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void bin_scatter_kernel(PartBatch<T> b) {
    const int blk = logical_block(b.xcd);
    const int r = real_of(b.map, blk);
    const Particles<T> &a = b.r[r];
    const int i = particle_of(blk - b.map.start[r], threadIdx.x, a.lnp, b.pmap);
    int key = -1;
    int c[3] = {0, 0, 0};
    T f[3] = {0, 0, 0}, sv[3];
    if (i < a.P) {
        particle_cell<T>(a, i, c, f, sv);
        key = bin_key(c, a.lnt);
    }
    const int slot = wave_aggregated_increment<true>(a.cursor, key);
    if (i < a.P) {
        const int lcell = ((c[2] & 7) * 8 + (c[1] & 7)) * 8 + (c[0] & 7);
        v4<T> e;
        e.x = f[0];
        e.y = f[1];
        e.z = f[2];
        if constexpr (sizeof(T) == 4) e.w = __int_as_float(lcell);
        else e.w = (double)lcell;
        a.sorted[slot] = e;
    }
}

// Exclusive scan, 1024 elements per block: local scan + block totals.
// The arrays one scan works on. LIST (the settle of a mover-list step): the full histogram
// (count -> offs, cursor: a re-binning) or the mover histogram (lcount -> loffs, lcursor:
// the sort of U), as list_rebuild decides from the step's control words; every block of
// the scan decides alike (the words are final once the kick-drift has run).
struct ScanArrays {
    unsigned int *count, *offs, *sums, *cursor;
    bool rebuild;
};
template <typename T, bool LIST>
__device__ __forceinline__ ScanArrays scan_arrays(const Particles<T> &a) {
    if constexpr (LIST) {
        const ListBufs<T> l = list_bufs(a);
        if (!list_rebuild(l.ctl[a.par], a.P)) return ScanArrays{l.lcount, l.loffs, l.lsums, l.lcursor, false};
        return ScanArrays{a.count, a.offs, a.sums, a.cursor, true};
    }
    return ScanArrays{a.count, a.offs, a.sums, a.cursor, false};
}

template <typename T, bool LIST>
__global__ __launch_bounds__(256) void scan_local_kernel(PartBatch<T> b) {
    __shared__ unsigned int sh[256];
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const ScanArrays s = scan_arrays<T, LIST>(a);
    const int blk = blockIdx.x - b.map.start[r];
    const int base = blk * 1024 + threadIdx.x * 4;
    unsigned int v[4], t = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < a.nbins) ? s.count[base + k] : 0u;
        t += v[k];
    }
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        unsigned int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned int run = sh[threadIdx.x] - t;   // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
        if (base + k < a.nbins) s.offs[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == 255) s.sums[blk] = sh[255];
}

// Exclusive scan of the block totals, one block of 1024 threads per realisation.
template <typename T, bool LIST>
__global__ __launch_bounds__(1024) void scan_sums_kernel(PartBatch<T> b) {
    __shared__ unsigned int sh[1024];
    const Particles<T> &a = b.r[blockIdx.x];
    const ScanArrays s = scan_arrays<T, LIST>(a);
    const int nb = a.nblk;
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    unsigned int t = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < nb) t += s.sums[b0 + k];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        unsigned int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    unsigned int run = sh[threadIdx.x] - t;
    for (int k = 0; k < per; ++k) {
        if (b0 + k < nb) {
            unsigned int v = s.sums[b0 + k];
            s.sums[b0 + k] = run;
            run += v;
        }
    }
    if (threadIdx.x == 1023) s.sums[nb] = sh[1023];
}

// FUSED (every realisation has at most 1024 blocks of 1024 bins): the block totals are not
// scanned by a kernel of their own; each workgroup sums the totals of the blocks before its
// own (and all of them, for the end offset) from the unscanned array, integer sums in any
// order. Otherwise scan_sums_kernel has scanned them in place.
// LIST: both histograms are cleared for the next kick-drift, and a re-binning empties S.
template <typename T, bool FUSED, bool LIST>
__global__ __launch_bounds__(256) void scan_add_kernel(PartBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const ScanArrays s = scan_arrays<T, LIST>(a);
    const int i0 = (blockIdx.x - b.map.start[r]) * 256, i = i0 + threadIdx.x;
    unsigned int pre, total;
    if constexpr (FUSED) {
        __shared__ unsigned int part[2][4];
        const int grp = i0 / 1024;              // uniform: 1024 is a multiple of 256
        unsigned int v = 0, vt = 0;
        for (int k = threadIdx.x; k < a.nblk; k += 256) {
            const unsigned int x = s.sums[k];
            v += k < grp ? x : 0u;
            vt += x;
        }
        for (int off = 32; off > 0; off >>= 1) {
            v += __shfl_xor(v, off);
            vt += __shfl_xor(vt, off);
        }
        if (__lane_id() == 0) {
            part[0][threadIdx.x >> 6] = v;
            part[1][threadIdx.x >> 6] = vt;
        }
        __syncthreads();
        pre = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        total = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    } else {
        pre = i < a.nbins ? s.sums[i / 1024] : 0u;
        total = s.sums[a.nblk];
    }
    if (i < a.nbins) {
        const unsigned int v = s.offs[i] + pre;
        s.offs[i] = v;
        s.cursor[i] = v;
        s.count[i] = 0u;       // consumed by scan_local: zero for the next count (kick-drift)
    }
    if (i == 0) s.offs[a.nbins] = total;
    if constexpr (LIST) {
        const ListBufs<T> l = list_bufs(a);
        if (i < a.nbins && s.rebuild) l.loffs[i] = 0u;    // S is empty after a re-binning
        if (i == 0 && s.rebuild) l.loffs[a.nbins] = 0u;
    }
}

// The 27 bin ranges whose particles reach tile (tx, ty, tz): the tile's own 8 bins and
// the upper-face bins of its 7 lower neighbours (a neighbour displaced by -1 along some
// axes contributes the bins whose face mask has those axes set). Computed in parallel by
// lanes 0..26 of the group's first wave and prefix-summed across the wave (visible after
// the caller's barrier): range r starts at sorted index rstart[r], the ranges' prefix sizes
// are rpre[0..27], rd[r] is the neighbour's offset. Each group's arrays are padded to 32
// entries and 16-byte aligned, so no access to one group's entries touches another's.
// The order of the ranges only changes the order of the integer sums, not their value.
__constant__ signed char kRangeTab[27][4] = {
    {0, 0, 0, 0}, {0, 0, 0, 1}, {0, 0, 0, 2}, {0, 0, 0, 3}, {0, 0, 0, 4}, {0, 0, 0, 5},
    {0, 0, 0, 6}, {0, 0, 0, 7},                                     // own tile, every mask
    {-1, 0, 0, 1}, {-1, 0, 0, 3}, {-1, 0, 0, 5}, {-1, 0, 0, 7},     // x - 1: masks with x
    {0, -1, 0, 2}, {0, -1, 0, 3}, {0, -1, 0, 6}, {0, -1, 0, 7},     // y - 1: masks with y
    {0, 0, -1, 4}, {0, 0, -1, 5}, {0, 0, -1, 6}, {0, 0, -1, 7},     // z - 1: masks with z
    {-1, -1, 0, 3}, {-1, -1, 0, 7}, {-1, 0, -1, 5}, {-1, 0, -1, 7}, // two axes
    {0, -1, -1, 6}, {0, -1, -1, 7}, {-1, -1, -1, 7}};               // three axes

// LIST (mover-list run): 54 ranges, the 27 bins' fronts in the record buffer and then the
// same 27 bins' entries of the sorted side list S (offsets loffs), as indices from rec0 (the
// fronts shifted by fo, S by so).
template <typename T, bool LIST = false>
__device__ __forceinline__ void tile_ranges(const Particles<T> &a, int tx, int ty, int tz, int *rstart,
                                            int *rpre, signed char (*rd)[3], int k,
                                            const unsigned int *loffs = nullptr, int fo = 0, int so = 0) {
    constexpr int NR = LIST ? 54 : 27;
    if (k >= 64) return;                        // the group's first wave does it all
    const int nt = a.n / kTile;
    int size = 0;
    if (k < NR) {
        const int kk = k < 27 ? k : k - 27;
        const int dx = kRangeTab[kk][0], dy = kRangeTab[kk][1], dz = kRangeTab[kk][2];
        const int tn = ((((tz + dz) & (nt - 1)) * nt + ((ty + dy) & (nt - 1))) * nt + ((tx + dx) & (nt - 1)));
        const int bb = tn * 8 + kRangeTab[kk][3];
        const unsigned int *const o = (LIST && k >= 27) ? loffs : a.offs;
        const unsigned int o0 = o[bb], o1 = o[bb + 1];
        rstart[k] = (int)o0 + (LIST ? (k >= 27 ? so : fo) : 0);    // LIST: indices from rec0
        size = (int)(o1 - o0);
        rd[k][0] = (signed char)dx;
        rd[k][1] = (signed char)dy;
        rd[k][2] = (signed char)dz;
    }
    int incl = size;                            // inclusive prefix over the wave's lanes
#pragma unroll
    for (int off = 1; off < (LIST ? 64 : 32); off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (k >= off) incl += v;
    }
    if constexpr (LIST) {
        // only the ranges that hold entries (and range 0, so that it stays range 0), so
        // that a lane's walk over the ranges skips the many empty ones of sparse tiles and
        // short lists; the entries' total is in rpre[63]
        const bool keep = k < NR && (size > 0 || k == 0);
        const unsigned long long km = __ballot(keep);
        const int kc = __popcll(km & ((1ull << k) - 1ull));
        const int s0 = rstart[k];
        const signed char d0 = rd[k][0], d1 = rd[k][1], d2 = rd[k][2];
        __builtin_amdgcn_wave_barrier();
        if (keep) {
            rstart[kc] = s0;
            rd[kc][0] = d0;
            rd[kc][1] = d1;
            rd[kc][2] = d2;
            rpre[kc + 1] = incl;
        }
        if (k == NR - 1) rpre[63] = incl;
    } else {
        if (k < NR) rpre[k + 1] = incl;
    }
    if (k == 0) rpre[0] = 0;
}

// LDS slot of tile node (x, y, z): rows padded to 9 entries and planes to 74, so that nodes
// with equal (x, y) in different planes (or equal x four rows apart) fall in different
// LDS banks; particles handled by one wave often sit at such nodes.
constexpr int kAccPlane = 74, kAccRow = 9, kAccSize = kTile * kAccPlane;
__device__ __forceinline__ int acc_slot(int x, int y, int z) { return z * kAccPlane + y * kAccRow + x; }

// FP32 sums as node pairs: slot (cx, y, z), cx = -1..7, holds the sums of nodes cx (low 32
// bits) and cx + 1 (high 32 bits) of row (y, z), so one 64-bit LDS add takes a particle's two
// x corners. A pair's low sum stays below 2^32 within a chunk (at most 1024 weights of at
// most 2^20 each), so no carry reaches the high sum and both are exact. Node x is the low
// half of slot x plus the high half of slot x - 1; nodes -1 and 8 (outside the tile) are
// never read. Rows of 9 slots, planes of 72.
constexpr int kPairRow = 9, kPairPlane = 72, kPairSize = kTile * kPairPlane;
__device__ __forceinline__ int pair_slot(int cx, int y, int z) { return z * kPairPlane + y * kPairRow + cx + 1; }

// Adds the CIC weights of one binned particle to the tile's LDS sums. INSIDE: the particle
// is in the tile's own bin that touches no upper face (range 0), so its 8 corners are all
// tile nodes and need no checks; otherwise corners outside the tile (a neighbour's face-bin
// particle, or an upper face) are skipped. FP32: 32-bit sums with the tile's own scale 2^s
// (round(w 2^s)); FP64 and dense tiles: 64-bit sums with the global scale. No contraction,
// so every instantiation of the paint kernel forms the same weights.
// FP32 form over node pairs (pair_slot): four 64-bit adds per particle, each of the two
// weights round(w 2^20) of one (y, z) corner row, with the same products as paint_one; only
// the y and z corners outside the tile are skipped.
template <bool INSIDE>
__device__ __forceinline__ void paint_pair(unsigned long long *acc, const v4<float> &e, int dx, int dy, int dz,
                                           float fscale) {
#pragma clang fp contract(off)
    const int lcell = __float_as_int(e.w);
    const int bx = (INSIDE ? 0 : kTile * dx) + (lcell & 7);
    const int by = (INSIDE ? 0 : kTile * dy) + ((lcell >> 3) & 7);
    const int bz = (INSIDE ? 0 : kTile * dz) + (lcell >> 6);
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const int nz = bz + cz;
        if (!INSIDE && (nz < 0 || nz >= kTile)) continue;
        const float wz = cz ? e.z : 1.0f - e.z;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int ny = by + cy;
            if (!INSIDE && (ny < 0 || ny >= kTile)) continue;
            const float wyz = wz * (cy ? e.y : 1.0f - e.y);
            const float w0 = wyz * (1.0f - e.x), w1 = wyz * e.x;
            const unsigned long long v = ((unsigned long long)(unsigned int)rintf(w1 * fscale) << 32) |
                                         (unsigned long long)(unsigned int)rintf(w0 * fscale);
            atomicAdd(&acc[pair_slot(bx, ny, nz)], v);
        }
    }
}

template <typename T, typename A, bool INSIDE>
__device__ __forceinline__ void paint_one(int fixed_bits, A *acc, const v4<T> &e, int dx, int dy,
                                          int dz, double scale, float fscale) {
#pragma clang fp contract(off)
    int lcell;
    if constexpr (sizeof(T) == 4) lcell = __float_as_int(e.w);
    else lcell = (int)e.w;
    const int bx = (INSIDE ? 0 : kTile * dx) + (lcell & 7);
    const int by = (INSIDE ? 0 : kTile * dy) + ((lcell >> 3) & 7);
    const int bz = (INSIDE ? 0 : kTile * dz) + (lcell >> 6);
#pragma unroll
    for (int cz = 0; cz < 2; ++cz) {
        const int nz = bz + cz;
        if (!INSIDE && (nz < 0 || nz >= kTile)) continue;
        const T wz = cz ? e.z : T(1) - e.z;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy) {
            const int ny = by + cy;
            if (!INSIDE && (ny < 0 || ny >= kTile)) continue;
            const T wyz = wz * (cy ? e.y : T(1) - e.y);
#pragma unroll
            for (int cx = 0; cx < 2; ++cx) {
                const int nx = bx + cx;
                if (!INSIDE && (nx < 0 || nx >= kTile)) continue;
                const T w = wyz * (cx ? e.x : T(1) - e.x);
                if constexpr (sizeof(A) == 4)
                    atomicAdd(&acc[acc_slot(nx, ny, nz)], (unsigned int)rintf((float)w * fscale));
                else
                    atomicAdd(&acc[acc_slot(nx, ny, nz)], to_fixed(w, scale, fixed_bits));
            }
        }
    }
}

// delta = sum inv - 1 (one rounding) at node k (x fastest) of tile (tx, ty, tz).
template <typename T>
__device__ __forceinline__ void store_delta(const Particles<T> &a, int tx, int ty, int tz, int k, double sum,
                                            double inv) {
    const int n = a.n;
    const int x = tx * kTile + (k & 7), y = ty * kTile + ((k >> 3) & 7), z = tz * kTile + (k >> 6);
    st_stream((T)fmadd(sum, inv, -1.0), a.delta + ((size_t)z * n + y) * n + x);
}

// TPB tiles per workgroup (256 / TPB lanes each): when particles are sparse relative to
// nodes (np = n/2: 64 per tile) a workgroup's fixed costs (clearing and storing 512 nodes,
// the bin-range round trip) are shared by several tiles; at one particle per node two tiles
// per workgroup keep twice as many tiles resident per CU (wave slots, not LDS, limit it).
// FP32: 32-bit sums at the scale 2^20 (weights rounded to 2^-21, about the FP32 rounding of
// the cell fractions themselves), kept as x-pairs of nodes (pair_slot), so a particle takes
// four 64-bit LDS adds instead of eight 32-bit ones. The entries are added in chunks of 3072:
// a node's chunk sum is below 3072 2^20 < 2^32 (weights <= 1), so no low half carries into
// its high neighbour. After each chunk every lane folds its nodes' two halves into 64-bit
// node sums (a tile of more than one chunk keeps them in the last copy's region). The scale
// is the same for every tile, so it depends on no count (the mover-list run's holes do not
// change it). NC copies of the sums (lane l adds into copy l mod NC, copies 24 banks apart)
// divide the same-node conflicts of one instruction by about NC; the fold sums the copies.
// FP64: exact 64-bit sums at the global scale, one pass.
// SORTED: the particles are sorted-state records (buffer cur) rather than the binned
// (fraction, local cell) entries of the Lagrangian-order scatter.
// The work of logical block blk (TPB tiles).
constexpr int kPaintDepth = 2;              // entries in flight per lane (more cost a wave per SIMD)
constexpr int kPaintChunk = 3072;           // FP32 entries per chunk of 32-bit sums
constexpr int kAccCopy = kPairSize + 12;    // stride of the FP32 copies (1176 words = 24 mod 64)

// LIST (mover-list run, SORTED): the front of each bin (holes skipped) in the record buffer
// of the step's control words, then its entries of the side list S.
template <typename T, int TPB, bool SORTED, int NC, bool LIST = false>
__device__ __forceinline__ void paint_tiles_body(const PartBatch<T> &b, int cur, int blk) {
    constexpr int NR = LIST ? 54 : 27, RS = LIST ? 64 : 32;   // ranges; their arrays' stride
    constexpr int G = kThreads / TPB;           // lanes per tile
    constexpr bool kWide = sizeof(T) == 8;
    constexpr int kCopies = kWide ? 1 : NC;
    constexpr int kStride = kWide ? kAccSize : kAccCopy;
    constexpr int kNodes = 512 / G;             // nodes per lane in the fold and the stores
    constexpr int ts = 20;                      // FP32 scale 2^ts
    static_assert(kPaintChunk % (kPaintDepth * G) == 0, "chunks of whole trips");
    static_assert((unsigned long long)kPaintChunk << ts < (1ull << 32), "a chunk's pair sums carry");
    using Acc = unsigned long long;             // FP64: node sums; FP32: node-pair sums
    __shared__ Acc acc[TPB][kCopies * kStride];
    // FP32 tiles of more than one chunk keep the node sums of the chunks so far in the last
    // copy's region (later chunks add into the other copies), or, with one copy, in the
    // tile's own nodes of the mesh (low halves in the delta slot, high halves in the phi
    // slot: neither holds anything yet)
    __shared__ __align__(16) int rstart[TPB][RS];
    __shared__ __align__(16) int rpre[TPB][RS];
    __shared__ __align__(16) signed char rd[TPB][RS][3];
    const int rr = real_of(b.map, blk);
    const Particles<T> &a = b.r[rr];
    const int n = a.n, nt = n / kTile;
    const int g = threadIdx.x / G, lane = threadIdx.x % G;
    const int t = (blk - b.map.start[rr]) * TPB + g;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    for (int k = lane; k < kCopies * kStride; k += G) acc[g][k] = Acc(0);
    const unsigned int *loffs = nullptr;
    int fo = 0;                                 // LIST: fronts from rec0 + fo, S from rec0 + P
    if constexpr (LIST) {
        const ListBufs<T> l = list_bufs(a);
        loffs = l.loffs;
        fo = uniform_load(&l.ctl[a.par].cur) ? 2 * a.P : 0;
        cur = 0;
    }
    tile_ranges<T, LIST>(a, tx, ty, tz, rstart[g], rpre[g], rd[g], lane, loffs, fo, a.P);
    __syncthreads();
    const int total = rpre[g][LIST ? 63 : NR];
    // chunks: uniform over the workgroup (every group passes the same barriers)
    int nch = 1;                                // at least one pass (its fold writes the sums)
    if constexpr (!kWide) {
#pragma unroll
        for (int gg = 0; gg < TPB; ++gg) nch = max(nch, (rpre[gg][LIST ? 63 : NR] + kPaintChunk - 1) / kPaintChunk);
    }
    const float fscale = ldexpf(1.0f, ts);
    Acc *mine = acc[g] + (kWide ? 0 : (lane % kCopies) * kStride);
    unsigned long long *const sums = acc[g] + (kCopies > 1 ? (kCopies - 1) * kStride : 0);
    const v4<T> *const src = SORTED ? a.rec[cur] : a.sorted;
    const CellGeom<T> cg = geom_of(a);
    const int fixed_bits = a.fixed_bits;
    const double scale = a.scale;
    // idx only grows, so the range index does too: (fr, fhi, fbase) belong to the furthest
    // entry requested and stay in registers until idx leaves that range. Each lane keeps
    // kPaintDepth entries in flight: entry idx + kPaintDepth G is requested before entry idx
    // is added (a tile's entries are then mostly all requested before the first returns).
    int fr = -1, fhi = 0, fbase = 0;
    auto request = [&](int idx, v4<T> &e, int &r) {
        if (idx >= fhi) {
            do {
                ++fr;
            } while (idx >= rpre[g][fr + 1]);
            fhi = rpre[g][fr + 1];
            fbase = rstart[g][fr] - rpre[g][fr];
        }
        e = src[fbase + idx];
        r = fr;
    };
    v4<T> ev[kPaintDepth];
    int rv[kPaintDepth];
#pragma unroll
    for (int k = 0; k < kPaintDepth; ++k) {
        ev[k] = v4<T>{};
        rv[k] = 0;
        if (lane + k * G < total) request(lane + k * G, ev[k], rv[k]);
    }
    for (int ch = 0; ch < nch; ++ch) {
        // a chunk is a whole number of trips, so the ring holds the next chunk's first entries
        const int cend = kWide ? total : min(total, (ch + 1) * kPaintChunk);
        for (int base = (kWide ? 0 : ch * kPaintChunk) + lane; base < cend; base += kPaintDepth * G) {
#pragma unroll
            for (int k = 0; k < kPaintDepth; ++k) {
                const int idx = base + k * G;
                if (idx >= cend) break;
                v4<T> e = ev[k];
                const int r = rv[k];
                if (idx + kPaintDepth * G < total) request(idx + kPaintDepth * G, ev[k], rv[k]);
                if (LIST && rec_index<T>(e) < 0) continue;   // a hole left by a mover
                if constexpr (SORTED) {             // record -> (fractions, local cell)
                    int c[3];
                    T f[3];
                    record_cell<T>(cg, e, c, f);
                    e.x = f[0];
                    e.y = f[1];
                    e.z = f[2];
                    e.w = index_field<T>(((c[2] & 7) * 8 + (c[1] & 7)) * 8 + (c[0] & 7));
                }
                // own tile, no upper face: 8 inside corners (the list's part of that bin,
                // range 27, takes the checked path: testing for it too costs 5 VGPRs)
                if (r == 0) {
                    if constexpr (kWide) paint_one<T, Acc, true>(fixed_bits, mine, e, 0, 0, 0, scale, fscale);
                    else paint_pair<true>(mine, e, 0, 0, 0, fscale);
                } else {
                    const int dx = rd[g][r][0], dy = rd[g][r][1], dz = rd[g][r][2];
                    if constexpr (kWide) paint_one<T, Acc, false>(fixed_bits, mine, e, dx, dy, dz, scale, fscale);
                    else paint_pair<false>(mine, e, dx, dy, dz, fscale);
                }
            }
        }
        __syncthreads();
        if constexpr (!kWide) {                 // fold the chunk's sums (x = k & 7: low half)
            const int nc = ch == 0 ? kCopies : (kCopies > 1 ? kCopies - 1 : 1);
            auto fold = [&](int k, unsigned long long v) {     // v: the sum of the chunks before
                const int sl = pair_slot(k & 7, (k >> 3) & 7, k >> 6);
#pragma unroll
                for (int cc = 0; cc < kCopies; ++cc)
                    if (cc < nc)
                        v += (acc[g][cc * kStride + sl] & 0xffffffffull) + (acc[g][cc * kStride + sl - 1] >> 32);
                return v;
            };
            if constexpr (kCopies > 1) {        // the sums overwrite the last copy: all reads first
                unsigned long long v[kNodes];
#pragma unroll
                for (int i = 0; i < kNodes; ++i) v[i] = fold(lane + i * G, ch > 0 ? sums[lane + i * G] : 0ull);
                __syncthreads();
#pragma unroll
                for (int i = 0; i < kNodes; ++i) sums[lane + i * G] = v[i];
            } else {                            // one copy: node by node, through the mesh
                const double inv = ldexp(a.inv_scale_rho * a.scale, -ts);
                const size_t n3 = (size_t)n * n * n;
                unsigned int *const lo = reinterpret_cast<unsigned int *>(a.delta);
#pragma unroll 1
                for (int i = 0; i < kNodes; ++i) {
                    const int k = lane + i * G;
                    const size_t at = ((size_t)(tz * kTile + (k >> 6)) * n + (ty * kTile + ((k >> 3) & 7))) * n +
                                      tx * kTile + (k & 7);
                    const unsigned long long prev =
                        ch > 0 ? ((unsigned long long)lo[n3 + at] << 32) | lo[at] : 0ull;
                    const unsigned long long v = fold(k, prev);
                    if (ch + 1 < nch) {
                        lo[at] = (unsigned int)v;
                        lo[n3 + at] = (unsigned int)(v >> 32);
                    } else {
                        store_delta<T>(a, tx, ty, tz, k, (double)v, inv);
                    }
                }
            }
            if (ch + 1 < nch) {                 // clear the copies still added to
                if (kCopies == 1) __syncthreads();
                for (int k = lane; k < (kCopies > 1 ? kCopies - 1 : 1) * kStride; k += G) acc[g][k] = 0ull;
                mine = acc[g] + (kCopies > 1 ? lane % (kCopies - 1) : 0) * kStride;
                __syncthreads();
            }
        }
    }
    if constexpr (!kWide && kCopies > 1) {
        // delta = sum / (2^ts rho_bar) - 1; inv_scale_rho = 1 / (2^fixed_bits rho_bar)
        const double inv = ldexp(a.inv_scale_rho * a.scale, -ts);
#pragma unroll
        for (int i = 0; i < kNodes; ++i) store_delta<T>(a, tx, ty, tz, lane + i * G, (double)sums[lane + i * G], inv);
    }
    if constexpr (kWide) {
        const double inv = a.inv_scale_rho;
#pragma unroll
        for (int i = 0; i < kNodes; ++i) {
            const int k = lane + i * G;
            store_delta<T>(a, tx, ty, tz, k, (double)(long long)acc[g][acc_slot(k & 7, (k >> 3) & 7, k >> 6)], inv);
        }
    }
}

template <typename T, int TPB, bool SORTED, int NC, bool LIST = false>
__global__ __launch_bounds__(kThreads) void paint_tiles_kernel(PartBatch<T> b, int cur) {
    paint_tiles_body<T, TPB, SORTED, NC, LIST>(b, cur, logical_block(b.xcd));
}

// One lane per ILP particles, particles in Lagrangian order (patch maps), optionally with
// XCD-grouped blocks so neighbouring particle patches (which read the same mesh rows)
// share one L2. With ILP = 2 a lane issues the loads and the 16 corner gathers of both
// its particles before using any of them (more memory requests in flight per wave).
// With COUNT the drifted particle is also counted into its paint bin for the next step
// (the key comes from the very value stored, so the next paint's scatter recomputes it
// bit for bit).
template <typename T, int ILP, bool COUNT>
__global__ __launch_bounds__(kThreads) void matter_kd_kernel(PartBatch<T> b) {
    const int blk = logical_block(b.xcd);
    const int r = real_of(b.map, blk);
    const Particles<T> &a = b.r[r];
    const int n = a.n;
    int idx[ILP], c[ILP][3];
    T f[ILP][3], sv[ILP][3], pv[ILP][3];
    v4<T> g[ILP][8];
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        idx[j] = particle_of((blk - b.map.start[r]) * ILP + j, threadIdx.x, a.lnp, b.pmap);
        if (idx[j] < a.P) particle_cell<T>(a, idx[j], c[j], f[j], sv[j]);
    }
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        if (idx[j] >= a.P) continue;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int z = (c[j][2] + (k >> 2)) & (n - 1);
            const int y = (c[j][1] + ((k >> 1) & 1)) & (n - 1);
            const int x = (c[j][0] + (k & 1)) & (n - 1);
            g[j][k] = a.grad[((size_t)z * n + y) * n + x];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) pv[j][d] = ld_stream(a.p[d] + idx[j]);
    }
#pragma unroll
    for (int j = 0; j < ILP; ++j) {
        if (idx[j] >= a.P) continue;
        cic_kick_drift<T>(f[j], g[j], a.K, a.D, sv[j], pv[j]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            st_stream(pv[j][d], a.p[d] + idx[j]);
            st_stream(sv[j][d], a.s[d] + idx[j]);
        }
    }
    if (COUNT) {
        const int pm = (1 << a.lnp) - 1;
#pragma unroll
        for (int j = 0; j < ILP; ++j) {
            int key = -1;
            if (idx[j] < a.P) {
                const int lat[3] = {idx[j] & pm, (idx[j] >> a.lnp) & pm, idx[j] >> (2 * a.lnp)};
                int cn[3];
                T fn;
#pragma unroll
                for (int d = 0; d < 3; ++d) axis_cell<T>(sv[j][d], lat[d], a.lratio, a.inv_cell, a.n - 1, cn[d], fn);
                key = bin_key(cn, a.lnt);
            }
            wave_aggregated_increment<false>(a.count, key);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Sorted-state run (hrt_run). From the first to the last step of a call the particles are
// kept in paint-bin order, as records (s_x, s_y, s_z, lattice index) plus momenta (3 x P,
// axis-major) in two buffers used in turn:
//   state_scatter  moves the state from the caller's arrays (first step) or from the other
//                  buffer into the bins of its current positions (counts and scan as for
//                  the paint; the order inside a bin is that of the atomics, and no result
//                  depends on it)
//   paint_tiles    reads the records directly (cell and fraction recomputed per particle)
//   kd_tiles       one workgroup per 8^3 tile forms G at the tile's 9^3 corner nodes from a
//                  block of phi in LDS (the differences of the mesh pass) and moves the
//                  tile's particles in place, reading G from LDS; it also counts the moved
//                  particles into the next step's bins
//   state_gather   writes the state back into the caller's arrays at the end.
// A particle's arithmetic (cell, fraction, readout, kick, drift) is the one of the
// Lagrangian-order kernels, so both orders give the same bits. The gain: every particle
// access streams, and G never goes through HBM (only phi, read once per tile with halos).
// (Moving each particle straight into its next bin from the kick-drift, after a counting
// pass, was measured slower at 256^3: the counting pass costs most of a kick-drift.)

// FROM_CALLER: thread (block, lane) takes particle particle_of(...) of the caller's arrays;
// otherwise sorted slot j of buffer 1 - dst. Writes into buffer dst at the bin cursor.
template <typename T, bool FROM_CALLER>
__global__ __launch_bounds__(kThreads) void state_scatter_kernel(PartBatch<T> b, int dst) {
    const int blk = FROM_CALLER ? logical_block(b.xcd) : (int)blockIdx.x;
    const int r = real_of(b.map, blk);
    const Particles<T> &a = b.r[r];
    const size_t P = (size_t)a.P;
    const int i = FROM_CALLER ? particle_of(blk - b.map.start[r], threadIdx.x, a.lnp, b.pmap)
                              : (blk - b.map.start[r]) * kThreads + (int)threadIdx.x;
    int key = -1;
    v4<T> rec;
    T pv[3];
    if (i < a.P) {
        if (FROM_CALLER) {
            rec.x = ld_stream(a.s[0] + i);
            rec.y = ld_stream(a.s[1] + i);
            rec.z = ld_stream(a.s[2] + i);
            rec.w = index_field<T>(i);
#pragma unroll
            for (int d = 0; d < 3; ++d) pv[d] = ld_stream(a.p[d] + i);
        } else {
            rec = a.rec[1 - dst][i];
#pragma unroll
            for (int d = 0; d < 3; ++d) pv[d] = ld_stream(a.mom[1 - dst] + d * P + i);
        }
        int c[3];
        T f[3];
        record_cell<T>(geom_of(a), rec, c, f);
        key = bin_key(c, a.lnt);
    }
    const int slot = wave_aggregated_increment<true>(a.cursor, key);
    if (i < a.P) {
        a.rec[dst][slot] = rec;
#pragma unroll
        for (int d = 0; d < 3; ++d) a.mom[dst][d * P + slot] = pv[d];
    }
}

// phi block of one tile in LDS: x from x0 - 4 (16 values: four aligned quadruples), y and z
// from y0 - 2 and z0 - 2 (13 values), periodic. G is needed at the 9^3 nodes x0..x0+8 (a
// cell's upper corners reach the next tile's first node), fd4 reaches 2 nodes further.
constexpr int kPhiX = 16, kPhiYZ = 13, kGN = 9;
constexpr int kPhiQuads = kPhiYZ * kPhiYZ * (kPhiX / 4);        // 676 aligned quadruples
static_assert(kPhiQuads > 2 * kThreads && kPhiQuads <= 3 * kThreads, "three phi quadruples per lane");

// Mesh offset of quadruple e of tile (tx, ty, tz)'s phi block.
__device__ __forceinline__ size_t phi_quad_offset(int e, int tx, int ty, int tz, int n) {
    const int m = n - 1, q = e & 3, row = e >> 2, ly = row % kPhiYZ, lz = row / kPhiYZ;
    const int gx = (tx * kTile - 4 + 4 * q) & m;
    const int gy = (ty * kTile - 2 + ly) & m, gz = (tz * kTile - 2 + lz) & m;
    return ((size_t)gz * n + gy) * n + gx;
}

// G at the tile's 9^3 nodes from the phi block (every thread of the workgroup calls).
template <typename T>
__device__ __forceinline__ void tile_gradient(const v4<T> *ph4, v4<T> *gl, T inv12cell) {
    // A lane takes four nodes along x (one aligned phi quadruple q = 1..3 of a row (y, z);
    // q = 3 holds only the last node, x = 12) and reads whole quadruples: the row's q - 1,
    // q and q + 1 for the x differences, quadruple q of the rows y +- 1, 2 and z +- 1, 2 for
    // the others. 81 rows x 3 quadruples = 243 lanes, one pass.
    constexpr int kTasks = kGN * kGN * 3;
    const int e = threadIdx.x;
    if (e >= kTasks) return;
    const int q = e % 3 + 1, row = e / 3, gy = row % kGN, gz = row / kGN;
    const int y = gy + 2, z = gz + 2;
    auto quad = [&](int yy, int zz, int qq) { return ph4[(zz * kPhiYZ + yy) * (kPhiX / 4) + qq]; };
    auto el = [](const v4<T> &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; };
    const v4<T> xm = quad(y, z, q - 1), x0 = quad(y, z, q);
    const v4<T> xp = q < 3 ? quad(y, z, q + 1) : x0;          // q = 3 needs only x <= 14
    const v4<T> ym2 = quad(y - 2, z, q), ym1 = quad(y - 1, z, q), yp1 = quad(y + 1, z, q), yp2 = quad(y + 2, z, q);
    const v4<T> zm2 = quad(y, z - 2, q), zm1 = quad(y, z - 1, q), zp1 = quad(y, z + 1, q), zp2 = quad(y, z + 2, q);
    // phi along the row from x = 4q - 4 to 4q + 7
    const T r[12] = {xm.x, xm.y, xm.z, xm.w, x0.x, x0.y, x0.z, x0.w, xp.x, xp.y, xp.z, xp.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int gx = 4 * q + k - 4;                           // node x = 4q + k
        if (gx >= kGN) break;
        v4<T> o;
        o.x = fd4<T>(r[k + 2], r[k + 3], r[k + 5], r[k + 6], inv12cell);
        o.y = fd4<T>(el(ym2, k), el(ym1, k), el(yp1, k), el(yp2, k), inv12cell);
        o.z = fd4<T>(el(zm2, k), el(zm1, k), el(zp1, k), el(zp2, k), inv12cell);
        o.w = T(0);
        gl[(gz * kGN + gy) * kGN + gx] = o;
    }
}

// One particle's state (sorted record and momenta) held in registers between its load and
// its move.
template <typename T>
struct KdItem {
    v4<T> rec;
    T p[3];
};

template <typename T>
__device__ __forceinline__ void kd_fetch(const v4<T> *recs, const T *mom, size_t P, int j, int j1,
                                         KdItem<T> &it) {
    if (j < j1) {
        it.rec = recs[j];
#pragma unroll
        for (int d = 0; d < 3; ++d) it.p[d] = ld_stream(mom + d * P + j);
    }
}

// Readout of G (from LDS) at particle j, kick, drift, store in place; with COUNT the moved
// particle is also counted into its next bin. All 64 lanes of a wave call (j >= j1: none).
// GX: the G block's x width (9 for one tile, 17 for an x-pair of tiles, whose first tile has
// an even tile index, so the cell's x within the pair is its x mod 16).
template <typename T, bool COUNT, int GX = kGN>
__device__ __forceinline__ void kd_move(v4<T> *recs, T *mom, size_t P, int j, int j1, KdItem<T> &it,
                                        const v4<T> *gl, T K, T D, const CellGeom<T> &cg, int lnt,
                                        unsigned int *count) {
    int key = -1;
    if (j < j1) {
        v4<T> rec = it.rec;
        int c[3];
        T f[3];
        record_cell<T>(cg, rec, c, f);
        constexpr int xm = GX == kGN ? 7 : 15;
        const int l0 = ((c[2] & 7) * kGN + (c[1] & 7)) * GX + (c[0] & xm);
        v4<T> g[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = gl[l0 + ((k >> 2) * kGN + ((k >> 1) & 1)) * GX + (k & 1)];
        T sv[3] = {rec.x, rec.y, rec.z};
        cic_kick_drift<T>(f, g, K, D, sv, it.p);
        rec.x = sv[0];
        rec.y = sv[1];
        rec.z = sv[2];
        asm volatile("" : "+v"(rec.w));         // store the whole record: no partial lines
        recs[j] = rec;
#pragma unroll
        for (int d = 0; d < 3; ++d) st_stream(it.p[d], mom + d * P + j);
        if (COUNT) {
            record_cell<T>(cg, rec, c, f);
            key = bin_key(c, lnt);
        }
    }
    if (COUNT) wave_aggregated_increment<false>(count, key);
}


// A phi block of NQ quadruples into LDS by TH lanes: every lane requests all of its
// quadruples before it stores the first, so the block costs one memory latency rather than
// one per pass of the workgroup over it (a store waits for its own load, and the wait
// covers every older request, the particle loads included).
template <typename T, int TH, int NQ, typename Off>
__device__ __forceinline__ void phi_block_load(v4<T> *ph4, const T *phi, Off off) {
    constexpr int R = (NQ + TH - 1) / TH;
    v4<T> v[R];
#pragma unroll
    for (int j = 0; j < R; ++j)
        v[j] = *reinterpret_cast<const v4<T> *>(phi + off(min((int)threadIdx.x + j * TH, NQ - 1)));
#pragma unroll
    for (int j = 0; j < R; ++j)     // all requested before any store (else each load would sink
        asm volatile("" : "+v"(v[j].x), "+v"(v[j].y), "+v"(v[j].z), "+v"(v[j].w));   // into its store's branch)
#pragma unroll
    for (int j = 0; j < R; ++j)
        if ((int)threadIdx.x + j * TH < NQ) ph4[threadIdx.x + j * TH] = v[j];
}

// One workgroup per tile (logical block blk).
template <typename T, bool COUNT>
__global__ __launch_bounds__(kThreads) void kd_tiles_kernel(PartBatch<T> b, int cur) {
    __shared__ v4<T> ph4[kPhiQuads];
    __shared__ v4<T> gl[kGN * kGN * kGN];
    const int blk = logical_block(b.xcd);
    const int rr = real_of(b.map, blk);
    const Particles<T> &a = b.r[rr];
    const int n = a.n, nt = n / kTile;
    const size_t P = (size_t)a.P;
    const int t = blk - b.map.start[rr];
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int j0 = (int)uniform_load(a.offs + t * 8), j1 = (int)uniform_load(a.offs + t * 8 + 8);
    if (j0 == j1) return;                       // empty tile (uniform over the block)
    v4<T> *const recs = a.rec[cur];
    T *const mom = a.mom[cur];
    // A lane handles two particles per trip (j and j + 256). The first trip's state is
    // requested before the phi block, so those loads overlap the G set-up; every later trip
    // requests the next one's before working on its own.
    KdItem<T> cur0, cur1;
    kd_fetch<T>(recs, mom, P, j0 + (int)threadIdx.x, j1, cur0);
    kd_fetch<T>(recs, mom, P, j0 + kThreads + (int)threadIdx.x, j1, cur1);
    phi_block_load<T, kThreads, kPhiQuads>(ph4, a.phi, [&](int e) { return phi_quad_offset(e, tx, ty, tz, n); });
    __syncthreads();
    tile_gradient<T>(ph4, gl, a.inv12cell);
    __syncthreads();
    const T K = a.K, D = a.D;
    const CellGeom<T> cg = geom_of(a);
    const int lnt = a.lnt;
    for (int base = j0; base < j1; base += 2 * kThreads) {   // same trip count for every lane
        KdItem<T> nxt0, nxt1;
        kd_fetch<T>(recs, mom, P, base + 2 * kThreads + (int)threadIdx.x, j1, nxt0);
        kd_fetch<T>(recs, mom, P, base + 3 * kThreads + (int)threadIdx.x, j1, nxt1);
        kd_move<T, COUNT>(recs, mom, P, base + (int)threadIdx.x, j1, cur0, gl, K, D, cg, lnt, a.count);
        kd_move<T, COUNT>(recs, mom, P, base + kThreads + (int)threadIdx.x, j1, cur1, gl, K, D, cg, lnt, a.count);
        cur0 = nxt0;
        cur1 = nxt1;
    }
}

// Two x-adjacent tiles per workgroup of 512 lanes (FP32): tiles 2w and 2w + 1 (their bins
// are contiguous), one phi block of 24 x 13 x 13 and G at the pair's 17 x 9 x 9 corner nodes,
// so the halo is read once for both and the block's load and barrier are paid once per two
// tiles. The differences and every particle's arithmetic are those of kd_tiles_kernel.
constexpr int kPairThreads = 512;
constexpr int kPhiX2 = 24, kGX2 = 17;
constexpr int kPhiQuads2 = kPhiYZ * kPhiYZ * (kPhiX2 / 4);      // 1014 aligned quadruples

__device__ __forceinline__ size_t phi_quad_offset2(int e, int tx0, int ty, int tz, int n) {
    const int m = n - 1, q = e % (kPhiX2 / 4), row = e / (kPhiX2 / 4), ly = row % kPhiYZ, lz = row / kPhiYZ;
    const int gx = (tx0 * kTile - 4 + 4 * q) & m;
    const int gy = (ty * kTile - 2 + ly) & m, gz = (tz * kTile - 2 + lz) & m;
    return ((size_t)gz * n + gy) * n + gx;
}

// The pair's phi block straight into LDS (global_load_lds, 16 bytes a lane: no registers
// and no LDS stores): each request of a wave fills 64 consecutive quadruples, so the block
// is held as 16 rows of 64 (the lanes past its 1014 quadruples repeat the last one into the
// padding). The caller waits for its requests (vmcnt) and then for the workgroup's (barrier).
constexpr int kPhiPad2 = 1024;
template <int TH>
__device__ __forceinline__ void phi_block_to_lds(v4<float> *ph4, const float *phi, int tx, int ty, int tz, int n) {
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = __lane_id();
#pragma unroll
    for (int j = 0; j < kPhiPad2 / TH; ++j) {
        const int row = j * (TH / 64) + w;
        const int e = min(row * 64 + lane, kPhiQuads2 - 1);
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(phi + phi_quad_offset2(e, tx, ty, tz, n)),
            (__attribute__((address_space(3))) void *)(ph4 + row * 64), 16, 0, 0);
    }
}

// G at the pair's 17 x 9 x 9 nodes: a lane takes four nodes along x (quadruple q = 1..5 of a
// row; q = 5 holds only the last node, x = 16): 81 rows x 5 = 405 lanes, one pass.
template <typename T>
__device__ __forceinline__ void pair_gradient(const v4<T> *ph4, v4<T> *gl, T inv12cell) {
    constexpr int kQ = kPhiX2 / 4;
    constexpr int kTasks = kGN * kGN * (kQ - 1);
    const int e = threadIdx.x;
    if (e >= kTasks) return;
    const int q = e % (kQ - 1) + 1, row = e / (kQ - 1), gy = row % kGN, gz = row / kGN;
    const int y = gy + 2, z = gz + 2;
    auto quad = [&](int yy, int zz, int qq) { return ph4[(zz * kPhiYZ + yy) * kQ + qq]; };
    auto el = [](const v4<T> &v, int k) { return k == 0 ? v.x : k == 1 ? v.y : k == 2 ? v.z : v.w; };
    const v4<T> xm = quad(y, z, q - 1), x0 = quad(y, z, q);
    const v4<T> xp = q < kQ - 1 ? quad(y, z, q + 1) : x0;     // q = 5 needs only x <= 22
    const v4<T> ym2 = quad(y - 2, z, q), ym1 = quad(y - 1, z, q), yp1 = quad(y + 1, z, q), yp2 = quad(y + 2, z, q);
    const v4<T> zm2 = quad(y, z - 2, q), zm1 = quad(y, z - 1, q), zp1 = quad(y, z + 1, q), zp2 = quad(y, z + 2, q);
    const T r[12] = {xm.x, xm.y, xm.z, xm.w, x0.x, x0.y, x0.z, x0.w, xp.x, xp.y, xp.z, xp.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int gx = 4 * q + k - 4;
        if (gx >= kGX2) break;
        v4<T> o;
        o.x = fd4<T>(r[k + 2], r[k + 3], r[k + 5], r[k + 6], inv12cell);
        o.y = fd4<T>(el(ym2, k), el(ym1, k), el(yp1, k), el(yp2, k), inv12cell);
        o.z = fd4<T>(el(zm2, k), el(zm1, k), el(zp1, k), el(zp2, k), inv12cell);
        o.w = T(0);
        gl[(gz * kGN + gy) * kGX2 + gx] = o;
    }
}

template <typename T, bool COUNT>
__global__ __launch_bounds__(kPairThreads) void kd_pairs_kernel(PartBatch<T> b, int cur) {
    __shared__ v4<T> ph4[kPhiPad2];
    __shared__ v4<T> gl[kGX2 * kGN * kGN];
    const int blk = logical_block(b.xcd);
    const int rr = real_of(b.map, blk);
    const Particles<T> &a = b.r[rr];
    const int n = a.n, nt = n / kTile;
    const size_t P = (size_t)a.P;
    const int t = 2 * (blk - b.map.start[rr]);          // the pair's first tile (even x)
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int j0 = (int)uniform_load(a.offs + t * 8), j1 = (int)uniform_load(a.offs + t * 8 + 16);
    if (j0 == j1) return;                       // both tiles empty (uniform over the block)
    v4<T> *const recs = a.rec[cur];
    T *const mom = a.mom[cur];
    KdItem<T> cur0, cur1;
    kd_fetch<T>(recs, mom, P, j0 + (int)threadIdx.x, j1, cur0);
    kd_fetch<T>(recs, mom, P, j0 + kPairThreads + (int)threadIdx.x, j1, cur1);
    phi_block_to_lds<kPairThreads>(ph4, a.phi, tx, ty, tz, n);
    __builtin_amdgcn_s_waitcnt(0);              // this wave's requests are in LDS
    __syncthreads();                            // ... and every wave's
    pair_gradient<T>(ph4, gl, a.inv12cell);
    __syncthreads();
    const T K = a.K, D = a.D;
    const CellGeom<T> cg = geom_of(a);
    const int lnt = a.lnt;
    // No request of the next trip ahead (unlike kd_tiles_kernel): the registers it would hold
    // cost a wave per SIMD (71 -> 62 VGPRs, 7 -> 8 waves), which measured faster at every
    // density (256^3 with np = n: 250 -> 239 us; 1024^3 with np = n/2: 6.7 -> 5.7 ms).
    for (int base = j0; base < j1; base += 2 * kPairThreads) {   // same trip count for every lane
        if (base != j0) {
            kd_fetch<T>(recs, mom, P, base + (int)threadIdx.x, j1, cur0);
            kd_fetch<T>(recs, mom, P, base + kPairThreads + (int)threadIdx.x, j1, cur1);
        }
        kd_move<T, COUNT, kGX2>(recs, mom, P, base + (int)threadIdx.x, j1, cur0, gl, K, D, cg, lnt, a.count);
        kd_move<T, COUNT, kGX2>(recs, mom, P, base + kPairThreads + (int)threadIdx.x, j1, cur1, gl, K, D, cg, lnt,
                                a.count);
    }
}

// Mover-list form of kd_pairs_kernel (kd_tiles variants 5 and 6, FP32). The pair's particles
// are the fronts of its 16 bins (one contiguous range of the record buffer named by the
// step's control words; holes skipped) followed by its 16 bins' entries of the side list S
// (one contiguous range). A front particle whose drifted position keeps its bin is stored in
// place; every other particle (a front one that changes bin, which leaves a hole, and every
// entry of S) is appended to the workgroup's part of U, [ubase, ubase + total): its slot
// comes from a workgroup counter in LDS (one LDS atomic per wave), so no global counter is
// contended. With COUNT every particle is counted into the full histogram and U's entries
// into the mover histogram. The arithmetic of a particle is that of kd_move, so the run gives
// the same bits as the other orders.
// G at the 8 corner nodes of pair-frame cell (x, y, z) (x in 0..15, y and z in 0..7),
// formed from the pair's phi block (24 x 13 x 13 values, x from the pair's x0 - 4, y and z
// from y0 - 2 and z0 - 2) with the differences pair_gradient takes at those nodes: the
// same operands in the same order, so the same values as the G block holds.
// The readout, kick and drift of cic_kick_drift (same operations in the same order) with
// each corner's G formed when it is added, so only one corner's values are held at a time.
template <typename T>
__device__ __forceinline__ void cic_kick_drift_phi(const T f[3], const T *ph, int x, int y, int z, T inv12cell, T K,
                                                   T D, T s[3], T p[3]) {
#pragma clang fp contract(off)
    constexpr int SY = kPhiX2, SZ = kPhiYZ * kPhiX2;
    const int n0 = ((z + 2) * kPhiYZ + (y + 2)) * kPhiX2 + (x + 4);
    T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {               // one corner's loads at a time (registers)
        const int n = n0 + (k >> 2) * SZ + ((k >> 1) & 1) * SY + (k & 1);
        const T wz = (k >> 2) ? f[2] : T(1) - f[2];
        const T wyz = wz * (((k >> 1) & 1) ? f[1] : T(1) - f[1]);
        const T w = wyz * ((k & 1) ? f[0] : T(1) - f[0]);
        gx = fmadd(w, fd4<T>(ph[n - 2], ph[n - 1], ph[n + 1], ph[n + 2], inv12cell), gx);
        gy = fmadd(w, fd4<T>(ph[n - 2 * SY], ph[n - SY], ph[n + SY], ph[n + 2 * SY], inv12cell), gy);
        gz = fmadd(w, fd4<T>(ph[n - 2 * SZ], ph[n - SZ], ph[n + SZ], ph[n + 2 * SZ], inv12cell), gz);
    }
    const T gg[3] = {gx, gy, gz};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p[d] = fmadd(K, gg[d], p[d]);
        s[d] = fmadd(D, p[d], s[d]);
    }
}

template <typename T, bool COUNT, bool DIRECT = false>
__device__ __forceinline__ void kd_move_list(v4<T> *rec0, T *mom0, int P, int rF, int mF, int F, int i, int total,
                                             KdItem<T> &it, const v4<T> *gl, T K, T D,
                                             const CellGeom<T> &cg, int lnt, unsigned int *count,
                                             const ListBufs<T> &l, unsigned int *nu, int ub, bool rebuild,
                                             const T *ph = nullptr, T inv12cell = T(0)) {
    int key = -1, okey = -1;
    bool mover = false, live = false;
    const bool front = i < F;
    if (i < total && !(front && rec_index<T>(it.rec) < 0)) {
        live = true;
        int c[3];
        T f[3];
        record_cell<T>(cg, it.rec, c, f);
        okey = bin_key(c, lnt);
        T sv[3] = {it.rec.x, it.rec.y, it.rec.z};
        if constexpr (DIRECT) {
            cic_kick_drift_phi<T>(f, ph, c[0] & 15, c[1] & 7, c[2] & 7, inv12cell, K, D, sv, it.p);
        } else {
            const int l0 = ((c[2] & 7) * kGN + (c[1] & 7)) * kGX2 + (c[0] & 15);
            v4<T> g[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) g[k] = gl[l0 + ((k >> 2) * kGN + ((k >> 1) & 1)) * kGX2 + (k & 1)];
            cic_kick_drift<T>(f, g, K, D, sv, it.p);
        }
        it.rec.x = sv[0];
        it.rec.y = sv[1];
        it.rec.z = sv[2];
        record_cell<T>(cg, it.rec, c, f);
        key = bin_key(c, lnt);
        mover = !front || key != okey;
    }
    // A front input rewrites its slot whole, every step: a stayer with its new state, a mover
    // (now a hole: index -1) or an earlier hole with what it holds, so that no line of the
    // fronts' records and momenta is left partly written (a partial line costs the memory a
    // read before the write). A mover's state also goes to its slot u of U (record 3P + u,
    // axis d at 9P + 2P d + u).
    if (front) {
        v4<T> r = it.rec;
        if (mover) r.w = index_field<T>(-1);
        asm volatile("" : "+v"(r.w));           // store the whole record
        rec0[i + rF] = r;
#pragma unroll
        for (int d = 0; d < 3; ++d) st_stream(it.p[d], mom0 + (i + mF + d * P));
    }
    const unsigned long long mv = __ballot(mover);
    if (mv) {                                   // wave-uniform
        const int lane = __lane_id(), leader = __ffsll((long long)mv) - 1;
        unsigned int base = 0;
        if (lane == leader) base = atomicAdd(nu, (unsigned int)__popcll(mv));
        base = __shfl(base, leader);
        if (mover) {
            const int u = ub + (int)base + __popcll(mv & ((1ull << lane) - 1ull));
            asm volatile("" : "+v"(it.rec.w));
            rec0[3 * P + u] = it.rec;
#pragma unroll
            for (int d = 0; d < 3; ++d) st_stream(it.p[d], mom0 + (9 * P + 2 * P * d + u));
        }
    }
    if (COUNT) {                                // full histogram before a re-binning, else U's
        if (rebuild) wave_aggregated_increment<false>(count, key);
        else wave_aggregated_increment<false>(l.lcount, mover ? key : -1);
    }
}

// Input i of the pair: front slot f0 + i of buffer cur (record i + rF, momenta d P + i + mF
// from rec0 / mom0) for i < F, else entry s0 + i - F of S (record i + rS, momenta
// d P + i + mS).
template <typename T>
__device__ __forceinline__ void kd_fetch_list(const v4<T> *rec0, const T *mom0, int P, int rF, int mF, int rS,
                                              int mS, int F, int i, int total, KdItem<T> &it) {
    if (i < total) {
        const bool front = i < F;
        it.rec = rec0[i + (front ? rF : rS)];
        const int m = i + (front ? mF : mS);
#pragma unroll
        for (int d = 0; d < 3; ++d) it.p[d] = ld_stream(mom0 + (d * P + m));
    }
}

// DIRECT (kd_tiles variant 7, for sparse particle sets): 256 lanes per pair and no G block:
// each particle forms G at its 8 corners from the phi block (corner_gradients), so the
// workgroup holds 16 KB of LDS instead of 38 KB and skips the G set-up and its barrier;
// eight workgroups fit on a CU instead of four. With few particles per pair (np = n/2:
// 128) the per-particle differences cost less than the set-up of all 1377 nodes.
template <typename T, bool COUNT, bool DIRECT = false>
__global__ __launch_bounds__(DIRECT ? 256 : kPairThreads) void kd_pairs_list_kernel(PartBatch<T> b) {
    constexpr int TH = DIRECT ? 256 : kPairThreads;
    __shared__ v4<T> ph4[kPhiPad2];
    __shared__ v4<T> gl[DIRECT ? 1 : kGX2 * kGN * kGN];
    __shared__ unsigned int nu;                 // entries this workgroup appended to U
    const int blk = logical_block(b.xcd);
    const int rr = real_of(b.map, blk);
    const Particles<T> &a = b.r[rr];
    const ListBufs<T> l = list_bufs(a);
    const int n = a.n, nt = n / kTile, P = a.P;
    const int pw = blk - b.map.start[rr];       // pair index
    const int t = 2 * pw;                       // the pair's first tile (even x)
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    const int f0 = (int)uniform_load(a.offs + t * 8), f1 = (int)uniform_load(a.offs + t * 8 + 16);
    const int s0 = (int)uniform_load(l.loffs + t * 8), s1 = (int)uniform_load(l.loffs + t * 8 + 16);
    const int F = f1 - f0, total = F + (s1 - s0);
    if (total == 0) {                           // both tiles empty (uniform over the block)
        if (threadIdx.x == 0) l.ucnt[pw] = 0u;
        return;
    }
    const int cur = (int)uniform_load(&l.ctl[a.par].cur);
    const bool rebuild = uniform_load(&l.ctl[a.par].nlist) > uniform_load(&l.ctl[a.par].limit);
    v4<T> *const rec0 = a.rec[0];
    T *const mom0 = a.mom[0];
    const int rF = (cur ? 2 * P : 0) + f0, mF = (cur ? 6 * P : 0) + f0;
    const int rS = P + s0 - F, mS = 3 * P + s0 - F;
    const int ub = f0 + s0;                     // this workgroup's part of U
    if (threadIdx.x == 0) nu = 0u;
    KdItem<T> c0, c1;
    kd_fetch_list<T>(rec0, mom0, P, rF, mF, rS, mS, F, (int)threadIdx.x, total, c0);
    kd_fetch_list<T>(rec0, mom0, P, rF, mF, rS, mS, F, TH + (int)threadIdx.x, total, c1);
    phi_block_to_lds<TH>(ph4, a.phi, tx, ty, tz, n);
    __builtin_amdgcn_s_waitcnt(0);              // this wave's requests are in LDS
    __syncthreads();                            // ... and every wave's
    if constexpr (!DIRECT) {
        pair_gradient<T>(ph4, gl, a.inv12cell);
        __syncthreads();
    }
    const T *const ph = reinterpret_cast<const T *>(ph4);
    const T K = a.K, D = a.D, inv12 = a.inv12cell;
    const CellGeom<T> cg = geom_of(a);
    const int lnt = a.lnt;
    for (int base = 0; base < total; base += 2 * TH) {   // same trip count for every lane
        if (base != 0) {
            kd_fetch_list<T>(rec0, mom0, P, rF, mF, rS, mS, F, base + (int)threadIdx.x, total, c0);
            kd_fetch_list<T>(rec0, mom0, P, rF, mF, rS, mS, F, base + TH + (int)threadIdx.x, total, c1);
        }
        kd_move_list<T, COUNT, DIRECT>(rec0, mom0, P, rF, mF, F, base + (int)threadIdx.x, total, c0, gl, K, D, cg,
                                       lnt, a.count, l, &nu, ub, rebuild, ph, inv12);
        kd_move_list<T, COUNT, DIRECT>(rec0, mom0, P, rF, mF, F, base + TH + (int)threadIdx.x, total, c1, gl, K, D,
                                       cg, lnt, a.count, l, &nu, ub, rebuild, ph, inv12);
    }
    __syncthreads();
    if (threadIdx.x == 0) {                     // (no global total: one atomic per workgroup on
        l.ubase[pw] = (unsigned int)ub;         // one address serialises at 1024^3, 10^6 of them)
        l.ucnt[pw] = nu;
    }
}

// Before the first step of a mover-list run: control words of the first step's parity
// (fronts in record buffer 0, nothing listed), empty S and mover histogram.
template <typename T>
__global__ __launch_bounds__(256) void list_init_kernel(PartBatch<T> b, int shift) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const ListBufs<T> l = list_bufs(a);
    const int i = (blockIdx.x - b.map.start[r]) * 256 + (int)threadIdx.x;
    if (i < a.nbins) {
        l.lcount[i] = 0u;
        l.loffs[i] = 0u;
    }
    if (i == 0) {
        l.loffs[a.nbins] = 0u;
        ListCtl z{};
        z.limit = (unsigned int)a.P >> shift;
        l.ctl[a.par] = z;
    }
}

// Entries of U: the kick-drift workgroup of pair w appended ucnt[w] of them from ubase[w]
// (record 3P + u, axis d of the momentum at 9P + 2P d + u from rec0 / mom0); the entry's bin
// is formed again from its position, as the kick-drift formed it.
template <typename T>
__device__ __forceinline__ int u_entry(const Particles<T> &a, const CellGeom<T> &cg, int u, v4<T> &rec, T pv[3]) {
    const size_t P = (size_t)a.P;
    rec = a.rec[0][3 * P + u];
#pragma unroll
    for (int d = 0; d < 3; ++d) pv[d] = a.mom[0][9 * P + 2 * d * P + u];
    int c[3];
    T fr[3];
    record_cell<T>(cg, rec, c, fr);
    return bin_key(c, a.lnt);
}

// Settle of a mover-list step, after its kick-drift and the list scan (launch_scan<T,
// true>), which took the same decision: without a re-binning the entries of U go to their
// bins' places in S (list cursors); with one, every particle of the fronts (holes skipped)
// and every entry of U goes to its bin in the other record buffer (bin cursors), which then
// holds the fronts, with no holes and nothing listed. Workgroup 0 writes the next step's
// control words. A fixed grid per realisation (the list's size is only known on the device):
// the fronts in chunks of 1024 consecutive slots per workgroup, four per lane, all loaded
// before any is placed; U one pair per workgroup at a time, likewise.
constexpr int kSettleQ = 4;
constexpr int kSettlePairs = 1024;         // pairs per settle workgroup at most
template <typename T>
__global__ __launch_bounds__(kThreads) void list_settle_kernel(PartBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const ListBufs<T> l = list_bufs(a);
    const ListCtl q = l.ctl[a.par];
    const bool rebuild = list_rebuild(q, a.P);
    const int nb = b.map.start[r + 1] - b.map.start[r];
    const int blk = (int)blockIdx.x - b.map.start[r];
    const long long Pl = a.P;
    const int cur = (int)q.cur, tid = (int)threadIdx.x, npairs = a.nbins / 16;
    const CellGeom<T> cg = geom_of(a);
    constexpr int CH = kSettleQ * kThreads;
    // destination: the other record buffer (re-binning) or S (record P + j, axis d at
    // 3P + d P + j from rec0 / mom0)
    unsigned int *const cursor = rebuild ? a.cursor : l.lcursor;
    v4<T> *const drec = rebuild ? a.rec[1 - cur] : a.rec[0] + a.P;
    T *const dmo = rebuild ? a.mom[1 - cur] : a.mom[0] + 3 * Pl;
    auto place = [&](const int (&key)[kSettleQ], const v4<T> (&rec)[kSettleQ], const T (&pv)[kSettleQ][3]) {
        WaveReservation w[kSettleQ];            // all of a lane's reservations in flight at once
#pragma unroll
        for (int k = 0; k < kSettleQ; ++k) w[k] = wave_reserve(cursor, key[k]);
#pragma unroll
        for (int k = 0; k < kSettleQ; ++k) {
            const int slot = wave_reserved_slot(w[k], key[k]);
            if (key[k] >= 0) {
                drec[slot] = rec[k];
#pragma unroll
                for (int d = 0; d < 3; ++d) dmo[d * Pl + slot] = pv[k][d];
            }
        }
    };
    if (rebuild) {                              // the fronts (whole buffer cur)
        const v4<T> *const srec = a.rec[cur];
        const T *const smo = a.mom[cur];
        for (int base = blk * CH; base < a.P; base += nb * CH) {
            int key[kSettleQ];
            v4<T> rec[kSettleQ];
            T pv[kSettleQ][3];
#pragma unroll
            for (int k = 0; k < kSettleQ; ++k) {
                const int j = base + k * kThreads + tid;
                key[k] = -1;
                if (j < a.P) {
                    rec[k] = srec[j];
#pragma unroll
                    for (int d = 0; d < 3; ++d) pv[k][d] = ld_stream(smo + d * Pl + j);
                }
            }
#pragma unroll
            for (int k = 0; k < kSettleQ; ++k) {
                const int j = base + k * kThreads + tid;
                if (j < a.P && rec_index<T>(rec[k]) >= 0) {
                    int c[3];
                    T f[3];
                    record_cell<T>(cg, rec[k], c, f);
                    key[k] = bin_key(c, a.lnt);
                }
            }
            place(key, rec, pv);
        }
    }
    // U: workgroup blk takes the pairs [p0, p1) (at most kSettlePairs; the grid has at least
    // npairs / kSettlePairs workgroups), lays their entries end to end by a prefix sum of
    // their counts in LDS, and places them 1024 at a time; an entry finds its pair by a
    // binary search over the prefix sums.
    __shared__ int pre[kSettlePairs + 1];
    const int per = (npairs + nb - 1) / nb;
    const int p0 = min(npairs, blk * per), p1 = min(npairs, p0 + per), np = p1 - p0;
    __shared__ int wsum[kThreads / 64];
    int cnt_t[kSettlePairs / kThreads], tot = 0;
#pragma unroll
    for (int k = 0; k < kSettlePairs / kThreads; ++k) {
        const int pi = tid * (kSettlePairs / kThreads) + k;
        cnt_t[k] = pi < np ? (int)l.ucnt[p0 + pi] : 0;
        tot += cnt_t[k];
    }
    int incl = tot;                             // block prefix of the thread totals
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off);
        if (__lane_id() >= off) incl += v;
    }
    if (__lane_id() == 63) wsum[tid >> 6] = incl;
    __syncthreads();
    int run = incl - tot;
    for (int w = 0; w < (tid >> 6); ++w) run += wsum[w];
#pragma unroll
    for (int k = 0; k < kSettlePairs / kThreads; ++k) {
        pre[tid * (kSettlePairs / kThreads) + k] = run;
        run += cnt_t[k];
    }
    int total = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) total += wsum[w];
    if (tid == 0) pre[kSettlePairs] = total;
    __syncthreads();
    for (int c0 = 0; c0 < total; c0 += CH) {
        int key[kSettleQ];
        v4<T> rec[kSettleQ];
        T pv[kSettleQ][3];
#pragma unroll
        for (int k = 0; k < kSettleQ; ++k) {
            const int e = c0 + k * kThreads + tid;
            key[k] = -1;
            if (e < total) {
                int lo = 0, hi = np - 1;        // last pair with pre <= e
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (pre[mid] <= e) lo = mid; else hi = mid - 1;
                }
                const int u = (int)l.ubase[p0 + lo] + (e - pre[lo]);
                key[k] = u_entry<T>(a, cg, u, rec[k], pv[k]);
            }
        }
        place(key, rec, pv);
    }
    if (blk == 0 && tid == 0) {
        // without a re-binning S now holds U's entries: the list scan's total
        const unsigned int listed = rebuild ? 0u : l.loffs[a.nbins];
        ListCtl nx{};
        nx.cur = rebuild ? 1u - q.cur : q.cur;
        nx.nlist = listed;
        nx.holes = listed;                   // every particle outside the fronts is listed
        nx.ucount = 0u;
        nx.rebuilds = q.rebuilds + (rebuild ? 1u : 0u);
        nx.limit = q.limit;
        l.ctl[1 - a.par] = nx;
    }
}

// Requests tile t (realisation rr, sorted slots j0..j1)'s phi block and first 512 particles
// into registers (nothing for an empty tile).
template <typename T>
__device__ __forceinline__ void kd_request(const PartBatch<T> &b, int cur, int rr, int t, int j0, int j1,
                                           v4<T> &f0, v4<T> &f1, v4<T> &f2, KdItem<T> &i0, KdItem<T> &i1) {
    if (j0 == j1) return;                       // uniform
    const Particles<T> &a = b.r[rr];
    const int nt = a.n / kTile;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    kd_fetch<T>(a.rec[cur], a.mom[cur], (size_t)a.P, j0 + (int)threadIdx.x, j1, i0);
    kd_fetch<T>(a.rec[cur], a.mom[cur], (size_t)a.P, j0 + kThreads + (int)threadIdx.x, j1, i1);
    const int e = (int)threadIdx.x;
    f0 = *reinterpret_cast<const v4<T> *>(a.phi + phi_quad_offset(e, tx, ty, tz, a.n));
    f1 = *reinterpret_cast<const v4<T> *>(a.phi + phi_quad_offset(e + kThreads, tx, ty, tz, a.n));
    if (e + 2 * kThreads < kPhiQuads)
        f2 = *reinterpret_cast<const v4<T> *>(a.phi + phi_quad_offset(e + 2 * kThreads, tx, ty, tz, a.n));
}

// Persistent, software-pipelined form: a grid of W resident workgroups, workgroup w taking
// tiles w, w + W, w + 2W, ... (logical numbering, XCD-grouped). While one tile's particles
// are moved, the phi block and first 512 particles of the workgroup's next tile are already
// requested into registers, so a tile's loads wait behind the previous tile's work rather
// than in front of its own. Particles past a tile's first 512 are loaded and moved in trips
// of 256 afterwards. Every tile is still done whole by one workgroup with the same
// arithmetic, so the result is the same bits.
template <typename T, bool COUNT>
__global__ __launch_bounds__(kThreads) void kd_tiles_stream_kernel(PartBatch<T> b, int cur, int nblocks) {
    __shared__ v4<T> ph4[kPhiQuads];
    __shared__ v4<T> gl[kGN * kGN * kGN];
    struct TileRef {
        int rr, t, j0, j1;
    };
    auto tile_at = [&](int L) {
        TileRef q{0, 0, 0, 0};
        if (L < nblocks) {
            q.rr = real_of(b.map, L);
            q.t = L - b.map.start[q.rr];
            q.j0 = (int)uniform_load(b.r[q.rr].offs + q.t * 8);
            q.j1 = (int)uniform_load(b.r[q.rr].offs + q.t * 8 + 8);
        }
        return q;
    };
    v4<T> f0{}, f1{}, f2{};                     // phi quadruples e, e + 256, e + 512 of lane e
    KdItem<T> nx0, nx1;
    const int W = (int)gridDim.x;
    int L = logical_block(b.xcd);
    TileRef cq = tile_at(L);
    kd_request<T>(b, cur, cq.rr, cq.t, cq.j0, cq.j1, f0, f1, f2, nx0, nx1);
    for (; L < nblocks; L += W) {
        const TileRef nq = tile_at(L + W);
        __syncthreads();                        // the previous tile's LDS reads are done
        const bool work = cq.j0 != cq.j1;       // uniform
        if (work) {
            const int e = (int)threadIdx.x;
            ph4[e] = f0;
            ph4[e + kThreads] = f1;
            if (e + 2 * kThreads < kPhiQuads) ph4[e + 2 * kThreads] = f2;
        }
        KdItem<T> c0 = nx0, c1 = nx1;
        kd_request<T>(b, cur, nq.rr, nq.t, nq.j0, nq.j1, f0, f1, f2, nx0, nx1);
        if (work) {
            const Particles<T> &a = b.r[cq.rr];
            const size_t P = (size_t)a.P;
            v4<T> *const recs = a.rec[cur];
            T *const mom = a.mom[cur];
            const T K = a.K, D = a.D;
            const CellGeom<T> cg = geom_of(a);
            const int lnt = a.lnt;
            __syncthreads();
            tile_gradient<T>(ph4, gl, a.inv12cell);
            __syncthreads();
            kd_move<T, COUNT>(recs, mom, P, cq.j0 + (int)threadIdx.x, cq.j1, c0, gl, K, D, cg, lnt, a.count);
            kd_move<T, COUNT>(recs, mom, P, cq.j0 + kThreads + (int)threadIdx.x, cq.j1, c1, gl, K, D, cg, lnt,
                              a.count);
            for (int base = cq.j0 + 2 * kThreads; base < cq.j1; base += kThreads) {
                KdItem<T> it;
                kd_fetch<T>(recs, mom, P, base + (int)threadIdx.x, cq.j1, it);
                kd_move<T, COUNT>(recs, mom, P, base + (int)threadIdx.x, cq.j1, it, gl, K, D, cg, lnt, a.count);
            }
        }
        cq = nq;
    }
}

// The sorted state (buffer cur) goes back to the caller's arrays in two passes. First the
// slot of every particle by lattice index, perm[i] = j (one scattered 4-byte store per
// particle, into the idle record buffer 1 - cur); then in lattice order each lane gathers its
// particle's record and momenta and writes s and p with contiguous stores. Writing s and p
// straight from sorted order would scatter six 4-byte stores per particle over partly
// written lines. Indices outside [0, P) (none in a consistent state) are skipped.
// LIST (mover-list run): the particles are the fronts of the record buffer named by the last
// step's control words (holes skipped: their index is -1) and the entries of U (list_uperm
// below); perm holds P + u for entry u of U.
template <typename T, bool LIST = false>
__global__ __launch_bounds__(kThreads) void state_perm_kernel(PartBatch<T> b, int cur) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const int j = (blockIdx.x - b.map.start[r]) * kThreads + (int)threadIdx.x;
    if (j >= a.P) return;
    if constexpr (LIST) cur = (int)list_bufs(a).ctl[a.par].cur;
    unsigned int *perm = reinterpret_cast<unsigned int *>(a.rec[1 - cur]);
    const int i = rec_index<T>(a.rec[cur][j]);
    if ((unsigned int)i < (unsigned int)a.P) perm[i] = (unsigned int)j;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void list_uperm_kernel(PartBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const Particles<T> &a = b.r[r];
    const ListBufs<T> l = list_bufs(a);
    const int nb = b.map.start[r + 1] - b.map.start[r];
    const int blk = (int)blockIdx.x - b.map.start[r];
    const int cur = (int)l.ctl[a.par].cur;
    unsigned int *perm = reinterpret_cast<unsigned int *>(a.rec[1 - cur]);
    const int lane = __lane_id(), npairs = a.nbins / 16, nwaves = nb * (kThreads / 64);
    for (int w = blk * (kThreads / 64) + (int)(threadIdx.x >> 6); w < npairs; w += nwaves) {
        const int ub = (int)l.ubase[w], cnt = (int)l.ucnt[w];
        for (int k = lane; k < cnt; k += 64) {
            const int i = rec_index<T>(a.rec[0][3 * (size_t)a.P + ub + k]);
            if ((unsigned int)i < (unsigned int)a.P) perm[i] = (unsigned int)(a.P + ub + k);
        }
    }
}

// A workgroup takes a Lagrangian patch of 32 x 8 particles (whole 128-byte lines of s and p;
// their sorted slots lie in a few tiles' bins, whose lines the patch shares), XCD-grouped so
// that neighbouring patches, which gather from the same tiles, share one L2: 568 -> 437 us at
// 256^3 against lattice-linear rows.
template <typename T, bool LIST = false>
__global__ __launch_bounds__(kThreads) void state_gather_kernel(PartBatch<T> b, int cur) {
    const int blk = xcd_block(gridDim.x);
    const int r = real_of(b.map, blk);
    const Particles<T> &a = b.r[r];
    const size_t P = (size_t)a.P;
    const int i = particle_of(blk - b.map.start[r], (int)threadIdx.x, a.lnp, 2);
    if (i >= a.P) return;
    const v4<T> *recs = nullptr;
    const T *mom = nullptr;
    size_t mstride = P;
    if constexpr (LIST) cur = (int)list_bufs(a).ctl[a.par].cur;
    unsigned int j = reinterpret_cast<const unsigned int *>(a.rec[1 - cur])[i];
    if constexpr (LIST) {
        if (j >= (unsigned int)a.P) {           // entry j - P of U
            j -= (unsigned int)a.P;
            if (j >= 2u * (unsigned int)a.P) return;
            recs = a.rec[0] + 3 * P;            // U: record 3P + u, axis d at 9P + 2P d + u
            mom = a.mom[0] + 9 * P;
            mstride = 2 * P;
        }
    }
    if (!recs) {
        if (j >= (unsigned int)a.P) return;
        recs = a.rec[cur];
        mom = a.mom[cur];
    }
    const v4<T> rec = recs[j];
    st_stream(rec.x, a.s[0] + i);
    st_stream(rec.y, a.s[1] + i);
    st_stream(rec.z, a.s[2] + i);
#pragma unroll
    for (int d = 0; d < 3; ++d) st_stream(mom[d * mstride + j], a.p[d] + i);
}

// ---------------------------------------------------------------------------------------
// Reverse mode, matter side (one realisation). matter_vjp_kernel: per particle
// p_bar' = p_bar + D s_bar, s_bar += K (d readout_G / dx)^T p_bar' (the CIC weight
// derivatives against G at the 8 corners), p_bar = p_bar'; the particle is binned again
// exactly as for the paint, and its weights K p_bar' are stored beside its cell fraction.
// gbar_tiles_kernel then pulls, per tile, the weighted CIC contributions K p_bar'_a w_c
// into LDS as 64-bit fixed point (the transpose of the readout, deterministic like the
// paint), adds the rays' part and writes the cotangent of G into the G slot.

template <typename T>
struct MatterAdj {
    Particles<T> a;
    T *sb[3], *pb[3];
    v4<T> *wsorted;
    v4<T> *gout;
    const unsigned long long *gbar;     // rays' part of G_bar_x, G_bar_y (or NULL)
    unsigned long long *maxbits;
    double K, D;
    int hbits;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void matter_vjp_kernel(MatterAdj<T> m) {
    const Particles<T> &a = m.a;
    const int blk = xcd_block(gridDim.x);
    const int i = particle_of(blk, threadIdx.x, a.lnp);
    int key = -1;
    int c[3] = {0, 0, 0};
    T f[3] = {0, 0, 0}, sv[3];
    T kp[3] = {0, 0, 0};
    double big = 0.0;
    if (i < a.P) {
        particle_cell<T>(a, i, c, f, sv);
        key = bin_key(c, a.lnt);
        T pt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) pt[d] = m.pb[d][i] + (T)m.D * m.sb[d][i];
        const int n = a.n;
        // gp[k] = p_bar' . G at corner k (FP64); the derivative of the trilinear weights along
        // axis d pairs corners that differ in d: xb_d = sum over the other two axes of their
        // weights times (gp[upper] - gp[lower])
        double gp[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int z = (c[2] + (k >> 2)) & (n - 1);
            const int y = (c[1] + ((k >> 1) & 1)) & (n - 1);
            const int x = (c[0] + (k & 1)) & (n - 1);
            const v4<T> g = a.grad[((size_t)z * n + y) * n + x];
            gp[k] = (double)pt[0] * (double)g.x + (double)pt[1] * (double)g.y + (double)pt[2] * (double)g.z;
        }
        const double w[3][2] = {{1.0 - (double)f[0], (double)f[0]},
                                {1.0 - (double)f[1], (double)f[1]},
                                {1.0 - (double)f[2], (double)f[2]}};
        double xb[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                xb[0] += w[1][u] * w[2][v] * (gp[(v << 2) | (u << 1) | 1] - gp[(v << 2) | (u << 1)]);
                xb[1] += w[0][u] * w[2][v] * (gp[(v << 2) | 2 | u] - gp[(v << 2) | u]);
                xb[2] += w[0][u] * w[1][v] * (gp[4 | (v << 1) | u] - gp[(v << 1) | u]);
            }
        const double kc = m.K * (double)a.inv_cell;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            m.sb[d][i] += (T)(kc * xb[d]);
            m.pb[d][i] = pt[d];
            kp[d] = (T)(m.K * (double)pt[d]);
            big = fmax(big, fabs((double)kp[d]));
        }
    }
    const int slot = wave_aggregated_increment<true>(a.cursor, key);
    if (i < a.P) {
        const int lcell = ((c[2] & 7) * 8 + (c[1] & 7)) * 8 + (c[0] & 7);
        v4<T> e, w;
        e.x = f[0];
        e.y = f[1];
        e.z = f[2];
        if constexpr (sizeof(T) == 4) e.w = __int_as_float(lcell);
        else e.w = (double)lcell;
        w.x = kp[0];
        w.y = kp[1];
        w.z = kp[2];
        w.w = T(0);
        a.sorted[slot] = e;
        m.wsorted[slot] = w;
    }
    block_max_to(m.maxbits, big);
}

template <typename T>
__global__ __launch_bounds__(256) void cursor_reset_kernel(MatterAdj<T> m) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m.a.nbins) m.a.cursor[i] = m.a.offs[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gbar_tiles_kernel(MatterAdj<T> m) {
    __shared__ unsigned long long acc[3][512];
    __shared__ __align__(16) int rstart[32];
    __shared__ __align__(16) int rpre[32];
    __shared__ __align__(16) signed char rd[32][3];
    const Particles<T> &a = m.a;
    const int t = xcd_block(gridDim.x);
    const int n = a.n, nt = n / kTile;
    const int tx = t % nt, ty = (t / nt) % nt, tz = t / (nt * nt);
    for (int k = threadIdx.x; k < 3 * 512; k += kThreads) acc[k >> 9][k & 511] = 0ull;
    tile_ranges<T>(a, tx, ty, tz, rstart, rpre, rd, threadIdx.x);
    __syncthreads();
    const int total = rpre[27];
    const double scale = adj_fixed_scale(m.maxbits, m.hbits);
    // range index per entry (idx only grows); the next entry is requested before the current
    // one is added, as in the paint
    int r = 0, nr = 0;
    auto entry = [&](int idx, int &rr) {
        while (idx >= rpre[rr + 1]) ++rr;
        return rstart[rr] + (idx - rpre[rr]);
    };
    v4<T> ne{}, nw{};
    if ((int)threadIdx.x < total) {
        const int at = entry(threadIdx.x, nr);
        ne = a.sorted[at];
        nw = m.wsorted[at];
    }
    for (int idx = threadIdx.x; idx < total; idx += kThreads) {
        r = nr;
        const v4<T> e = ne, wv = nw;
        if (idx + kThreads < total) {
            const int at = entry(idx + kThreads, nr);
            ne = a.sorted[at];
            nw = m.wsorted[at];
        }
        const double kw[3] = {(double)wv.x * scale, (double)wv.y * scale, (double)wv.z * scale};
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
            const double wz = cz ? (double)e.z : 1.0 - (double)e.z;
#pragma unroll
            for (int cy = 0; cy < 2; ++cy) {
                const int ny = by + cy;
                if (ny < 0 || ny >= kTile) continue;
                const double wyz = wz * (cy ? (double)e.y : 1.0 - (double)e.y);
#pragma unroll
                for (int cx = 0; cx < 2; ++cx) {
                    const int nx = bx + cx;
                    if (nx < 0 || nx >= kTile) continue;
                    const double w = wyz * (cx ? (double)e.x : 1.0 - (double)e.x);
                    const int node = (nz * kTile + ny) * kTile + nx;
#pragma unroll
                    for (int d = 0; d < 3; ++d)
                        atomicAdd(&acc[d][node], (unsigned long long)llrint(w * kw[d]));
                }
            }
        }
    }
    __syncthreads();
    const double inv = 1.0 / scale;
    const size_t n3 = (size_t)n * n * n;
    for (int k = threadIdx.x; k < 512; k += kThreads) {
        const int x = tx * kTile + (k & 7), y = ty * kTile + ((k >> 3) & 7), z = tz * kTile + (k >> 6);
        const size_t node = ((size_t)z * n + y) * n + x;
        unsigned long long gx = acc[0][k], gy = acc[1][k];
        if (m.gbar) {
            gx += m.gbar[node];
            gy += m.gbar[n3 + node];
        }
        v4<T> o;
        o.x = (T)((double)(long long)gx * inv);
        o.y = (T)((double)(long long)gy * inv);
        o.z = (T)((double)(long long)acc[2][k] * inv);
        o.w = T(0);
        m.gout[node] = o;
    }
}

template <typename T>
void fill_particles(hrt_ctx *c, int r, const hrt_matter &m, Particles<T> &a, double K, double D) {
    const Real &re = c->re[r];
    const int n = re.n, np = re.np;
    for (int d = 0; d < 3; ++d) {
        a.s[d] = static_cast<T *>(m.s[d]);
        a.p[d] = static_cast<T *>(m.p[d]);
    }
    a.count = reinterpret_cast<unsigned int *>(re.ws + re.lay.bins);
    a.offs = a.count + re.lay.nbins;
    a.sums = a.offs + re.lay.nbins + 1;
    a.cursor = reinterpret_cast<unsigned int *>(re.ws + re.lay.cursor);
    a.sorted = reinterpret_cast<v4<T> *>(re.ws + re.lay.sorted);
    a.grad = reinterpret_cast<const v4<T> *>(re.ws + re.lay.grad);
    a.delta = reinterpret_cast<T *>(re.ws + re.lay.mesh_r);
    a.n = n;
    a.lnp = ilog2(np);
    a.lratio = ilog2(n / np);
    a.lnt = ilog2(n / kTile);
    a.P = np * np * np;
    a.nbins = (int)re.lay.nbins;
    a.nblk = (int)((re.lay.nbins + 1023) / 1024);
    a.inv_cell = (T)(1.0 / re.cell);
    a.K = (T)K;
    a.D = (T)D;
    a.scale = std::ldexp(1.0, re.fixed_bits);
    a.fixed_bits = re.fixed_bits;
    a.inv_scale_rho = 1.0 / (a.scale * ((double)a.P / ((double)n * n * n)));
    a.inv12cell = (T)(1.0 / (12.0 * re.cell));
    a.phi = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r) + (size_t)n * n * n;
    a.rec[0] = a.sorted;
    if (re.lay.list) {                  // records [rec0 | S | rec1 | U], momenta [mom0 | S | mom1 | U]
        a.rec[1] = a.sorted + (size_t)2 * a.P;
        a.mom[0] = reinterpret_cast<T *>(re.ws + re.lay.state);
        a.mom[1] = a.mom[0] + (size_t)6 * a.P;
    } else {
        a.rec[1] = re.lay.state ? reinterpret_cast<v4<T> *>(re.ws + re.lay.state) : nullptr;
        a.mom[0] = re.lay.state ? reinterpret_cast<T *>(a.rec[1] + a.P) : nullptr;
        a.mom[1] = re.lay.state ? a.mom[0] + (size_t)3 * a.P : nullptr;
    }
    a.lbase = re.lay.list ? re.ws + re.lay.list : nullptr;
    a.par = 0;
}

template <typename T, typename F>
void set_map(PartBatch<T> &b, int R, F blocks) {
    b.map.R = R;
    b.map.start[0] = 0;
    for (int k = 0; k < R; ++k) b.map.start[k + 1] = b.map.start[k] + blocks(b.r[k]);
}

inline int particle_blocks(int P) { return (P + kThreads - 1) / kThreads; }

// Particle-kernel variant v (0..7): particle map v % 4; v >= 4 flips the kernel's default
// XCD block grouping.
template <typename T>
void set_variant(PartBatch<T> &b, int v, int default_xcd) {
    b.pmap = v % 4;
    b.xcd = (v >= 4) ? 1 - default_xcd : default_xcd;
}

// Paint launch shapes: (tiles per workgroup, FP32 copies of the LDS sums); the first is the
// default (the fastest at one particle per node).
constexpr int kPaintShapes[7][2] = {{2, 2}, {4, 1}, {2, 1}, {1, 1}, {2, 4}, {1, 4}, {1, 8}};

constexpr int kNumPaintShapes = sizeof(kPaintShapes) / sizeof(kPaintShapes[0]);

template <typename T, int I>
void launch_paint_shape(int shape, dim3 grid, hipStream_t st, const PartBatch<T> &b, int cur, bool sorted,
                        bool list = false) {
    if constexpr (I + 1 < kNumPaintShapes) {
        if (shape != I) return launch_paint_shape<T, I + 1>(shape, grid, st, b, cur, sorted, list);
    }
    constexpr int TPB = kPaintShapes[I][0], NC = kPaintShapes[I][1];
    if constexpr (sizeof(T) == 4) {
        if (list) {
            paint_tiles_kernel<T, TPB, true, NC, true><<<grid, kThreads, 0, st>>>(b, cur);
            return;
        }
    }
    if (sorted) paint_tiles_kernel<T, TPB, true, NC><<<grid, kThreads, 0, st>>>(b, cur);
    else paint_tiles_kernel<T, TPB, false, NC><<<grid, kThreads, 0, st>>>(b, cur);
}

// Exclusive scan of the bin counts into offsets and cursors, every realisation of b.
template <typename T, bool LIST = false>
void launch_scan(hrt_ctx *c, PartBatch<T> &b, int R) {
    hipStream_t st = c->stream;
    prof_begin(c);
    set_map(b, R, [](const Particles<T> &a) { return a.nblk; });
    scan_local_kernel<T, LIST><<<b.map.start[R], 256, 0, st>>>(b);
    int max_nblk = 0;
    for (int k = 0; k < R; ++k) max_nblk = std::max(max_nblk, b.r[k].nblk);
    const bool fused = max_nblk <= 1024;
    if (!fused) scan_sums_kernel<T, LIST><<<R, 1024, 0, st>>>(b);
    set_map(b, R, [](const Particles<T> &a) { return (a.nbins + 255) / 256; });
    if (fused) scan_add_kernel<T, true, LIST><<<b.map.start[R], 256, 0, st>>>(b);
    else scan_add_kernel<T, false, LIST><<<b.map.start[R], 256, 0, st>>>(b);
    prof_end(c, K_BIN_SCAN);
}

// Workgroups of the pipelined tile kick-drift that fit on one CU at once (its grid is one
// such wave over all CUs), from the runtime's occupancy calculator (4 if that fails).
template <typename T>
int kd_stream_per_cu(bool count) {
    static int cached[2] = {0, 0};
    int &v = cached[count ? 1 : 0];
    if (v == 0) {
        int nb = 0;
        const hipError_t e =
            count ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kd_tiles_stream_kernel<T, true>, kThreads, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kd_tiles_stream_kernel<T, false>, kThreads, 0);
        v = (e == hipSuccess && nb > 0) ? nb : 4;
    }
    return v;
}

// Workgroups of a persistent tile kernel: per_cu resident per compute unit.
inline int resident_blocks(int per_cu) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return cus * per_cu;
}

template <typename T>
hipError_t paint_impl(hrt_ctx *c, const StepArgs &args) {
    // the sorted state is only ever counted by the previous step's kick-drift
    if (args.state == STATE_SORTED && !args.counts_ready) return hipErrorInvalidValue;
    hipStream_t st = c->stream;
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PartBatch<T> b{};
        for (int k = 0; k < R; ++k) fill_particles<T>(c, r0 + k, args.m[r0 + k], b.r[k], 0.0, 0.0);
        const int cur = args.cur;
        const bool list = args.list && sizeof(T) == 4;
        for (int k = 0; k < R; ++k) b.r[k].par = args.par;
        // mover-list run: after its first step the bins are settled by the previous step's
        // list_settle, so nothing is counted, scanned or scattered here
        if (!(list && args.state == STATE_SORTED)) {
            if (!args.counts_ready) {
                prof_begin(c);
                set_map(b, R, [](const Particles<T> &a) { return (a.nbins + 255) / 256; });
                fill_counts_kernel<T><<<b.map.start[R], 256, 0, st>>>(b);
                set_map(b, R, [](const Particles<T> &a) { return particle_blocks(a.P); });
                set_variant(b, c->variant[K_BIN_COUNT], 0);
                bin_count_kernel<T><<<b.map.start[R], kThreads, 0, st>>>(b);
                prof_end(c, K_BIN_COUNT);
            }
            launch_scan<T>(c, b, R);
            prof_begin(c);
            set_map(b, R, [](const Particles<T> &a) { return particle_blocks(a.P); });
            set_variant(b, c->variant[K_BIN_SCATTER], 0);
            if (args.state == STATE_LAGRANGIAN) {
                bin_scatter_kernel<T><<<b.map.start[R], kThreads, 0, st>>>(b);
                prof_end(c, K_BIN_SCATTER);
            } else if (args.state == STATE_FROM_CALLER) {
                state_scatter_kernel<T, true><<<b.map.start[R], kThreads, 0, st>>>(b, cur);
                prof_end(c, K_STATE_SCATTER);
            } else {
                state_scatter_kernel<T, false><<<b.map.start[R], kThreads, 0, st>>>(b, cur);
                prof_end(c, K_STATE_SCATTER);
            }
        }
        prof_begin(c);
        // variant: bit 0 = no XCD grouping; pv >> 1 = launch shape kPaintShapes[pv >> 1]
        // (tiles per workgroup, FP32 copies of the sums)
        const int pv = c->variant[K_PAINT];
        const bool sorted = args.state != STATE_LAGRANGIAN;
        const int shape = pv >> 1, tpb = kPaintShapes[shape][0];
        set_map(b, R, [tpb](const Particles<T> &a) { const int nt = a.n / kTile; return nt * nt * nt / tpb; });
        b.pmap = 0;
        b.xcd = (pv & 1) == 0 ? 1 : 0;
        const dim3 grid(b.map.start[R]);
        launch_paint_shape<T, 0>(shape, grid, st, b, cur, sorted, list);
        prof_end(c, K_PAINT);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t matter_impl(hrt_ctx *c, const StepArgs &args) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PartBatch<T> b{};
        for (int k = 0; k < R; ++k) {
            const Real &re = c->re[r0 + k];
            fill_particles<T>(c, r0 + k, args.m[r0 + k], b.r[k], re.tab.K[args.step],
                              re.tab.D[args.step]);
        }
        prof_begin(c);
        // with count_next the counts start from zero: the scan of this step's paint cleared them
        if (args.state != STATE_LAGRANGIAN) {
            auto tiles = [](const Particles<T> &a) { const int nt = a.n / kTile; return nt * nt * nt; };
            set_map(b, R, tiles);
            b.pmap = 0;
            b.xcd = 1;
            // FP32: x-pairs of tiles per workgroup unless one tile per workgroup is asked for
            // (the pair's LDS block would exceed 64 KB in FP64)
            const int kdv = c->variant[K_KD_TILES];
            if (sizeof(T) == 4 && args.list) {          // mover-list run (variants 5, 6, 7)
                if constexpr (sizeof(T) == 4) {
                    for (int k = 0; k < R; ++k) b.r[k].par = args.par;
                    set_map(b, R, [](const Particles<T> &a) { const int nt = a.n / kTile; return nt * nt * nt / 2; });
                    const dim3 grid(b.map.start[R]);
                    // G per particle from phi: variant 7, and the automatic choice when every
                    // realisation has at most one particle per 8 mesh nodes (np <= n/2)
                    bool sparse = true;
                    for (int k = 0; k < R; ++k) sparse = sparse && (2 << b.r[k].lnp) <= b.r[k].n;
                    if (kdv == 7 || (kdv == 0 && sparse)) {
                        if (args.count_next) kd_pairs_list_kernel<T, true, true><<<grid, 256, 0, c->stream>>>(b);
                        else kd_pairs_list_kernel<T, false, true><<<grid, 256, 0, c->stream>>>(b);
                    } else if (args.count_next) {
                        kd_pairs_list_kernel<T, true><<<grid, kPairThreads, 0, c->stream>>>(b);
                    } else {
                        kd_pairs_list_kernel<T, false><<<grid, kPairThreads, 0, c->stream>>>(b);
                    }
                }
            } else if (sizeof(T) == 4 && (kdv == 0 || kdv == 4)) {
                if constexpr (sizeof(T) == 4) {
                    set_map(b, R, [](const Particles<T> &a) { const int nt = a.n / kTile; return nt * nt * nt / 2; });
                    const dim3 grid(b.map.start[R]);
                    if (args.count_next) kd_pairs_kernel<T, true><<<grid, kPairThreads, 0, c->stream>>>(b, args.cur);
                    else kd_pairs_kernel<T, false><<<grid, kPairThreads, 0, c->stream>>>(b, args.cur);
                }
            } else if (c->variant[K_KD_TILES] == 3) {          // persistent, software-pipelined form
                const int nblk = b.map.start[R];
                const int grid = std::min(nblk, resident_blocks(kd_stream_per_cu<T>(args.count_next)));
                if (args.count_next) kd_tiles_stream_kernel<T, true><<<grid, kThreads, 0, c->stream>>>(b, args.cur, nblk);
                else kd_tiles_stream_kernel<T, false><<<grid, kThreads, 0, c->stream>>>(b, args.cur, nblk);
            } else if (args.count_next) {
                kd_tiles_kernel<T, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
            } else {
                kd_tiles_kernel<T, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
            }
            prof_end(c, K_KD_TILES);
            continue;
        }
        const int v = c->variant[K_MATTER_KD];
        const int ilp = v >= 8 ? 2 : 1;
        set_map(b, R, [ilp](const Particles<T> &a) { return (particle_blocks(a.P) + ilp - 1) / ilp; });
        set_variant(b, v % 8, 1);
        if (args.count_next) {
            if (ilp == 2) matter_kd_kernel<T, 2, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
            else matter_kd_kernel<T, 1, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        } else {
            if (ilp == 2) matter_kd_kernel<T, 2, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
            else matter_kd_kernel<T, 1, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        }
        prof_end(c, K_MATTER_KD);
    }
    return hipGetLastError();
}

template <typename T>
MatterAdj<T> matter_adj(hrt_ctx *c, int k, const hrt_matter *m, const hrt_matter *mc, int step,
                        const AdjScratch &sc, bool rays) {
    const Real &re = c->re[k];
    MatterAdj<T> ma{};
    fill_particles<T>(c, k, *m, ma.a, 0.0, 0.0);
    if (mc) {
        for (int d = 0; d < 3; ++d) {
            ma.sb[d] = static_cast<T *>(mc->s[d]);
            ma.pb[d] = static_cast<T *>(mc->p[d]);
        }
    }
    ma.wsorted = static_cast<v4<T> *>(sc.wsorted);
    ma.gout = reinterpret_cast<v4<T> *>(re.ws + re.lay.grad);
    ma.gbar = rays ? sc.gbar : nullptr;
    ma.maxbits = sc.maxbits;
    ma.K = re.tab.K[step];
    ma.D = re.tab.D[step];
    ma.hbits = sc.hbits;
    return ma;
}

template <typename T>
hipError_t matter_vjp_impl(hrt_ctx *c, int k, const hrt_matter *m, const hrt_matter *mc, int step,
                           const AdjScratch &sc) {
    const MatterAdj<T> ma = matter_adj<T>(c, k, m, mc, step, sc, false);
    cursor_reset_kernel<T><<<(ma.a.nbins + 255) / 256, 256, 0, c->stream>>>(ma);
    matter_vjp_kernel<T><<<particle_blocks(ma.a.P), kThreads, 0, c->stream>>>(ma);
    return hipGetLastError();
}

template <typename T>
hipError_t gbar_tiles_impl(hrt_ctx *c, int k, bool rays, const AdjScratch &sc) {
    hrt_matter none{};
    const MatterAdj<T> ma = matter_adj<T>(c, k, &none, nullptr, 0, sc, rays);
    const int nt = ma.a.n / kTile;
    gbar_tiles_kernel<T><<<nt * nt * nt, kThreads, 0, c->stream>>>(ma);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_matter_vjp(hrt_ctx *c, int k, const hrt_matter *m, const hrt_matter *mc, int step,
                             const AdjScratch &s) {
    return c->f64 ? matter_vjp_impl<double>(c, k, m, mc, step, s) : matter_vjp_impl<float>(c, k, m, mc, step, s);
}

hipError_t launch_gbar_tiles(hrt_ctx *c, int k, bool rays, const AdjScratch &s) {
    return c->f64 ? gbar_tiles_impl<double>(c, k, rays, s) : gbar_tiles_impl<float>(c, k, rays, s);
}

template <typename T>
hipError_t list_init_impl(hrt_ctx *c, const StepArgs &args) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PartBatch<T> b{};
        for (int k = 0; k < R; ++k) {
            fill_particles<T>(c, r0 + k, args.m[r0 + k], b.r[k], 0.0, 0.0);
            b.r[k].par = args.par;
        }
        set_map(b, R, [](const Particles<T> &a) { return (a.nbins + 1 + 255) / 256; });
        list_init_kernel<T><<<b.map.start[R], 256, 0, c->stream>>>(b, args.list_shift);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t list_settle_impl(hrt_ctx *c, const StepArgs &args) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PartBatch<T> b{};
        for (int k = 0; k < R; ++k) {
            fill_particles<T>(c, r0 + k, args.m[r0 + k], b.r[k], 0.0, 0.0);
            b.r[k].par = args.par;
        }
        launch_scan<T, true>(c, b, R);
        prof_begin(c);
        // up to 2048 workgroups per realisation (eight waves per SIMD on every CU), and at
        // least one per kSettlePairs pairs
        set_map(b, R, [](const Particles<T> &a) {
            return std::max(std::min(2048, particle_blocks(a.P)), (a.nbins / 16 + kSettlePairs - 1) / kSettlePairs);
        });
        list_settle_kernel<T><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        prof_end(c, K_LIST_SETTLE);
    }
    return hipGetLastError();
}

hipError_t launch_list_init(hrt_ctx *c, const StepArgs &a) {
    if (c->f64) return hipErrorInvalidValue;
    return list_init_impl<float>(c, a);
}

hipError_t launch_list_settle(hrt_ctx *c, const StepArgs &a) {
    if (c->f64) return hipErrorInvalidValue;
    return list_settle_impl<float>(c, a);
}

hipError_t launch_paint(hrt_ctx *c, const StepArgs &a) {
    return c->f64 ? paint_impl<double>(c, a) : paint_impl<float>(c, a);
}

hipError_t launch_matter_kd(hrt_ctx *c, const StepArgs &a) {
    return c->f64 ? matter_impl<double>(c, a) : matter_impl<float>(c, a);
}

template <typename T>
hipError_t state_gather_impl(hrt_ctx *c, const StepArgs &args) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PartBatch<T> b{};
        for (int k = 0; k < R; ++k) fill_particles<T>(c, r0 + k, args.m[r0 + k], b.r[k], 0.0, 0.0);
        set_map(b, R, [](const Particles<T> &a) { return particle_blocks(a.P); });
        prof_begin(c);
        if (sizeof(T) == 4 && args.list) {
            for (int k = 0; k < R; ++k) b.r[k].par = args.par;
            state_perm_kernel<T, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
            PartBatch<T> bu = b;
            set_map(bu, R, [](const Particles<T> &a) { return std::max(1, std::min(2048, a.nbins / 16 / 4)); });
            list_uperm_kernel<T><<<bu.map.start[R], kThreads, 0, c->stream>>>(bu);
            state_gather_kernel<T, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
        } else {
            state_perm_kernel<T><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
            state_gather_kernel<T><<<b.map.start[R], kThreads, 0, c->stream>>>(b, args.cur);
        }
        prof_end(c, K_STATE_GATHER);
    }
    return hipGetLastError();
}

hipError_t launch_state_gather(hrt_ctx *c, const StepArgs &a) {
    return c->f64 ? state_gather_impl<double>(c, a) : state_gather_impl<float>(c, a);
}

}  // namespace hrt
