// FFT Poisson solve and gradient of the PM step (paper Sec. 2 Poisson equation; Sec. 5.1:
// the potential gradient is obtained with FFTs once per step).
//
// Hand-written Stockham FFTs (radix 8 where every thread still gets a butterfly, else
// radix 4; one radix-2 stage when needed), one workgroup of 256 threads per batch of lines;
// a pass's first stage reads HBM straight into registers and its last stage writes HBM
// (except where a split step needs whole lines), the stages between work in LDS:
//   x_r2c      real rows -> half spectrum, written transposed as C[kx][z][y]
//              (length-N/2 complex FFT of packed even/odd samples + split step)
//   yz_lines   forward FFT along y (contiguous lines in the transposed layout)
//   z_poisson  forward FFT along z, multiply by -1/(k^2 n^3) (k = 0 -> 0), inverse FFT
//              along z, all in LDS: the spectrum of the potential never leaves the chip
//              between the two z transforms
//   yz_lines   inverse FFT along y
//   x_c2r      half spectrum -> real potential phi [z][y][x]
// then fd4_gradient: G = grad(phi) by fourth-order central differences (the gradient
// reading adopted for this method; it is exact on lattice modes up to its transfer
// function and leaves no Nyquist odd-even artefact next to unresolved sources).
// Realisations of equal mesh size share one launch per pass (block b belongs to
// realisation b / blocks_per_realisation); the gradient covers all realisations at once.
#include <algorithm>

#include "device_common.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;

// In-register DFT of R points in natural order (X[m] = sum_r v[r] W_R^{rm}, W_R = e^{-2 pi i/R},
// conjugate for INV). Radix 8 as 4 x 2: DFT4 over the even and the odd samples, twiddles
// W_8^{m0} on the odd ones (from the LDS table: W_R^q = tw[q * twq]), DFT2 across. Radix 16
// as 4 x 4: DFT4 over each residue n1 of r mod 4, twiddles W_16^{n1 k1}, DFT4 across n1
// (output k1 + 4 k2).
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(c2<T> *v, const c2<T> *__restrict__ tw = nullptr, int twq = 0) {
    if constexpr (R == 16) {
        c2<T> a[4][4];
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) {
            c2<T> t[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
            dft<T, 4, INV>(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) {
                if (n1 * k1 > 0) {
                    c2<T> w = tw[n1 * k1 * twq];
                    if (INV) w.y = -w.y;
                    t[k1] = cmul<T>(t[k1], w);
                }
                a[n1][k1] = t[k1];
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            c2<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
            dft<T, 4, INV>(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    } else if constexpr (R == 8) {
        c2<T> e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft<T, 4, INV>(e);
        dft<T, 4, INV>(o);
#pragma unroll
        for (int m0 = 0; m0 < 4; ++m0) {
            c2<T> b = o[m0];
            if (m0 > 0) {
                c2<T> w = tw[m0 * twq];
                if (INV) w.y = -w.y;
                b = cmul<T>(b, w);
            }
            v[m0] = c2<T>{e[m0].x + b.x, e[m0].y + b.y};
            v[m0 + 4] = c2<T>{e[m0].x - b.x, e[m0].y - b.y};
        }
    } else if constexpr (R == 2) {
        const c2<T> a = v[0], b = v[1];
        v[0] = c2<T>{a.x + b.x, a.y + b.y};
        v[1] = c2<T>{a.x - b.x, a.y - b.y};
    } else {
        const c2<T> a0{v[0].x + v[2].x, v[0].y + v[2].y};
        const c2<T> a1{v[0].x - v[2].x, v[0].y - v[2].y};
        const c2<T> a2{v[1].x + v[3].x, v[1].y + v[3].y};
        const c2<T> d{v[1].x - v[3].x, v[1].y - v[3].y};
        // a3 = d * (-i) forward, d * (+i) inverse
        const c2<T> a3 = INV ? c2<T>{-d.y, d.x} : c2<T>{d.y, -d.x};
        v[0] = c2<T>{a0.x + a2.x, a0.y + a2.y};
        v[2] = c2<T>{a0.x - a2.x, a0.y - a2.y};
        v[1] = c2<T>{a1.x + a3.x, a1.y + a3.y};
        v[3] = c2<T>{a1.x - a3.x, a1.y - a3.y};
    }
}

// Fewest stages for 2^e points with radix-8 stages (and radix 16 when allowed), the last
// one of 2, 4 or 8 points.
__host__ __device__ constexpr int fewest_stages(int e, bool r16) {
    if (e <= 3) return e > 0 ? 1 : 0;
    const int s8 = fewest_stages(e - 3, r16);
    const int s16 = r16 ? fewest_stages(e - 4, r16) : s8;
    return 1 + (s16 < s8 ? s16 : s8);
}
__host__ __device__ constexpr int log2i(int v) { return v > 1 ? 1 + log2i(v / 2) : 0; }

// Radix of the Stockham stage that starts at span Ns: 8 where it keeps every thread busy
// (LINES x L/8 butterflies), else 4, a last 2 when needed; 16 where that also keeps every
// thread busy and saves a stage (a stage is one round trip of the lines through LDS).
template <int L, int LINES>
__host__ __device__ constexpr int radix_at(int Ns) {
    const bool r16 = LINES * (L / 16) >= kThreads;
    const int e = log2i(L / Ns);
    if (r16 && e >= 4 && fewest_stages(e - 4, true) < fewest_stages(e - 3, true)) return 16;
    return (Ns * 8 <= L && LINES * (L / 8) >= kThreads) ? 8 : (Ns * 4 <= L) ? 4 : 2;
}
// Span of the last stage (the one whose outputs are in natural order).
template <int L, int LINES>
__host__ __device__ constexpr int last_span() {
    int Ns = 1;
    while (Ns * radix_at<L, LINES>(Ns) < L) Ns *= radix_at<L, LINES>(Ns);
    return Ns;
}

// Butterfly j of the stage at span Ns: v[r] = x[j + r L/R] on entry; twiddles W_{Ns R}^{kk r}
// (kk = j mod Ns; tw in LDS holds W_n^m, W_L^m = tw[m twmul]) on the inputs, then the R-point
// DFT. Its outputs belong at (j / Ns) Ns R + kk + r Ns.
template <typename T, int L, int R, bool INV, int Ns>
__device__ __forceinline__ void butterfly(c2<T> *v, int j, const c2<T> *__restrict__ tw, int twmul) {
    const int kk = j % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) {
        c2<T> w = tw[(kk * r * (L / (Ns * R))) * twmul];
        if (INV) w.y = -w.y;
        v[r] = cmul<T>(v[r], w);
    }
    dft<T, R, INV>(v, tw, twmul * (L / R));
}

// Position of element i within a line in LDS: one padding element after every 2^SK
// (SK = 0: none), so that the strided writes of the Stockham stages (lane j writing
// j R + r, or groups of Ns consecutive elements Ns R apart) spread over more LDS banks.
template <int SK>
__host__ __device__ constexpr int skw(int i) { return SK ? i + (i >> SK) : i; }

// One Stockham stage over LINES lines of length L in LDS (line stride LS), then the next
// (up to the last stage, or up to but not including it when STOP_BEFORE_LAST).
template <typename T, int L, int LINES, bool INV, int Ns, bool STOP_BEFORE_LAST = false, int SK = 0>
__device__ __forceinline__ void fft_stage(c2<T> *buf, int LS, const c2<T> *__restrict__ tw,
                                          int twmul) {
    if constexpr (Ns < L && !(STOP_BEFORE_LAST && Ns == last_span<L, LINES>())) {
        constexpr int R = radix_at<L, LINES>(Ns);
        constexpr int NB = LINES * (L / R);
        constexpr int BF = (NB + kThreads - 1) / kThreads;
        c2<T> v[BF][R];
#pragma unroll
        for (int k = 0; k < BF; ++k) {
            const int b = threadIdx.x + k * kThreads;
            if (b < NB) {
                const int line = b / (L / R), j = b % (L / R);
                const c2<T> *src = buf + line * LS;
#pragma unroll
                for (int r = 0; r < R; ++r) v[k][r] = src[skw<SK>(j + r * (L / R))];
                butterfly<T, L, R, INV, Ns>(v[k], j, tw, twmul);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BF; ++k) {
            const int b = threadIdx.x + k * kThreads;
            if (b < NB) {
                const int line = b / (L / R), j = b % (L / R);
                const int kk = j % Ns;
                c2<T> *dst = buf + line * LS;
                const int o = (j / Ns) * Ns * R + kk;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[skw<SK>(o + r * Ns)] = v[k][r];
            }
        }
        __syncthreads();
        fft_stage<T, L, LINES, INV, Ns * R, STOP_BEFORE_LAST, SK>(buf, LS, tw, twmul);
    }
}

// Butterfly b of a stage that reads or writes global memory directly: LINE_FAST puts
// consecutive butterflies on consecutive lines (for lines that are strided in memory, so a
// wave's accesses to one element index form contiguous segments), else on consecutive j
// (contiguous lines).
template <int L, int LINES, int R, bool LINE_FAST>
__device__ __forceinline__ void global_bfly(int b, int &line, int &j) {
    if (LINE_FAST) {
        line = b % LINES;
        j = b / LINES;
    } else {
        line = b / (L / R);
        j = b % (L / R);
    }
}

// First stage with its inputs read from global memory: ld(line, m) is element m of the
// block's line `line` (never called for lines with !valid(line)); the outputs go to LDS.
// The loads are issued first, then the block synchronises (which also makes the twiddles
// the caller staged visible), then the butterflies run.
template <typename T, int L, int LINES, bool INV, bool LINE_FAST, int SK = 0, class Ld, class Valid>
__device__ __forceinline__ void first_stage_global(c2<T> *buf, int LS, const c2<T> *__restrict__ tw,
                                                   int twmul, Ld ld, Valid valid) {
    constexpr int R = radix_at<L, LINES>(1);
    constexpr int NB = LINES * (L / R);
    constexpr int BF = (NB + kThreads - 1) / kThreads;
    c2<T> v[BF][R];
#pragma unroll
    for (int k = 0; k < BF; ++k) {
        const int b = threadIdx.x + k * kThreads;
        int line, j;
        global_bfly<L, LINES, R, LINE_FAST>(b, line, j);
        if (b < NB && valid(line)) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[k][r] = ld(line, j + r * (L / R));
        }
    }
    __syncthreads();                            // twiddles staged by the caller
#pragma unroll
    for (int k = 0; k < BF; ++k) {
        const int b = threadIdx.x + k * kThreads;
        int line, j;
        global_bfly<L, LINES, R, LINE_FAST>(b, line, j);
        if (b < NB && valid(line)) {
            butterfly<T, L, R, INV, 1>(v[k], j, tw, twmul);
            c2<T> *dst = buf + line * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) dst[skw<SK>(j * R + r)] = v[k][r];
        }
    }
    __syncthreads();
}

// Last stage, inputs from LDS, outputs handed to st(line, m, value) in natural order m
// (never for lines with !valid(line)). With SYNC the block synchronises between reading
// and handing out (for a st that writes the same LDS buffer).
template <typename T, int L, int LINES, bool INV, bool LINE_FAST, bool SYNC, int SK = 0, class St, class Valid>
__device__ __forceinline__ void last_stage_out(const c2<T> *buf, int LS, const c2<T> *__restrict__ tw,
                                               int twmul, St st, Valid valid) {
    constexpr int Ns = last_span<L, LINES>();
    constexpr int R = radix_at<L, LINES>(Ns);
    static_assert(Ns * R == L, "last stage spans the line");
    constexpr int NB = LINES * (L / R);
    constexpr int BF = (NB + kThreads - 1) / kThreads;
    c2<T> v[BF][R];
#pragma unroll
    for (int k = 0; k < BF; ++k) {
        const int b = threadIdx.x + k * kThreads;
        int line, j;
        global_bfly<L, LINES, R, LINE_FAST>(b, line, j);
        if (b < NB && valid(line)) {
            const c2<T> *src = buf + line * LS;
#pragma unroll
            for (int r = 0; r < R; ++r) v[k][r] = src[skw<SK>(j + r * (L / R))];
            butterfly<T, L, R, INV, Ns>(v[k], j, tw, twmul);
        }
    }
    if (SYNC) __syncthreads();
#pragma unroll
    for (int k = 0; k < BF; ++k) {
        const int b = threadIdx.x + k * kThreads;
        int line, j;
        global_bfly<L, LINES, R, LINE_FAST>(b, line, j);
        if (b < NB && valid(line)) {
#pragma unroll
            for (int r = 0; r < R; ++r) st(line, j + r * Ns, v[k][r]);
        }
    }
}

// Stage the N twiddles W_N^m (every tws-th entry of the table) in LDS; the caller's next
// __syncthreads makes them visible.
template <typename T, int N>
__device__ __forceinline__ void stage_twiddles(c2<T> *stw, const c2<T> *__restrict__ tw, int tws) {
    for (int j = threadIdx.x; j < N; j += kThreads) stw[j] = tw[j * tws];
}

// Work per block (complex values staged in LDS). Small blocks keep many blocks resident per
// CU, so one block's loads overlap other blocks' LDS stages (measured on gfx950 at 256^3:
// 2048 values for the x passes, 1024 for y and 2048 for z were fastest). The x passes
// write (read) the spectrum transposed and the z pass reads strided rows, so both keep 16
// (x) and 8 (z) lines per block, 128- and 64-byte segments, while that fits in 32 KB of LDS
// (4096 FP32 complex values); larger meshes take fewer lines rather than fewer resident
// blocks (at 1024^3: 8 and 4 lines), and the XCD-grouped block order of these passes
// puts the blocks that share a segment's line on one L2.
template <typename T, int N>
struct Cfg {
    static constexpr int F = sizeof(T) == 4 ? 1 : 2;
    static constexpr int EXW = (2048 / F > 16 * N / (2 * F)) ? 2048 / F : 16 * N / (2 * F);
    static constexpr int EXC = (4096 / F > N / 2) ? 4096 / F : N / 2;
    static constexpr int EX = EXW < EXC ? EXW : EXC;
    static constexpr int EY = (1024 / F > N) ? 1024 / F : N;
    static constexpr int EZW = (2048 / F > 8 * N / F) ? 2048 / F : 8 * N / F;
    static constexpr int EZC = (4096 / F > N) ? 4096 / F : N;
    static constexpr int EZ = EZW < EZC ? EZW : EZC;
    static constexpr int XROWS = (EX / (N / 2)) < 1 ? 1 : ((EX / (N / 2)) < N * N ? EX / (N / 2) : N * N);
    // x_c2r reads the transposed spectrum in segments of XROWS values: at N >= 1024 twice
    // the rows (128-byte FP32 segments, 64 KB of LDS) measured faster than more blocks
    static constexpr int XROWS_INV = N >= 1024 ? 2 * XROWS : XROWS;
    static constexpr int YLINES = EY / N < 1 ? 1 : EY / N;
    // LDS padding of the lines (skw): one element per 32 in FP32 (measured on gfx950: z pass
    // 38.5 -> 34.6 us, x_c2r 27.2 -> 25.1 us at 256^3; every pass 1-5 % faster at 1024^3);
    // x_r2c only from N = 512 on (at 256^3 its rows measured 30.4 us unpadded, 32.2 padded)
    static constexpr int SK = sizeof(T) == 4 && N >= 64 ? 5 : 0;
    static constexpr int SKX = sizeof(T) == 4 && N >= 512 ? 5 : 0;
    static constexpr int ZLINES = EZ / N < 1 ? 1 : EZ / N;
};

// Per-launch arguments of the FFT passes: realisations of one mesh size N.
template <typename T>
struct FftBatch {
    const T *rin[kMaxBatch];       // x_r2c input rows
    T *rout[kMaxBatch];            // x_c2r output rows
    c2<T> *spec[kMaxBatch];        // transposed spectrum [kx][z][y]
    const c2<T> *tw[kMaxBatch];    // twiddles W_table^m
    double kf2[kMaxBatch];         // (2 pi / box)^2
    int tws;                       // twiddle-table stride (table size / N)
    int bpr;                       // blocks per realisation
};

// tws: stride of the twiddle table (its size over N) when transforming a lattice smaller
// than the mesh the table was built for.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void x_r2c_kernel(FftBatch<T> fb) {
    constexpr int L = N / 2, ROWS = Cfg<T, N>::XROWS, SK = Cfg<T, N>::SKX, LS = skw<SK>(L) + 1;
    __shared__ c2<T> buf[ROWS * LS];
    __shared__ c2<T> tw[N];
    // XCD-grouped block order only when a block's transposed segments are under 128 bytes
    const int blk = ROWS * (int)sizeof(c2<T>) < 128 ? xcd_block(gridDim.x) : (int)blockIdx.x;
    const int r = blk / fb.bpr;
    const T *__restrict__ in = fb.rin[r];
    c2<T> *__restrict__ out = fb.spec[r];
    const int row0 = (blk % fb.bpr) * ROWS;
    stage_twiddles<T, N>(tw, fb.tw[r], fb.tws);
    auto ld = [&](int rr, int m) { return reinterpret_cast<const c2<T> *>(in + (size_t)(row0 + rr) * N)[m]; };
    if constexpr (last_span<L, ROWS>() > 1) {
        // the first stage reads the packed rows from HBM directly, the rest run in LDS
        first_stage_global<T, L, ROWS, false, false, SK>(buf, LS, tw, N / L, ld, [](int) { return true; });
        fft_stage<T, L, ROWS, false, radix_at<L, ROWS>(1), false, SK>(buf, LS, tw, N / L);
    } else {                                    // one stage (N = 16): staged through LDS
        for (int e = threadIdx.x; e < ROWS * L; e += kThreads) buf[(e / L) * LS + skw<SK>(e % L)] = ld(e / L, e % L);
        __syncthreads();
        fft_stage<T, L, ROWS, false, 1, false, SK>(buf, LS, tw, N / L);
    }
    // split step: X[k] = (Z[k] + conj Z[L-k])/2 - (i/2) W_N^k (Z[k] - conj Z[L-k]),
    // each thread owns the pair (k, L-k); X[L] (Nyquist) comes from Z[0].
    for (int e = threadIdx.x; e < ROWS * (L / 2 + 1); e += kThreads) {
        const int rr = e / (L / 2 + 1), k = e % (L / 2 + 1);
        c2<T> *line = buf + rr * LS;
        const c2<T> zk = line[skw<SK>(k)];
        const c2<T> zp = line[skw<SK>(k == 0 ? 0 : L - k)];
        const c2<T> w = tw[k];
        // A = zk + conj(zp), B = zk - conj(zp); X[k] = A/2 - (i/2) w B
        const c2<T> A{zk.x + zp.x, zk.y - zp.y}, B{zk.x - zp.x, zk.y + zp.y};
        const c2<T> wB = cmul<T>(w, B);
        line[skw<SK>(k)] = c2<T>{T(0.5) * (A.x + wB.y), T(0.5) * (A.y - wB.x)};
        if (k == 0) {
            line[skw<SK>(L)] = c2<T>{T(0.5) * (A.x - wB.y), T(0.5) * (A.y + wB.x)};   // W_N^L = -1
        } else if (k != L - k) {
            // X[L-k] = A'/2 - (i/2) W_N^{L-k} B', A' = conj(A), B' = -conj(B), W_N^{L-k} = -conj(w)
            const c2<T> Ap{A.x, -A.y}, Bp{-B.x, B.y}, wp{-w.x, w.y};
            const c2<T> wBp = cmul<T>(wp, Bp);
            line[skw<SK>(L - k)] = c2<T>{T(0.5) * (Ap.x + wBp.y), T(0.5) * (Ap.y - wBp.x)};
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ROWS * (L + 1); e += kThreads) {
        const int kx = e / ROWS, rr = e % ROWS;
        const int row = row0 + rr, z = row / N, y = row % N;
        out[((size_t)kx * N + z) * N + y] = buf[rr * LS + skw<SK>(kx)];
    }
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void x_c2r_kernel(FftBatch<T> fb) {
    constexpr int L = N / 2, ROWS = Cfg<T, N>::XROWS_INV, SK = Cfg<T, N>::SK, LS = skw<SK>(L) + 1;
    __shared__ c2<T> buf[ROWS * LS];
    __shared__ c2<T> tw[N];
    // XCD-grouped block order only when a block's transposed segments are under 128 bytes
    const int blk = ROWS * (int)sizeof(c2<T>) < 128 ? xcd_block(gridDim.x) : (int)blockIdx.x;
    const int r = blk / fb.bpr;
    const c2<T> *__restrict__ in = fb.spec[r];
    T *__restrict__ out = fb.rout[r];
    const int row0 = (blk % fb.bpr) * ROWS;
    stage_twiddles<T, N>(tw, fb.tw[r], fb.tws);
    // Z[k] = (X[k] + conj X[L-k]) + i W_N^{-k} (X[k] - conj X[L-k]), pairs (k, L-k), read
    // straight from the transposed spectrum (consecutive lanes on consecutive rows of one k,
    // so a wave's loads form segments of ROWS values); the loads go out before the barrier
    // that makes the twiddles visible.
    constexpr int NP = ROWS * (L / 2 + 1), PI = (NP + kThreads - 1) / kThreads;
    auto get = [&](int rr, int kx) {
        const int row = row0 + rr, z = row / N, y = row % N;
        return in[((size_t)kx * N + z) * N + y];
    };
    c2<T> xk[PI], xp[PI];
#pragma unroll
    for (int q = 0; q < PI; ++q) {
        const int e = (int)threadIdx.x + q * kThreads;
        if (e < NP) {
            const int rr = e % ROWS, k = e / ROWS;
            xk[q] = get(rr, k);
            xp[q] = get(rr, L - k);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PI; ++q) {
        const int e = (int)threadIdx.x + q * kThreads;
        if (e < NP) {
            const int rr = e % ROWS, k = e / ROWS;
            c2<T> *line = buf + rr * LS;
            const c2<T> w = tw[k];
            const c2<T> wc{w.x, -w.y};
            const c2<T> A{xk[q].x + xp[q].x, xk[q].y - xp[q].y}, B{xk[q].x - xp[q].x, xk[q].y + xp[q].y};
            const c2<T> wB = cmul<T>(wc, B);
            line[skw<SK>(k)] = c2<T>{A.x - wB.y, A.y + wB.x};
            if (k != 0 && k != L - k) {
                // Z[L-k] = conj(A) + i (-w) (-conj(B))
                const c2<T> Ap{A.x, -A.y}, Bp{-B.x, B.y}, wp{-w.x, -w.y};
                const c2<T> wBp = cmul<T>(wp, Bp);
                line[skw<SK>(L - k)] = c2<T>{Ap.x - wBp.y, Ap.y + wBp.x};
            }
        }
    }
    __syncthreads();
    auto st = [&](int rr, int m, const c2<T> &v) { reinterpret_cast<c2<T> *>(out + (size_t)(row0 + rr) * N)[m] = v; };
    if constexpr (last_span<L, ROWS>() > 1) {
        // all stages but the last in LDS; the last writes the rows of phi to HBM directly
        fft_stage<T, L, ROWS, true, 1, true, SK>(buf, LS, tw, N / L);
        last_stage_out<T, L, ROWS, true, false, false, SK>(buf, LS, tw, N / L, st, [](int) { return true; });
    } else {                                    // one stage (N = 16): staged through LDS
        fft_stage<T, L, ROWS, true, 1, false, SK>(buf, LS, tw, N / L);
        for (int e = threadIdx.x; e < ROWS * L; e += kThreads) st(e / L, e % L, buf[(e / L) * LS + skw<SK>(e % L)]);
    }
}

// FFT along y of the transposed spectrum C[kx][z][y]: lines are contiguous. The first
// stage reads the lines from HBM and the last writes them back (no staging pass through
// LDS); the stages in between work in LDS.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void y_lines_kernel(FftBatch<T> fb) {
    constexpr int LINES = Cfg<T, N>::YLINES, SK = Cfg<T, N>::SK, LS = skw<SK>(N) + 1;
    constexpr int TOTAL = (N / 2 + 1) * N;
    static_assert(last_span<N, LINES>() > 1, "at least two stages");
    __shared__ c2<T> buf[LINES * LS];
    __shared__ c2<T> tw[N];
    const int r = blockIdx.x / fb.bpr;
    c2<T> *__restrict__ data = fb.spec[r];
    const int l0 = (blockIdx.x % fb.bpr) * LINES;
    stage_twiddles<T, N>(tw, fb.tw[r], fb.tws);
    auto valid = [&](int li) { return l0 + li < TOTAL; };
    first_stage_global<T, N, LINES, INV, false, SK>(
        buf, LS, tw, 1, [&](int li, int m) { return data[(size_t)(l0 + li) * N + m]; }, valid);
    fft_stage<T, N, LINES, INV, radix_at<N, LINES>(1), true, SK>(buf, LS, tw, 1);
    last_stage_out<T, N, LINES, INV, false, false, SK>(
        buf, LS, tw, 1, [&](int li, int m, const c2<T> &v) { data[(size_t)(l0 + li) * N + m] = v; },
        valid);
}

// FFT along z; MODE 0: forward, 1: inverse, 2: forward, multiply by -1/(k^2 n^3) (k = 0
// -> 0), inverse. Line l = kx * N + y, element stride N. The first stage reads HBM and the
// last writes it (consecutive lanes on consecutive lines: LINES consecutive y form one
// contiguous segment per z); MODE 2 applies the multiply to the forward transform's last
// stage as it writes LDS. Line stride N + 9 (complex) spreads the line-strided and the
// Stockham accesses over the LDS banks.
template <typename T, int N, int MODE>
__global__ __launch_bounds__(kThreads) void z_lines_kernel(FftBatch<T> fb) {
    constexpr int LINES = Cfg<T, N>::ZLINES, SK = Cfg<T, N>::SK, LS = SK ? skw<SK>(N) + 1 : N + 9;
    constexpr int TOTAL = (N / 2 + 1) * N;
    static_assert(last_span<N, LINES>() > 1, "at least two stages");
    __shared__ c2<T> buf[LINES * LS];
    __shared__ c2<T> tw[N];
    // A block's rows are LINES consecutive y (LINES x 8 bytes of a 128-byte line in FP32):
    // XCD-grouped block order puts the blocks that share those lines on one XCD, so each line
    // comes from HBM once rather than once per XCD.
    const int blk = xcd_block(gridDim.x);
    const int r = blk / fb.bpr;
    c2<T> *__restrict__ data = fb.spec[r];
    const int l0 = (blk % fb.bpr) * LINES;
    stage_twiddles<T, N>(tw, fb.tw[r], fb.tws);
    auto at = [&](int li, int z) {
        const int l = l0 + li;
        return ((size_t)(l / N) * N + z) * N + (l % N);
    };
    auto valid = [&](int li) { return l0 + li < TOTAL; };
    auto store = [&](int li, int z, const c2<T> &v) { data[at(li, z)] = v; };
    first_stage_global<T, N, LINES, MODE == 1, true, SK>(
        buf, LS, tw, 1, [&](int li, int z) { return data[at(li, z)]; }, valid);
    fft_stage<T, N, LINES, MODE == 1, radix_at<N, LINES>(1), true, SK>(buf, LS, tw, 1);
    if constexpr (MODE == 2) {
        const double kf2 = fb.kf2[r], inv_n3 = 1.0 / ((double)N * N * N);
        last_stage_out<T, N, LINES, false, false, true, SK>(
            buf, LS, tw, 1,
            [&](int li, int kz, const c2<T> &v) {
                const int l = l0 + li, kx = l / N, ky = l % N;
                const int fy = ky <= N / 2 ? ky : ky - N, fz = kz <= N / 2 ? kz : kz - N;
                const double k2 = kf2 * (double)(kx * kx + fy * fy + fz * fz);
                const T g = k2 > 0.0 ? (T)(-inv_n3 / k2) : T(0);
                buf[li * LS + skw<SK>(kz)] = c2<T>{v.x * g, v.y * g};
            },
            valid);
        __syncthreads();
        fft_stage<T, N, LINES, true, 1, true, SK>(buf, LS, tw, 1);
        last_stage_out<T, N, LINES, true, true, false, SK>(buf, LS, tw, 1, store, valid);
    } else {
        last_stage_out<T, N, LINES, MODE == 1, true, false, SK>(buf, LS, tw, 1, store, valid);
    }
}

template <typename T>
struct GradR {
    const T *phi;
    v4<T> *g;
    int n, log2n;
    T inv12cell;
};
template <typename T>
struct GradBatch {
    BlockMap map;
    GradR<T> r[kMaxBatch];
};

// One lane per node, x fastest; blocks XCD-remapped so the +-2 neighbour rows and
// planes a block reads are mostly in its own XCD's L2.
template <typename T>
__global__ __launch_bounds__(kThreads) void fd4_gradient_kernel(GradBatch<T> b) {
    const int blk = xcd_block(gridDim.x);
    const int r = real_of(b.map, blk);
    const GradR<T> &a = b.r[r];
    const int64_t idx = (int64_t)(blk - b.map.start[r]) * kThreads + threadIdx.x;
    const int n = a.n, log2n = a.log2n;
    if (idx >= ((int64_t)1 << (3 * log2n))) return;
    const T *__restrict__ phi = a.phi;
    const int m = n - 1;
    const int x = (int)(idx & m), y = (int)((idx >> log2n) & m), z = (int)(idx >> (2 * log2n));
    const size_t row = ((size_t)z * n + y) * n;
    auto at = [&](int xx, int yy, int zz) {
        return phi[(((size_t)(zz & m) * n + (yy & m)) * n) + (xx & m)];
    };
    v4<T> out;
    out.x = fd4<T>(phi[row + ((x - 2) & m)], phi[row + ((x - 1) & m)], phi[row + ((x + 1) & m)],
                   phi[row + ((x + 2) & m)], a.inv12cell);
    out.y = fd4<T>(at(x, y - 2, z), at(x, y - 1, z), at(x, y + 1, z), at(x, y + 2, z), a.inv12cell);
    out.z = fd4<T>(at(x, y, z - 2), at(x, y, z - 1), at(x, y, z + 1), at(x, y, z + 2), a.inv12cell);
    out.w = T(0);
    a.g[idx] = out;
}

// The lens planes of one step (Sec. 5.2: the mesh points in the shell): entry e of the
// step's plane list holds, for every node (u, v) of line-of-sight plane j in the frame of
// its replica, the transverse gradient (G_u, G_v) of phi by the fourth-order differences of
// fd4_gradient_kernel. A replica row maps replica node (u, v, w = plane index in the
// replica) to box node x[perm[a]] = sign[a] u[a] + shift[perm[a]] (mod n), and the
// difference along replica axis a reads phi at x + sign[a] * k * e_perm[a], k = -2..2, so
// a mirrored axis gives the exact negative of the box difference. One lane per node, u
// fastest; the stack is [e][v][u] pairs of the dtype, read by the ray kernels.
template <typename T>
struct PlaneGradR {
    const T *phi;
    const T *delta;
    c2<T> *stack;
    T *sphi, *sdelta;          // scalar lens planes of phi and delta (NULL when not needed)
    const PlaneEntry *planes;
    const int32_t *reps;       // replica rows, 9 values each
    int n, log2n, begin, count, identity;
    T inv12cell;
};
template <typename T>
struct PlaneGradBatch {
    BlockMap map;
    PlaneGradR<T> r[kMaxBatch];
};

template <typename T>
__global__ __launch_bounds__(kThreads) void plane_gradient_kernel(PlaneGradBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const PlaneGradR<T> &a = b.r[r];
    const int n = a.n, log2n = a.log2n, m = n - 1;
    const int64_t idx = (int64_t)(blockIdx.x - b.map.start[r]) * kThreads + threadIdx.x;
    const int e = (int)(idx >> (2 * log2n));
    if (e >= a.count) return;
    const PlaneEntry pe = a.planes[a.begin + e];
    const int u = (int)(idx & m), v = (int)((idx >> log2n) & m), w = pe.mesh;
    const T *__restrict__ phi = a.phi;
    auto at = [&](int xx, int yy, int zz) {
        return phi[(((size_t)(zz & m) * n + (yy & m)) * n) + (xx & m)];
    };
    c2<T> out;
    int xb[3] = {u, v, w};                     // box node of replica node (u, v, w)
    if (a.identity) {
        out.x = fd4<T>(at(u - 2, v, w), at(u - 1, v, w), at(u + 1, v, w), at(u + 2, v, w), a.inv12cell);
        out.y = fd4<T>(at(u, v - 2, w), at(u, v - 1, w), at(u, v + 1, w), at(u, v + 2, w), a.inv12cell);
    } else {
        const int32_t *row = a.reps + 9 * pe.rep;
        const int uu[3] = {u, v, w};
        for (int ax = 0; ax < 3; ++ax) xb[row[ax]] = row[3 + ax] * uu[ax] + row[6 + row[ax]];
        auto along = [&](int ax, int k) {          // phi at replica node u + k e_ax
            int c[3] = {xb[0], xb[1], xb[2]};
            c[row[ax]] += row[3 + ax] * k;
            return at(c[0], c[1], c[2]);
        };
        out.x = fd4<T>(along(0, -2), along(0, -1), along(0, 1), along(0, 2), a.inv12cell);
        out.y = fd4<T>(along(1, -2), along(1, -1), along(1, 1), along(1, 2), a.inv12cell);
    }
    a.stack[idx] = out;
    if (a.sphi) a.sphi[idx] = at(xb[0], xb[1], xb[2]);
    if (a.sdelta)
        a.sdelta[idx] = a.delta[(((size_t)(xb[2] & m) * n + (xb[1] & m)) * n) + (xb[0] & m)];
}

template <typename T, int N>
FftBatch<T> fft_batch(hrt_ctx *c, const std::vector<int> &ids, int bpr, int tws) {
    FftBatch<T> fb{};
    fb.tws = tws;
    fb.bpr = bpr;
    for (size_t k = 0; k < ids.size(); ++k) {
        const Real &re = c->re[ids[k]];
        const size_t n3 = (size_t)re.n * re.n * re.n;
        fb.rin[k] = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r);
        fb.rout[k] = reinterpret_cast<T *>(re.ws + re.lay.mesh_r) + n3;
        fb.spec[k] = reinterpret_cast<c2<T> *>(re.ws + re.lay.spec);
        fb.tw[k] = reinterpret_cast<const c2<T> *>(re.ws + re.lay.twiddle);
        const double kf = 2.0 * 3.14159265358979323846 / re.box;
        fb.kf2[k] = kf * kf;
    }
    return fb;
}

template <typename T, int N>
hipError_t poisson_n(hrt_ctx *c, const std::vector<int> &ids) {
    hipStream_t st = c->stream;
    constexpr int XROWS = Cfg<T, N>::XROWS, YL = Cfg<T, N>::YLINES, ZL = Cfg<T, N>::ZLINES;
    const int xb = N * N / XROWS;
    const int yb = ((N / 2 + 1) * N + YL - 1) / YL, zb = ((N / 2 + 1) * N + ZL - 1) / ZL;
    const int xbi = N * N / Cfg<T, N>::XROWS_INV;
    const int R = (int)ids.size();
    FftBatch<T> fx = fft_batch<T, N>(c, ids, xb, 1), fy = fft_batch<T, N>(c, ids, yb, 1),
                fz = fft_batch<T, N>(c, ids, zb, 1), fxi = fft_batch<T, N>(c, ids, xbi, 1);
    prof_begin(c);
    x_r2c_kernel<T, N><<<xb * R, kThreads, 0, st>>>(fx);
    prof_end(c, K_FFT_X_R2C);
    prof_begin(c);
    y_lines_kernel<T, N, false><<<yb * R, kThreads, 0, st>>>(fy);
    prof_end(c, K_FFT_Y_FWD);
    prof_begin(c);
    z_lines_kernel<T, N, 2><<<zb * R, kThreads, 0, st>>>(fz);
    prof_end(c, K_FFT_Z_POISSON);
    prof_begin(c);
    y_lines_kernel<T, N, true><<<yb * R, kThreads, 0, st>>>(fy);
    prof_end(c, K_FFT_Y_INV);
    prof_begin(c);
    x_c2r_kernel<T, N><<<xbi * R, kThreads, 0, st>>>(fxi);
    prof_end(c, K_FFT_X_C2R);
    return hipGetLastError();
}

template <typename T>
hipError_t poisson_size(hrt_ctx *c, int n, const std::vector<int> &ids) {
    switch (n) {
        case 16: return poisson_n<T, 16>(c, ids);
        case 32: return poisson_n<T, 32>(c, ids);
        case 64: return poisson_n<T, 64>(c, ids);
        case 128: return poisson_n<T, 128>(c, ids);
        case 256: return poisson_n<T, 256>(c, ids);
        case 512: return poisson_n<T, 512>(c, ids);
        case 1024: return poisson_n<T, 1024>(c, ids);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t poisson_impl(hrt_ctx *c, int only) {
    if (only >= 0) return poisson_size<T>(c, c->re[only].n, std::vector<int>{only});
    // group realisations by mesh size, in order of first appearance, <= kMaxBatch per launch
    std::vector<int> sizes;
    for (const Real &re : c->re)
        if (std::find(sizes.begin(), sizes.end(), re.n) == sizes.end()) sizes.push_back(re.n);
    for (int n : sizes) {
        std::vector<int> ids;
        for (int r = 0; r < (int)c->re.size(); ++r) {
            if (c->re[r].n != n) continue;
            ids.push_back(r);
            if ((int)ids.size() == kMaxBatch) {
                if (hipError_t e = poisson_size<T>(c, n, ids)) return e;
                ids.clear();
            }
        }
        if (!ids.empty())
            if (hipError_t e = poisson_size<T>(c, n, ids)) return e;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t gradient_impl(hrt_ctx *c) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        GradBatch<T> b{};
        b.map.R = R;
        b.map.start[0] = 0;
        for (int k = 0; k < R; ++k) {
            const Real &re = c->re[r0 + k];
            const size_t n3 = (size_t)re.n * re.n * re.n;
            b.r[k].phi = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r) + n3;
            b.r[k].g = reinterpret_cast<v4<T> *>(re.ws + re.lay.grad);
            b.r[k].n = re.n;
            b.r[k].log2n = ilog2(re.n);
            b.r[k].inv12cell = (T)(1.0 / (12.0 * re.cell));
            b.map.start[k + 1] = b.map.start[k] + (int)((n3 + kThreads - 1) / kThreads);
        }
        prof_begin(c);
        fd4_gradient_kernel<T><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        prof_end(c, K_GRADIENT);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t plane_gradient_impl(hrt_ctx *c, int step) {
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        PlaneGradBatch<T> b{};
        b.map.R = R;
        b.map.start[0] = 0;
        for (int k = 0; k < R; ++k) {
            const Real &re = c->re[r0 + k];
            const size_t n3 = (size_t)re.n * re.n * re.n;
            PlaneGradR<T> &a = b.r[k];
            a.phi = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r) + n3;
            a.delta = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r);
            a.stack = reinterpret_cast<c2<T> *>(re.ws + re.lay.stack);
            a.sphi = (c->delay || c->los == HRT_LOS_POTENTIAL) ? reinterpret_cast<T *>(re.ws + re.lay.stack_phi)
                                                               : nullptr;
            a.sdelta = c->los == HRT_LOS_DENSITY ? reinterpret_cast<T *>(re.ws + re.lay.stack_delta) : nullptr;
            a.planes = reinterpret_cast<const PlaneEntry *>(re.ws + re.lay.planes);
            a.reps = reinterpret_cast<const int32_t *>(re.ws + re.lay.reps);
            a.identity = re.identity_reps ? 1 : 0;
            a.n = re.n;
            a.log2n = ilog2(re.n);
            a.begin = re.tab.plane_begin[step];
            a.count = re.tab.plane_count[step];
            a.inv12cell = (T)(1.0 / (12.0 * re.cell));
            const int64_t nodes = (int64_t)a.count * re.n * re.n;
            b.map.start[k + 1] = b.map.start[k] + (int)((nodes + kThreads - 1) / kThreads);
        }
        if (b.map.start[R] == 0) continue;
        prof_begin(c);
        plane_gradient_kernel<T><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        prof_end(c, K_PLANE_GRADIENT);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// The kick operator on the 2D ray mesh (Sec. 5.2, 5.3, App. C; HRT_RAY_MESH). The mesh is
// square, N x N complex (x = kick along u, y = along v), node k at angle (k - N/2) mu.
//   rm_paint   each mesh node pulls, from every lens plane of the shell, the plane nodes
//              whose projected angle (X - X_obs) / chi_j lies within one mesh cell of it,
//              with CIC weights, the plane's kick weight and the solid-angle ratio
//              (cell / chi_j)^2 / mu^2 (a fixed summation order: no atomics, exact reruns)
//   rm_rows    forward FFT of every row (x)
//   rm_cols    forward FFT of every column (y), times sinc(k_x mu/2)^-4 sinc(k_y mu/2)^-4
//              exp(-(k_x^2 + k_y^2) lam^2 / 2), inverse FFT of the column
//   rm_rows    inverse FFT of every row, scaled by 1 / N^2
// Every pass keeps whole lines in LDS (the Stockham stages of fft_stage).
struct RmArgs {
    void *mesh;                // N^2 complex of the dtype
    const void *tw;            // N twiddles W_N^m
    const void *stack;         // the step's lens planes (G_u, G_v) [e][v][u]
    const PlaneEntry *planes;
    int begin, count, n, N;
    double mu, lam, cell, obsx, obsy;
};

template <typename T>
__global__ __launch_bounds__(kThreads) void rm_paint_kernel(RmArgs a) {
    const int N = a.N;
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (idx >= (int64_t)N * N) return;
    const int kx = (int)(idx % N), ky = (int)(idx / N);
    const double t0 = -0.5 * N * a.mu;
    const double tx = t0 + kx * a.mu, ty = t0 + ky * a.mu;
    const c2<T> *stack = static_cast<const c2<T> *>(a.stack);
    const int n = a.n, m = n - 1;
    double su = 0.0, sv = 0.0;
    for (int e = 0; e < a.count; ++e) {
        const PlaneEntry pe = a.planes[a.begin + e];
        const double chi = pe.chi;
        const double scale = pe.w * (a.cell / chi) * (a.cell / chi) / (a.mu * a.mu);
        const c2<T> *pl = stack + (size_t)e * n * n;
        // plane nodes i with |(i cell - X_obs) / chi - t| < mu, along each axis
        const int ix0 = (int)floor((a.obsx + chi * (tx - a.mu)) / a.cell);
        const int ix1 = (int)ceil((a.obsx + chi * (tx + a.mu)) / a.cell);
        const int iy0 = (int)floor((a.obsy + chi * (ty - a.mu)) / a.cell);
        const int iy1 = (int)ceil((a.obsy + chi * (ty + a.mu)) / a.cell);
        for (int iy = iy0; iy <= iy1; ++iy) {
            const double uy = (((double)iy * a.cell - a.obsy) / chi - t0) / a.mu;
            const double wy = 1.0 - fabs(uy - ky);
            if (!(wy > 0.0)) continue;
            const c2<T> *row = pl + (size_t)(iy & m) * n;
            for (int ix = ix0; ix <= ix1; ++ix) {
                const double ux = (((double)ix * a.cell - a.obsx) / chi - t0) / a.mu;
                const double wx = 1.0 - fabs(ux - kx);
                if (!(wx > 0.0)) continue;
                const c2<T> g = row[ix & m];
                const double wgt = scale * wx * wy;
                su += wgt * (double)g.x;
                sv += wgt * (double)g.y;
            }
        }
    }
    static_cast<c2<T> *>(a.mesh)[idx] = c2<T>{(T)su, (T)sv};
}

// Lines per workgroup of the ray-mesh passes: at most 32 KB of lines in LDS (plus the
// twiddle table), at most 8 lines.
template <typename T, int N>
__host__ __device__ constexpr int rm_lines() {
    constexpr int b = 32768 / (N * (int)sizeof(c2<T>));
    return b < 1 ? 1 : (b > 8 ? 8 : b);
}

// Rows: LINES consecutive rows per workgroup. INV: inverse transform scaled by 1 / N^2.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void rm_rows_kernel(RmArgs a) {
    constexpr int LINES = rm_lines<T, N>();
    __shared__ c2<T> buf[LINES * N];
    __shared__ c2<T> tw[N];
    c2<T> *mesh = static_cast<c2<T> *>(a.mesh);
    const c2<T> *gtw = static_cast<const c2<T> *>(a.tw);
    const size_t base = (size_t)blockIdx.x * LINES * N;
    for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = gtw[i];
    for (int i = threadIdx.x; i < LINES * N; i += kThreads) buf[i] = mesh[base + i];
    __syncthreads();
    fft_stage<T, N, LINES, INV, 1>(buf, N, tw, 1);
    const T sc = INV ? (T)(1.0 / ((double)N * N)) : T(1);
    for (int i = threadIdx.x; i < LINES * N; i += kThreads) {
        c2<T> v = buf[i];
        if (INV) v = c2<T>{v.x * sc, v.y * sc};
        mesh[base + i] = v;
    }
}

// Columns: LINES consecutive columns per workgroup; forward FFT, the filter, inverse FFT.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void rm_cols_kernel(RmArgs a) {
    constexpr int LINES = rm_lines<T, N>();
    __shared__ c2<T> buf[LINES * N];
    __shared__ c2<T> tw[N];
    c2<T> *mesh = static_cast<c2<T> *>(a.mesh);
    const c2<T> *gtw = static_cast<const c2<T> *>(a.tw);
    const int col0 = blockIdx.x * LINES;
    for (int i = threadIdx.x; i < N; i += kThreads) tw[i] = gtw[i];
    for (int i = threadIdx.x; i < LINES * N; i += kThreads) {
        const int line = i % LINES, y = i / LINES;          // consecutive lanes: adjacent columns
        buf[line * N + y] = mesh[(size_t)y * N + col0 + line];
    }
    __syncthreads();
    fft_stage<T, N, LINES, false, 1>(buf, N, tw, 1);
    const double kf = 2.0 * 3.14159265358979323846 / (N * a.mu);
    for (int i = threadIdx.x; i < LINES * N; i += kThreads) {
        const int line = i / N, y = i % N;
        const int fx = col0 + line, fy = y;
        const double kx = kf * (fx < N / 2 ? fx : fx - N), ky = kf * (fy < N / 2 ? fy : fy - N);
        const double hx = 0.5 * kx * a.mu, hy = 0.5 * ky * a.mu;
        const double sx = hx == 0.0 ? 1.0 : sin(hx) / hx, sy = hy == 0.0 ? 1.0 : sin(hy) / hy;
        const double s2x = sx * sx, s2y = sy * sy;
        const double h = exp(-0.5 * (kx * kx + ky * ky) * a.lam * a.lam) / (s2x * s2x * s2y * s2y);
        const c2<T> v = buf[i];
        buf[i] = c2<T>{(T)((double)v.x * h), (T)((double)v.y * h)};
    }
    __syncthreads();
    fft_stage<T, N, LINES, true, 1>(buf, N, tw, 1);
    for (int i = threadIdx.x; i < LINES * N; i += kThreads) {
        const int line = i % LINES, y = i / LINES;
        mesh[(size_t)y * N + col0 + line] = buf[line * N + y];
    }
}

template <typename T, int N>
hipError_t ray_mesh_n(hrt_ctx *c, const RmArgs &a) {
    constexpr int LINES = rm_lines<T, N>();
    rm_rows_kernel<T, N, false><<<N / LINES, kThreads, 0, c->stream>>>(a);
    rm_cols_kernel<T, N><<<N / LINES, kThreads, 0, c->stream>>>(a);
    rm_rows_kernel<T, N, true><<<N / LINES, kThreads, 0, c->stream>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t ray_mesh_impl(hrt_ctx *c, int step) {
    for (size_t r = 0; r < c->re.size(); ++r) {
        const Real &re = c->re[r];
        RmArgs a{};
        a.mesh = re.ws + re.lay.rm_mesh;
        a.tw = re.ws + re.lay.rm_tw;
        a.stack = re.ws + re.lay.stack;
        a.planes = reinterpret_cast<const PlaneEntry *>(re.ws + re.lay.planes);
        a.begin = re.tab.plane_begin[step];
        a.count = re.tab.plane_count[step];
        a.n = re.n;
        a.N = re.tab.rm_n;
        a.mu = re.tab.rm_mu[step];
        a.lam = re.tab.rm_lam[step];
        a.cell = re.cell;
        a.obsx = re.cfg.observer[0];
        a.obsy = re.cfg.observer[1];
        if (a.count == 0) continue;              // no planes: the ray step adds no kick
        const int64_t nodes = (int64_t)a.N * a.N;
        prof_begin(c);
        rm_paint_kernel<T><<<(int)((nodes + kThreads - 1) / kThreads), kThreads, 0, c->stream>>>(a);
        hipError_t e = hipSuccess;
        switch (a.N) {
            case 16: e = ray_mesh_n<T, 16>(c, a); break;
            case 32: e = ray_mesh_n<T, 32>(c, a); break;
            case 64: e = ray_mesh_n<T, 64>(c, a); break;
            case 128: e = ray_mesh_n<T, 128>(c, a); break;
            case 256: e = ray_mesh_n<T, 256>(c, a); break;
            case 512: e = ray_mesh_n<T, 512>(c, a); break;
            case 1024: e = ray_mesh_n<T, 1024>(c, a); break;
            case 2048: e = ray_mesh_n<T, 2048>(c, a); break;
            default: e = hipErrorInvalidValue;
        }
        prof_end(c, K_RAY_MESH);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Initial conditions: Gaussian field with the Eisenstein-Hu no-wiggle spectrum and its
// 2LPT displacements (standard recipe; the paper starts from 2LPT at a = 1/64, Sec. 6.2).
// Spectra use the transposed layout [kx][kz][ky] left by the forward passes. Derivatives
// use i k_d with the Nyquist wavenumber zeroed; second derivatives apply it twice.

enum { OP_PHI1 = 0, OP_GRAD = 1, OP_HESS = 2, OP_INVLAP = 3 };

__device__ __forceinline__ double eh_nowiggle(double k, const IcParams &p) {
    const double ks = 0.43 * k * p.h * p.s_sound;
    const double gamma_eff = p.omega_m * p.h * (p.alpha + (1.0 - p.alpha) / (1.0 + ks * ks * ks * ks));
    const double q = k * p.theta2 / gamma_eff;
    const double l0 = log(2.0 * 2.718281828459045 + 1.8 * q);
    const double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
    return l0 / (l0 + c0 * q * q);
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void spec_op_kernel(const c2<T> *__restrict__ in,
                                                           c2<T> *__restrict__ out, int op, int a,
                                                           int b, double scale, IcParams p,
                                                           int acc) {
    const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (int64_t)(N / 2 + 1) * N * N) return;
    const int iky = (int)(e % N), ikz = (int)((e / N) % N), ikx = (int)(e / ((int64_t)N * N));
    const int fy = iky <= N / 2 ? iky : iky - N, fz = ikz <= N / 2 ? ikz : ikz - N;
    const double kf = p.kf;
    const double k2 = kf * kf * (double)(ikx * ikx + fy * fy + fz * fz);
    // derivative wavenumbers with the Nyquist entry zeroed
    const double kd[3] = {ikx == N / 2 ? 0.0 : kf * ikx, iky == N / 2 ? 0.0 : kf * fy,
                          ikz == N / 2 ? 0.0 : kf * fz};
    const c2<T> v = in[e];
    double re = 0.0, im = 0.0;        // factor re + i im
    if (k2 > 0.0) {
        if (op == OP_PHI1) {
            const double k = sqrt(k2), t = eh_nowiggle(k, p);
            re = -sqrt(p.amp * pow(k, p.n_s) * t * t / p.cell_volume) / k2 * scale;
        } else if (op == OP_GRAD) {
            im = kd[a] * scale;
        } else if (op == OP_HESS) {
            re = -kd[a] * kd[b] * scale;
        } else {
            re = -scale / k2;
        }
    }
    c2<T> r{(T)(re * v.x - im * v.y), (T)(re * v.y + im * v.x)};
    if (acc) {                        // accumulate (reverse mode)
        const c2<T> o = out[e];
        r.x += o.x;
        r.y += o.y;
    }
    out[e] = r;
}

template <typename T>
__global__ void lpt_source_diag_kernel(const T *__restrict__ A, const T *__restrict__ B,
                                       const T *__restrict__ C, T *__restrict__ src, int64_t P) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < P) src[i] = A[i] * B[i] + A[i] * C[i] + B[i] * C[i];
}

template <typename T>
__global__ void lpt_source_off_kernel(const T *__restrict__ t, T *__restrict__ src, int64_t P) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < P) src[i] -= t[i] * t[i];
}

// s = g1 s1 + g2 s2, p = m1 s1 + m2 s2 (s holds s1, p holds s2 on entry)
template <typename T>
__global__ void lpt_combine_kernel(T *__restrict__ s, T *__restrict__ p, int64_t P, double g1,
                                   double g2, double m1, double m2) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < P) {
        const double a = s[i], b = p[i];
        s[i] = (T)(g1 * a + g2 * b);
        p[i] = (T)(m1 * a + m2 * b);
    }
}

// 3D transforms of one lattice of size N (the IC's particle lattice) in a realisation's
// workspace; tws = mesh size / N.
template <typename T, int N>
void fwd3d(hrt_ctx *c, int r, const T *real_in, c2<T> *spec, int tws) {
    constexpr int XROWS = Cfg<T, N>::XROWS, YL = Cfg<T, N>::YLINES, ZL = Cfg<T, N>::ZLINES;
    const int xb = N * N / XROWS;
    const int yb = ((N / 2 + 1) * N + YL - 1) / YL, zb = ((N / 2 + 1) * N + ZL - 1) / ZL;
    FftBatch<T> fb{};
    fb.tws = tws;
    fb.rin[0] = real_in;
    fb.spec[0] = spec;
    fb.tw[0] = reinterpret_cast<const c2<T> *>(c->re[r].ws + c->re[r].lay.twiddle);
    fb.bpr = xb;
    x_r2c_kernel<T, N><<<xb, kThreads, 0, c->stream>>>(fb);
    fb.bpr = yb;
    y_lines_kernel<T, N, false><<<yb, kThreads, 0, c->stream>>>(fb);
    fb.bpr = zb;
    z_lines_kernel<T, N, 0><<<zb, kThreads, 0, c->stream>>>(fb);
}

template <typename T, int N>
void inv3d(hrt_ctx *c, int r, c2<T> *spec, T *real_out, int tws) {
    constexpr int YL = Cfg<T, N>::YLINES, ZL = Cfg<T, N>::ZLINES;
    const int yb = ((N / 2 + 1) * N + YL - 1) / YL, zb = ((N / 2 + 1) * N + ZL - 1) / ZL;
    FftBatch<T> fb{};
    fb.tws = tws;
    fb.rout[0] = real_out;
    fb.spec[0] = spec;
    fb.tw[0] = reinterpret_cast<const c2<T> *>(c->re[r].ws + c->re[r].lay.twiddle);
    fb.bpr = zb;
    z_lines_kernel<T, N, 1><<<zb, kThreads, 0, c->stream>>>(fb);
    fb.bpr = yb;
    y_lines_kernel<T, N, true><<<yb, kThreads, 0, c->stream>>>(fb);
    fb.bpr = N * N / Cfg<T, N>::XROWS_INV;
    x_c2r_kernel<T, N><<<fb.bpr, kThreads, 0, c->stream>>>(fb);
}

template <typename T, int N>
hipError_t ic_n(hrt_ctx *c, int r, const T *noise, const IcParams &p, const hrt_matter *m) {
    const Real &re = c->re[r];
    const int tws = re.n / N;
    const int64_t P = (int64_t)N * N * N;
    const int64_t ns = (int64_t)(N / 2 + 1) * N * N;
    const int sblocks = (int)((ns + kThreads - 1) / kThreads), pblocks = (int)((P + kThreads - 1) / kThreads);
    c2<T> *base = reinterpret_cast<c2<T> *>(re.ws + re.lay.spec2);
    c2<T> *work = reinterpret_cast<c2<T> *>(re.ws + re.lay.spec);
    T *scratch = reinterpret_cast<T *>(re.ws + re.lay.grad);        // 4 lattices of P values
    T *A = scratch, *B = scratch + P, *C = scratch + 2 * P, *tmp = scratch + 3 * P;
    T *src = reinterpret_cast<T *>(re.ws + re.lay.mesh_r);
    T *s[3] = {static_cast<T *>(m->s[0]), static_cast<T *>(m->s[1]), static_cast<T *>(m->s[2])};
    T *q[3] = {static_cast<T *>(m->p[0]), static_cast<T *>(m->p[1]), static_cast<T *>(m->p[2])};
    const double inv_n3 = 1.0 / (double)P;
    hipStream_t st = c->stream;
    fwd3d<T, N>(c, r, noise, base, tws);
    spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, base, OP_PHI1, 0, 0, 1.0, p, 0);
    for (int d = 0; d < 3; ++d) {          // s1 = -grad phi1
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, work, OP_GRAD, d, 0, -inv_n3, p, 0);
        inv3d<T, N>(c, r, work, s[d], tws);
    }
    T *diag[3] = {A, B, C};
    for (int d = 0; d < 3; ++d) {
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, work, OP_HESS, d, d, inv_n3, p, 0);
        inv3d<T, N>(c, r, work, diag[d], tws);
    }
    lpt_source_diag_kernel<T><<<pblocks, kThreads, 0, st>>>(A, B, C, src, P);
    const int off[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int k = 0; k < 3; ++k) {
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, work, OP_HESS, off[k][0], off[k][1],
                                                           inv_n3, p, 0);
        inv3d<T, N>(c, r, work, tmp, tws);
        lpt_source_off_kernel<T><<<pblocks, kThreads, 0, st>>>(tmp, src, P);
    }
    fwd3d<T, N>(c, r, src, base, tws);
    spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, base, OP_INVLAP, 0, 0, 1.0, p, 0);
    for (int d = 0; d < 3; ++d) {          // s2 = +grad phi2, parked in the momentum arrays
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(base, work, OP_GRAD, d, 0, inv_n3, p, 0);
        inv3d<T, N>(c, r, work, q[d], tws);
    }
    for (int d = 0; d < 3; ++d)
        lpt_combine_kernel<T><<<pblocks, kThreads, 0, st>>>(s[d], q[d], P, p.g1, p.g2, p.m1, p.m2);
    return hipGetLastError();
}

// Reverse mode of the 2LPT state (linear in s1, s2; s2 quadratic in phi1):
// tmp = g s_bar + m p_bar for one component.
template <typename T>
__global__ void lpt_cot_kernel(const T *__restrict__ sb, const T *__restrict__ pb, T *__restrict__ out,
                               int64_t P, double g, double m) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < P) out[i] = (T)(g * (double)sb[i] + m * (double)pb[i]);
}

// Hessians H = (H00, H11, H22, H01, H02, H12) of phi1 -> their cotangents in place from the
// cotangent u of the source sum_{i<j} (H_ii H_jj - H_ij^2).
template <typename T>
__global__ void lpt_hess_bar_kernel(T *__restrict__ h0, T *__restrict__ h1, T *__restrict__ h2,
                                    T *__restrict__ h3, T *__restrict__ h4, T *__restrict__ h5,
                                    const T *__restrict__ u, int64_t P) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= P) return;
    const T a = h0[i], b = h1[i], cc = h2[i], ui = u[i];
    h0[i] = ui * (b + cc);
    h1[i] = ui * (a + cc);
    h2[i] = ui * (a + b);
    h3[i] = T(-2) * ui * h3[i];
    h4[i] = T(-2) * ui * h4[i];
    h5[i] = T(-2) * ui * h5[i];
}

// noise_bar from (s_bar, p_bar): recompute the six Hessians of phi1; src_bar =
// L(-sum_d D_d s2_bar_d); Hessian cotangents; phi1_bar = sum_d D_d s1_bar_d +
// sum_ij D_i D_j H_bar_ij; noise_bar = Phi phi1_bar (Phi: the real even multiplier of the
// noise -> phi1 map). Spectra are accumulated in the second spectrum; the caller's
// noise_bar array serves as the one real temporary until the last transform.
template <typename T, int N>
hipError_t ic_vjp_n(hrt_ctx *c, int r, const T *noise, const IcParams &p, const hrt_matter *cot,
                    T *noise_bar) {
    const Real &re = c->re[r];
    const int tws = re.n / N;
    const int64_t P = (int64_t)N * N * N;
    const int64_t ns = (int64_t)(N / 2 + 1) * N * N;
    const int sblocks = (int)((ns + kThreads - 1) / kThreads), pblocks = (int)((P + kThreads - 1) / kThreads);
    c2<T> *acc = reinterpret_cast<c2<T> *>(re.ws + re.lay.spec2);
    c2<T> *work = reinterpret_cast<c2<T> *>(re.ws + re.lay.spec);
    T *g4 = reinterpret_cast<T *>(re.ws + re.lay.grad);        // 4 lattices of P values
    T *m2 = reinterpret_cast<T *>(re.ws + re.lay.mesh_r);      // 2 lattices of P values
    T *H[6] = {g4, g4 + P, g4 + 2 * P, g4 + 3 * P, m2, m2 + P};
    const int hij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    const T *sb[3] = {static_cast<const T *>(cot->s[0]), static_cast<const T *>(cot->s[1]),
                      static_cast<const T *>(cot->s[2])};
    const T *pb[3] = {static_cast<const T *>(cot->p[0]), static_cast<const T *>(cot->p[1]),
                      static_cast<const T *>(cot->p[2])};
    T *tmp = noise_bar;
    const double inv_n3 = 1.0 / (double)P;
    hipStream_t st = c->stream;
    // forward: phi1 spectrum, Hessians
    fwd3d<T, N>(c, r, noise, acc, tws);
    spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(acc, acc, OP_PHI1, 0, 0, 1.0, p, 0);
    for (int k = 0; k < 6; ++k) {
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(acc, work, OP_HESS, hij[k][0], hij[k][1],
                                                           inv_n3, p, 0);
        inv3d<T, N>(c, r, work, H[k], tws);
    }
    // src_bar = L(-sum_d D_d s2_bar_d), s2_bar = g2 s_bar + m2 p_bar
    for (int d = 0; d < 3; ++d) {
        lpt_cot_kernel<T><<<pblocks, kThreads, 0, st>>>(sb[d], pb[d], tmp, P, p.g2, p.m2);
        fwd3d<T, N>(c, r, tmp, work, tws);
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(work, acc, OP_GRAD, d, 0, -1.0, p, d > 0);
    }
    spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(acc, work, OP_INVLAP, 0, 0, inv_n3, p, 0);
    inv3d<T, N>(c, r, work, tmp, tws);
    lpt_hess_bar_kernel<T><<<pblocks, kThreads, 0, st>>>(H[0], H[1], H[2], H[3], H[4], H[5], tmp, P);
    // phi1_bar spectrum: sum_d (i k_d) FFT(s1_bar_d) + sum_ij (-k_i k_j) FFT(H_bar_ij)
    for (int d = 0; d < 3; ++d) {
        lpt_cot_kernel<T><<<pblocks, kThreads, 0, st>>>(sb[d], pb[d], tmp, P, p.g1, p.m1);
        fwd3d<T, N>(c, r, tmp, work, tws);
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(work, acc, OP_GRAD, d, 0, 1.0, p, d > 0);
    }
    for (int k = 0; k < 6; ++k) {
        fwd3d<T, N>(c, r, H[k], work, tws);
        spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(work, acc, OP_HESS, hij[k][0], hij[k][1],
                                                           1.0, p, 1);
    }
    spec_op_kernel<T, N><<<sblocks, kThreads, 0, st>>>(acc, work, OP_PHI1, 0, 0, inv_n3, p, 0);
    inv3d<T, N>(c, r, work, noise_bar, tws);
    return hipGetLastError();
}

template <typename T>
hipError_t ic_vjp_impl(hrt_ctx *c, int r, const void *noise, const IcParams &p, const hrt_matter *cot,
                       void *noise_bar) {
    const T *nz = static_cast<const T *>(noise);
    T *nb = static_cast<T *>(noise_bar);
    switch (c->re[r].np) {
        case 16: return ic_vjp_n<T, 16>(c, r, nz, p, cot, nb);
        case 32: return ic_vjp_n<T, 32>(c, r, nz, p, cot, nb);
        case 64: return ic_vjp_n<T, 64>(c, r, nz, p, cot, nb);
        case 128: return ic_vjp_n<T, 128>(c, r, nz, p, cot, nb);
        case 256: return ic_vjp_n<T, 256>(c, r, nz, p, cot, nb);
        case 512: return ic_vjp_n<T, 512>(c, r, nz, p, cot, nb);
        case 1024: return ic_vjp_n<T, 1024>(c, r, nz, p, cot, nb);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t ic_impl(hrt_ctx *c, int r, const void *noise, const IcParams &p, const hrt_matter *m) {
    const T *nz = static_cast<const T *>(noise);
    switch (c->re[r].np) {
        case 16: return ic_n<T, 16>(c, r, nz, p, m);
        case 32: return ic_n<T, 32>(c, r, nz, p, m);
        case 64: return ic_n<T, 64>(c, r, nz, p, m);
        case 128: return ic_n<T, 128>(c, r, nz, p, m);
        case 256: return ic_n<T, 256>(c, r, nz, p, m);
        case 512: return ic_n<T, 512>(c, r, nz, p, m);
        case 1024: return ic_n<T, 1024>(c, r, nz, p, m);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_poisson(hrt_ctx *c, int only) {
    return c->f64 ? poisson_impl<double>(c, only) : poisson_impl<float>(c, only);
}

hipError_t launch_ic(hrt_ctx *c, int r, const void *noise, const IcParams &p, const hrt_matter *m) {
    return c->f64 ? ic_impl<double>(c, r, noise, p, m) : ic_impl<float>(c, r, noise, p, m);
}

hipError_t launch_ic_vjp(hrt_ctx *c, int r, const void *noise, const IcParams &p, const hrt_matter *cot,
                         void *noise_bar) {
    return c->f64 ? ic_vjp_impl<double>(c, r, noise, p, cot, noise_bar)
                  : ic_vjp_impl<float>(c, r, noise, p, cot, noise_bar);
}

hipError_t launch_gradient(hrt_ctx *c) {
    return c->f64 ? gradient_impl<double>(c) : gradient_impl<float>(c);
}

hipError_t launch_plane_gradient(hrt_ctx *c, int step) {
    return c->f64 ? plane_gradient_impl<double>(c, step) : plane_gradient_impl<float>(c, step);
}

hipError_t launch_ray_mesh(hrt_ctx *c, int step) {
    return c->f64 ? ray_mesh_impl<double>(c, step) : ray_mesh_impl<float>(c, step);
}

}  // namespace hrt
