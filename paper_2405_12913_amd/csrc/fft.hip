// FFT Poisson solve and gradient of the PM step (paper Sec. 2 Poisson equation; Sec. 4.1:
// the potential gradient is obtained with FFTs once per step).
//
// Hand-written LDS-staged Stockham FFTs (radix 4, one radix-2 stage when log2 L is
// odd), one workgroup of 256 threads per batch of lines:
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
#include "device_common.h"
#include "hrt_internal.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(c2<T> *v) {
    if constexpr (R == 2) {
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

// One Stockham stage over LINES lines of length L in LDS (line stride LS), then the next.
// tw holds W_n^m = exp(-2 pi i m / n); W_L^m = tw[m * twmul] with twmul = n / L.
template <typename T, int L, int LINES, bool INV, int Ns>
__device__ __forceinline__ void fft_stage(c2<T> *buf, int LS, const c2<T> *__restrict__ tw,
                                          int twmul) {
    if constexpr (Ns < L) {
        constexpr int R = (Ns * 4 <= L) ? 4 : 2;
        constexpr int NB = LINES * (L / R);
        constexpr int BF = (NB + kThreads - 1) / kThreads;
        c2<T> v[BF][R];
#pragma unroll
        for (int k = 0; k < BF; ++k) {
            const int b = threadIdx.x + k * kThreads;
            if (b < NB) {
                const int line = b / (L / R), j = b % (L / R);
                const int kk = j % Ns;
                const c2<T> *src = buf + line * LS;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    c2<T> x = src[j + r * (L / R)];
                    if (r > 0) {
                        c2<T> w = tw[(kk * r * (L / (Ns * R))) * twmul];
                        if (INV) w.y = -w.y;
                        x = cmul<T>(x, w);
                    }
                    v[k][r] = x;
                }
                dft<T, R, INV>(v[k]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < BF; ++k) {
            const int b = threadIdx.x + k * kThreads;
            if (b < NB) {
                const int line = b / (L / R), j = b % (L / R);
                const int kk = j % Ns;
                c2<T> *dst = buf + line * LS + (j / Ns) * Ns * R + kk;
#pragma unroll
                for (int r = 0; r < R; ++r) dst[r * Ns] = v[k][r];
            }
        }
        __syncthreads();
        fft_stage<T, L, LINES, INV, Ns * R>(buf, LS, tw, twmul);
    }
}

template <typename T, int N>
struct Cfg {
    static constexpr int ELEMS = sizeof(T) == 4 ? 4096 : 2048;   // complex values per block
    static constexpr int XROWS = (ELEMS / (N / 2)) < N * N ? ELEMS / (N / 2) : N * N;
    static constexpr int LINES = ELEMS / N;                        // y and z passes
};

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void x_r2c_kernel(const T *__restrict__ in,
                                                         c2<T> *__restrict__ out,
                                                         const c2<T> *__restrict__ tw) {
    constexpr int L = N / 2, ROWS = Cfg<T, N>::XROWS, LS = L + 1;
    __shared__ c2<T> buf[ROWS * LS];
    const int row0 = blockIdx.x * ROWS;
    for (int e = threadIdx.x; e < ROWS * L; e += kThreads) {
        const int r = e / L, m = e % L;
        buf[r * LS + m] = reinterpret_cast<const c2<T> *>(in + (size_t)(row0 + r) * N)[m];
    }
    __syncthreads();
    fft_stage<T, L, ROWS, false, 1>(buf, LS, tw, N / L);
    // split step: X[k] = (Z[k] + conj Z[L-k])/2 - (i/2) W_N^k (Z[k] - conj Z[L-k]),
    // each thread owns the pair (k, L-k); X[L] (Nyquist) comes from Z[0].
    for (int e = threadIdx.x; e < ROWS * (L / 2 + 1); e += kThreads) {
        const int r = e / (L / 2 + 1), k = e % (L / 2 + 1);
        c2<T> *line = buf + r * LS;
        const c2<T> zk = line[k];
        const c2<T> zp = line[k == 0 ? 0 : L - k];
        const c2<T> w = tw[k];
        // A = zk + conj(zp), B = zk - conj(zp); X[k] = A/2 - (i/2) w B
        const c2<T> A{zk.x + zp.x, zk.y - zp.y}, B{zk.x - zp.x, zk.y + zp.y};
        const c2<T> wB = cmul<T>(w, B);
        line[k] = c2<T>{T(0.5) * (A.x + wB.y), T(0.5) * (A.y - wB.x)};
        if (k == 0) {
            line[L] = c2<T>{T(0.5) * (A.x - wB.y), T(0.5) * (A.y + wB.x)};   // W_N^L = -1
        } else if (k != L - k) {
            // X[L-k] = A'/2 - (i/2) W_N^{L-k} B', A' = conj(A), B' = -conj(B), W_N^{L-k} = -conj(w)
            const c2<T> Ap{A.x, -A.y}, Bp{-B.x, B.y}, wp{-w.x, w.y};
            const c2<T> wBp = cmul<T>(wp, Bp);
            line[L - k] = c2<T>{T(0.5) * (Ap.x + wBp.y), T(0.5) * (Ap.y - wBp.x)};
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ROWS * (L + 1); e += kThreads) {
        const int kx = e / ROWS, r = e % ROWS;
        const int row = row0 + r, z = row / N, y = row % N;
        out[((size_t)kx * N + z) * N + y] = buf[r * LS + kx];
    }
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void x_c2r_kernel(const c2<T> *__restrict__ in,
                                                         T *__restrict__ out,
                                                         const c2<T> *__restrict__ tw) {
    constexpr int L = N / 2, ROWS = Cfg<T, N>::XROWS, LS = L + 1;
    __shared__ c2<T> buf[ROWS * LS];
    const int row0 = blockIdx.x * ROWS;
    for (int e = threadIdx.x; e < ROWS * (L + 1); e += kThreads) {
        const int kx = e / ROWS, r = e % ROWS;
        const int row = row0 + r, z = row / N, y = row % N;
        buf[r * LS + kx] = in[((size_t)kx * N + z) * N + y];
    }
    __syncthreads();
    // Z[k] = (X[k] + conj X[L-k]) + i W_N^{-k} (X[k] - conj X[L-k]), pairs (k, L-k)
    for (int e = threadIdx.x; e < ROWS * (L / 2 + 1); e += kThreads) {
        const int r = e / (L / 2 + 1), k = e % (L / 2 + 1);
        c2<T> *line = buf + r * LS;
        const c2<T> xk = line[k], xp = line[L - k];
        const c2<T> w = tw[k];
        const c2<T> wc{w.x, -w.y};
        const c2<T> A{xk.x + xp.x, xk.y - xp.y}, B{xk.x - xp.x, xk.y + xp.y};
        const c2<T> wB = cmul<T>(wc, B);
        line[k] = c2<T>{A.x - wB.y, A.y + wB.x};
        if (k != 0 && k != L - k) {
            // Z[L-k] = conj(A) + i (-w) (-conj(B))
            const c2<T> Ap{A.x, -A.y}, Bp{-B.x, B.y}, wp{-w.x, -w.y};
            const c2<T> wBp = cmul<T>(wp, Bp);
            line[L - k] = c2<T>{Ap.x - wBp.y, Ap.y + wBp.x};
        }
    }
    __syncthreads();
    fft_stage<T, L, ROWS, true, 1>(buf, LS, tw, N / L);
    for (int e = threadIdx.x; e < ROWS * L; e += kThreads) {
        const int r = e / L, m = e % L;
        reinterpret_cast<c2<T> *>(out + (size_t)(row0 + r) * N)[m] = buf[r * LS + m];
    }
}

// FFT along y of the transposed spectrum C[kx][z][y]: lines are contiguous.
template <typename T, int N, bool INV>
__global__ __launch_bounds__(kThreads) void y_lines_kernel(c2<T> *__restrict__ data,
                                                           const c2<T> *__restrict__ tw,
                                                           int total_lines) {
    constexpr int LINES = Cfg<T, N>::LINES, LS = N + 1;
    __shared__ c2<T> buf[LINES * LS];
    const int l0 = blockIdx.x * LINES;
    for (int e = threadIdx.x; e < LINES * N; e += kThreads) {
        const int li = e / N, m = e % N;
        if (l0 + li < total_lines) buf[li * LS + m] = data[(size_t)(l0 + li) * N + m];
    }
    __syncthreads();
    fft_stage<T, N, LINES, INV, 1>(buf, LS, tw, 1);
    for (int e = threadIdx.x; e < LINES * N; e += kThreads) {
        const int li = e / N, m = e % N;
        if (l0 + li < total_lines) data[(size_t)(l0 + li) * N + m] = buf[li * LS + m];
    }
}

// Forward FFT along z, Green's function, inverse FFT along z. Line l = kx * N + y.
template <typename T, int N>
__global__ __launch_bounds__(kThreads) void z_poisson_kernel(c2<T> *__restrict__ data,
                                                             const c2<T> *__restrict__ tw,
                                                             int total_lines, double kf2,
                                                             double inv_n3) {
    constexpr int LINES = Cfg<T, N>::LINES, LS = N + 1;
    __shared__ c2<T> buf[LINES * LS];
    const int l0 = blockIdx.x * LINES;
    for (int e = threadIdx.x; e < LINES * N; e += kThreads) {
        const int z = e / LINES, li = e % LINES, l = l0 + li;
        if (l < total_lines) buf[li * LS + z] = data[((size_t)(l / N) * N + z) * N + (l % N)];
    }
    __syncthreads();
    fft_stage<T, N, LINES, false, 1>(buf, LS, tw, 1);
    for (int e = threadIdx.x; e < LINES * N; e += kThreads) {
        const int li = e / N, kz = e % N, l = l0 + li;
        const int kx = l / N, ky = l % N;
        const int fy = ky <= N / 2 ? ky : ky - N, fz = kz <= N / 2 ? kz : kz - N;
        const double k2 = kf2 * (double)(kx * kx + fy * fy + fz * fz);
        const T g = k2 > 0.0 ? (T)(-inv_n3 / k2) : T(0);
        c2<T> v = buf[li * LS + kz];
        buf[li * LS + kz] = c2<T>{v.x * g, v.y * g};
    }
    __syncthreads();
    fft_stage<T, N, LINES, true, 1>(buf, LS, tw, 1);
    for (int e = threadIdx.x; e < LINES * N; e += kThreads) {
        const int z = e / LINES, li = e % LINES, l = l0 + li;
        if (l < total_lines) data[((size_t)(l / N) * N + z) * N + (l % N)] = buf[li * LS + z];
    }
}

// One lane per node, x fastest; blocks XCD-remapped so the +-2 neighbour rows and
// planes a block reads are mostly in its own XCD's L2.
template <typename T>
__global__ __launch_bounds__(kThreads) void fd4_gradient_kernel(const T *__restrict__ phi,
                                                                v4<T> *__restrict__ g, int n,
                                                                int log2n, T inv12cell) {
    const int64_t idx = (int64_t)xcd_block(gridDim.x) * kThreads + threadIdx.x;
    if (idx >= ((int64_t)1 << (3 * log2n))) return;
    const int m = n - 1;
    const int x = (int)(idx & m), y = (int)((idx >> log2n) & m), z = (int)(idx >> (2 * log2n));
    const size_t row = ((size_t)z * n + y) * n;
    auto at = [&](int xx, int yy, int zz) {
        return phi[(((size_t)(zz & m) * n + (yy & m)) * n) + (xx & m)];
    };
    const T dx = T(8) * (phi[row + ((x + 1) & m)] - phi[row + ((x - 1) & m)]) -
                 (phi[row + ((x + 2) & m)] - phi[row + ((x - 2) & m)]);
    const T dy = T(8) * (at(x, y + 1, z) - at(x, y - 1, z)) - (at(x, y + 2, z) - at(x, y - 2, z));
    const T dz = T(8) * (at(x, y, z + 1) - at(x, y, z - 1)) - (at(x, y, z + 2) - at(x, y, z - 2));
    v4<T> out;
    out.x = dx * inv12cell;
    out.y = dy * inv12cell;
    out.z = dz * inv12cell;
    out.w = T(0);
    g[idx] = out;
}

template <typename T, int N>
hipError_t poisson_n(hrt_ctx *c) {
    const T *delta = reinterpret_cast<const T *>(c->ws + c->lay.mesh_r);
    T *phi = reinterpret_cast<T *>(c->ws + c->lay.mesh_r) + (size_t)N * N * N;
    c2<T> *spec = reinterpret_cast<c2<T> *>(c->ws + c->lay.spec);
    const c2<T> *tw = reinterpret_cast<const c2<T> *>(c->ws + c->lay.twiddle);
    hipStream_t st = c->stream;
    constexpr int XROWS = Cfg<T, N>::XROWS, LINES = Cfg<T, N>::LINES;
    const int xblocks = N * N / XROWS;
    const int total_lines = (N / 2 + 1) * N;
    const int lblocks = (total_lines + LINES - 1) / LINES;
    const double kf = 2.0 * 3.14159265358979323846 / c->box;
    prof_begin(c);
    x_r2c_kernel<T, N><<<xblocks, kThreads, 0, st>>>(delta, spec, tw);
    prof_end(c, K_FFT_X_R2C);
    prof_begin(c);
    y_lines_kernel<T, N, false><<<lblocks, kThreads, 0, st>>>(spec, tw, total_lines);
    prof_end(c, K_FFT_Y_FWD);
    prof_begin(c);
    z_poisson_kernel<T, N><<<lblocks, kThreads, 0, st>>>(spec, tw, total_lines, kf * kf,
                                                          1.0 / ((double)N * N * N));
    prof_end(c, K_FFT_Z_POISSON);
    prof_begin(c);
    y_lines_kernel<T, N, true><<<lblocks, kThreads, 0, st>>>(spec, tw, total_lines);
    prof_end(c, K_FFT_Y_INV);
    prof_begin(c);
    x_c2r_kernel<T, N><<<xblocks, kThreads, 0, st>>>(spec, phi, tw);
    prof_end(c, K_FFT_X_C2R);
    return hipGetLastError();
}

template <typename T>
hipError_t poisson_impl(hrt_ctx *c) {
    switch (c->n) {
        case 16: return poisson_n<T, 16>(c);
        case 32: return poisson_n<T, 32>(c);
        case 64: return poisson_n<T, 64>(c);
        case 128: return poisson_n<T, 128>(c);
        case 256: return poisson_n<T, 256>(c);
        case 512: return poisson_n<T, 512>(c);
        case 1024: return poisson_n<T, 1024>(c);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t gradient_impl(hrt_ctx *c) {
    const int n = c->n;
    int log2n = 0;
    while ((1 << log2n) < n) ++log2n;
    const T *phi = reinterpret_cast<const T *>(c->ws + c->lay.mesh_r) + (size_t)n * n * n;
    const int64_t nodes = (int64_t)n * n * n;
    prof_begin(c);
    fd4_gradient_kernel<T><<<(int)((nodes + kThreads - 1) / kThreads), kThreads, 0, c->stream>>>(
        phi, reinterpret_cast<v4<T> *>(c->ws + c->lay.grad), n, log2n, (T)(1.0 / (12.0 * c->cell)));
    prof_end(c, K_GRADIENT);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_poisson(hrt_ctx *c) {
    return c->f64 ? poisson_impl<double>(c) : poisson_impl<float>(c);
}

hipError_t launch_gradient(hrt_ctx *c) {
    return c->f64 ? gradient_impl<double>(c) : gradient_impl<float>(c);
}

}  // namespace hrt
