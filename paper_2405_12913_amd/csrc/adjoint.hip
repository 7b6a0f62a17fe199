// Reverse mode of the co-evolution step and of the convergence map (vector-Jacobian
// products). The paper leaves gradients through HRT to future work (Sec. 7: the adjoint
// method of its ref. LiEtAl2024); this is the hand-written adjoint of the discretisation
// the forward kernels compute.
//
// Step n, forward: G = D L paint(q + s); p' = p + K readout(G, q + s); s' = s + D_n p';
// p_r' = p_r + sum_j w_j B_j(G, X_obs + chi_j theta); dth' = dth + d_n p_r'.
// Reverse, from the cotangents after the step (in place):
//   1. recompute G for the state before the step (pm_force, which also bins the particles);
//   2. p_r_bar += d dth_bar                                           (ray_vjp_prep_kernel)
//   3. matter: p_bar += D s_bar; s_bar += K (d readout / dx)^T p_bar; particles re-binned
//      with their weights K p_bar                              (matter_vjp_kernel, pm.hip)
//   4. rays: dth_bar += sum_j w_j chi_j / cell (dB_j/du)^T p_r_bar; the bilinear weights
//      of w_j p_r_bar scattered into G_bar_x, G_bar_y                   (ray_vjp_kernel)
//   5. G_bar = the particles' CIC-weighted K p_bar pulled per tile + the rays' part
//                                                               (gbar_tiles_kernel, pm.hip)
//   6. phi_bar = -sum_d D_d G_bar_d (4th-order differences are antisymmetric), delta_bar =
//      L phi_bar (the Poisson operator is symmetric), s_bar += (d paint / dx)^T delta_bar
//      / rho_bar                                                       (paint_vjp_kernel)
// G_bar is summed in 64-bit fixed point (adj_fixed_scale), so the result is exact and
// order-independent: reruns are bit-identical and no floating-point atomics are used.
#include <algorithm>
#include <climits>
#include <cmath>

#include "device_common.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;
constexpr int kWaveWindow = 256;   // nodes of a wave's LDS window in the ray scatter

template <typename T>
struct AdjArgs {
    const T *s[3];               // state before the step
    const T *dth[2];
    T *sb[3], *db[2], *prb[2];   // cotangents (in place)
    const v4<T> *grad;           // G of the step (forward), later the G_bar slot
    v4<T> *gout;
    unsigned long long *gbar;    // 2 x n^3 fixed-point accumulators (rays' part)
    unsigned long long *maxbits; // largest |contribution| (double bits)
    const T *phi;                // delta_bar after the Poisson solve
    T *div;                      // phi_bar
    const PlaneEntry *planes;
    int begin, count;
    double *tbpart;              // ray VJP: per plane group, per ray (dth_bar x, y) partial sums
    int parts, chunk;            //   plane groups and plane entries per group
    int n, lnp, lratio, P, mx, my, nrays;
    int patch;                   // rays in 16 x 16 pixel patches per block
    int hbits;                   // log2 bound of the contributions per node
    double inv_cell, d, wmax, rho_bar;
    double obsx, obsy, mux, muy, half_mx, half_my;
};

template <typename T>
__global__ void adj_zero_kernel(AdjArgs<T> a, int with_gbar) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    if (with_gbar && i < 2 * n3) a.gbar[i] = 0ull;
    if (i == 0) *a.maxbits = 0ull;
}

// Ray handled by (block, thread): 16 x 16 pixel patches when both grid sides are multiples
// of 16 (a patch lands on few mesh cells of every plane), else rows of the grid.
template <typename T>
__device__ __forceinline__ int ray_of(const AdjArgs<T> &a) {
    if (!a.patch) return blockIdx.x * kThreads + threadIdx.x;
    const int pw = a.mx >> 4;
    const int bx = blockIdx.x % pw, by = blockIdx.x / pw;
    return ((by << 4) + (threadIdx.x >> 4)) * a.mx + (bx << 4) + (threadIdx.x & 15);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void ray_vjp_prep_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    double m = 0.0;
    if (i < a.nrays) {
        for (int d = 0; d < 2; ++d) {
            const T pt = a.prb[d][i] + (T)a.d * a.db[d][i];
            a.prb[d][i] = pt;
            m = fmax(m, fabs(a.wmax * (double)pt));
        }
    }
    block_max_to(a.maxbits, m);
}

__device__ __forceinline__ int wave_min(int v) {
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off));
    return v;
}
__device__ __forceinline__ int wave_max(int v) {
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
    return v;
}

// One lane per ray, the step's lens planes split over gridDim.y groups (blockIdx.y takes
// `chunk` consecutive entries; its partial dth_bar goes to tbpart). Per plane: the
// transposed bilinear derivative gathers into dth_bar,
// and the bilinear weights of w_j p_r_bar go into G_bar. A wave's rays fall on a small patch
// of the plane, so their contributions are first summed in the wave's own LDS window over
// the wave's bounding box (integer atomics, exact) and each touched node then receives one
// global atomic per wave; a box larger than the window falls back to direct atomics. The
// window is private to the wave, whose LDS operations execute in order, so no workgroup
// barrier is needed between planes (wave_barrier only keeps the compiler from moving LDS
// accesses across the phases).
template <typename T>
__global__ __launch_bounds__(kThreads) void ray_vjp_kernel(AdjArgs<T> a) {
    __shared__ unsigned long long win[kThreads / 64][2][kWaveWindow];
    const int i = ray_of(a);
    const bool valid = i < a.nrays;
    const double scale = adj_fixed_scale(a.maxbits, a.hbits);
    const int n = a.n, m = n - 1;
    const size_t n3 = (size_t)n * n * n;
    const int lane = __lane_id();
    unsigned long long *wx = win[threadIdx.x >> 6][0], *wy = win[threadIdx.x >> 6][1];
    double thx = 0.0, thy = 0.0, ptx = 0.0, pty = 0.0;
    if (valid) {
        const int ix = i % a.mx, iy = i / a.mx;
        thx = ((ix + 0.5) - a.half_mx) * a.mux + (double)a.dth[0][i];
        thy = ((iy + 0.5) - a.half_my) * a.muy + (double)a.dth[1][i];
        ptx = a.prb[0][i];
        pty = a.prb[1][i];
    }
    double tbx = 0.0, tby = 0.0;
    const int e0 = a.begin + (int)blockIdx.y * a.chunk;
    const int e1 = min(e0 + a.chunk, a.begin + a.count);
    for (int e = e0; e < e1; ++e) {
        const PlaneEntry pe = a.planes[e];
        int ux = 0, uy = 0;            // unwrapped cell of the ray on this plane
        double q[4][2];                // fixed-point contributions of the 4 corners
        if (valid) {
            double flx, fly, frx, fry;
            plane_cell(a.obsx, pe.chi, thx, a.inv_cell, flx, frx);
            plane_cell(a.obsy, pe.chi, thy, a.inv_cell, fly, fry);
            ux = (int)flx;
            uy = (int)fly;
            const T fx = (T)frx, fy = (T)fry;
            const int x0 = ux & m, y0 = uy & m;
            const int x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
            const v4<T> *plane = a.grad + (size_t)pe.mesh * n * n;
            const v4<T> g00 = plane[(size_t)y0 * n + x0], g01 = plane[(size_t)y0 * n + x1];
            const v4<T> g10 = plane[(size_t)y1 * n + x0], g11 = plane[(size_t)y1 * n + x1];
            const T dxa = (T(1) - fy) * (g01.x - g00.x) + fy * (g11.x - g10.x);
            const T dya = (T(1) - fx) * (g10.x - g00.x) + fx * (g11.x - g01.x);
            const T dxb = (T(1) - fy) * (g01.y - g00.y) + fy * (g11.y - g10.y);
            const T dyb = (T(1) - fx) * (g10.y - g00.y) + fx * (g11.y - g01.y);
            const double f = pe.w * pe.chi * a.inv_cell;
            tbx += f * (ptx * (double)dxa + pty * (double)dxb);
            tby += f * (ptx * (double)dya + pty * (double)dyb);
            const double wx0 = 1.0 - (double)fx, wx1 = fx, wy0 = 1.0 - (double)fy, wy1 = fy;
            const double cw[4] = {wx0 * wy0, wx1 * wy0, wx0 * wy1, wx1 * wy1};
            for (int c = 0; c < 4; ++c) {
                q[c][0] = pe.w * cw[c] * ptx * scale;
                q[c][1] = pe.w * cw[c] * pty * scale;
            }
        }
        // bounding box of the wave's cells on this plane (uniform over the wave)
        const int bx0 = wave_min(valid ? ux : INT_MAX), by0 = wave_min(valid ? uy : INT_MAX);
        const int bx1 = wave_max(valid ? ux : INT_MIN), by1 = wave_max(valid ? uy : INT_MIN);
        if (bx1 < bx0) continue;                   // no valid ray in this wave
        const long long W = (long long)bx1 - bx0 + 2, H = (long long)by1 - by0 + 2;
        const size_t base = (size_t)pe.mesh * n * n;
        if (W * H <= kWaveWindow) {
            const int wn = (int)(W * H);
            for (int k = lane; k < wn; k += 64) {
                wx[k] = 0ull;
                wy[k] = 0ull;
            }
            __builtin_amdgcn_wave_barrier();
            if (valid) {
                const int lx = ux - bx0, ly = uy - by0;
                const int slot[4] = {ly * (int)W + lx, ly * (int)W + lx + 1, (ly + 1) * (int)W + lx,
                                     (ly + 1) * (int)W + lx + 1};
                for (int c = 0; c < 4; ++c) {
                    atomicAdd(&wx[slot[c]], (unsigned long long)llrint(q[c][0]));
                    atomicAdd(&wy[slot[c]], (unsigned long long)llrint(q[c][1]));
                }
            }
            __builtin_amdgcn_wave_barrier();
            for (int k = lane; k < wn; k += 64) {
                const unsigned long long vx = wx[k], vy = wy[k];
                if (vx | vy) {
                    const int gx = (bx0 + k % (int)W) & m, gy = (by0 + k / (int)W) & m;
                    const size_t node = base + (size_t)gy * n + gx;
                    if (vx) atomicAdd(a.gbar + node, vx);
                    if (vy) atomicAdd(a.gbar + n3 + node, vy);
                }
            }
            __builtin_amdgcn_wave_barrier();
        } else if (valid) {
            const int x0 = ux & m, y0 = uy & m, x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
            const size_t id[4] = {base + (size_t)y0 * n + x0, base + (size_t)y0 * n + x1,
                                  base + (size_t)y1 * n + x0, base + (size_t)y1 * n + x1};
            for (int c = 0; c < 4; ++c) {
                atomicAdd(a.gbar + id[c], (unsigned long long)llrint(q[c][0]));
                atomicAdd(a.gbar + n3 + id[c], (unsigned long long)llrint(q[c][1]));
            }
        }
    }
    if (valid) {
        double *tp = a.tbpart + ((size_t)blockIdx.y * a.nrays + i) * 2;
        tp[0] = tbx;
        tp[1] = tby;
    }
}

// dth_bar += the plane groups' partial sums, added in group order (deterministic).
template <typename T>
__global__ __launch_bounds__(kThreads) void ray_vjp_sum_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nrays) return;
    double sx = 0.0, sy = 0.0;
    for (int g = 0; g < a.parts; ++g) {
        const double *tp = a.tbpart + ((size_t)g * a.nrays + i) * 2;
        sx += tp[0];
        sy += tp[1];
    }
    a.db[0][i] += (T)sx;
    a.db[1][i] += (T)sy;
}

// Static lens (no matter VJP): G_bar from the rays' part only.
template <typename T>
__global__ __launch_bounds__(kThreads) void gbar_convert_kernel(AdjArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    if (i >= n3) return;
    const double inv = 1.0 / adj_fixed_scale(a.maxbits, a.hbits);
    v4<T> o;
    o.x = (T)((double)(long long)a.gbar[i] * inv);
    o.y = (T)((double)(long long)a.gbar[n3 + i] * inv);
    o.z = T(0);
    o.w = T(0);
    a.gout[i] = o;
}

// phi_bar = -(D_x G_bar_x + D_y G_bar_y + D_z G_bar_z), D the 4th-order difference / cell.
template <typename T>
__global__ __launch_bounds__(kThreads) void fd4_div_kernel(AdjArgs<T> a) {
    const int64_t idx = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int n = a.n, m = n - 1;
    if (idx >= (int64_t)n * n * n) return;
    const int x = (int)(idx % n), y = (int)((idx / n) % n), z = (int)(idx / ((int64_t)n * n));
    auto at = [&](int xx, int yy, int zz) {
        return a.gout[(((size_t)(zz & m) * n + (yy & m)) * n) + (xx & m)];
    };
    const T dx = T(8) * (at(x + 1, y, z).x - at(x - 1, y, z).x) - (at(x + 2, y, z).x - at(x - 2, y, z).x);
    const T dy = T(8) * (at(x, y + 1, z).y - at(x, y - 1, z).y) - (at(x, y + 2, z).y - at(x, y - 2, z).y);
    const T dz = T(8) * (at(x, y, z + 1).z - at(x, y, z - 1).z) - (at(x, y, z + 2).z - at(x, y, z - 2).z);
    a.div[idx] = -(dx + dy + dz) * (T)(a.inv_cell / 12.0);
}

template <typename T>
__device__ __forceinline__ void cell_of(const AdjArgs<T> &a, int i, int c[3], double f[3]) {
    const int pmk = (1 << a.lnp) - 1;
    const int lat[3] = {i & pmk, (i >> a.lnp) & pmk, i >> (2 * a.lnp)};
    for (int d = 0; d < 3; ++d) {
        T fd;
        axis_cell<T>(a.s[d][i], lat[d], a.lratio, (T)a.inv_cell, a.n - 1, c[d], fd);
        f[d] = fd;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void paint_vjp_kernel(AdjArgs<T> a) {
    const int i = particle_of(xcd_block(gridDim.x), threadIdx.x, a.lnp);
    if (i >= a.P) return;
    int c[3];
    double f[3];
    cell_of(a, i, c, f);
    const int n = a.n;
    double xb[3] = {0.0, 0.0, 0.0};
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const double w1[3] = {cx ? f[0] : 1.0 - f[0], cy ? f[1] : 1.0 - f[1], cz ? f[2] : 1.0 - f[2]};
                const double s1[3] = {cx ? 1.0 : -1.0, cy ? 1.0 : -1.0, cz ? 1.0 : -1.0};
                const size_t node = ((size_t)((c[2] + cz) & (n - 1)) * n + ((c[1] + cy) & (n - 1))) * n +
                                    ((c[0] + cx) & (n - 1));
                const double v = a.phi[node];
                xb[0] += v * s1[0] * w1[1] * w1[2];
                xb[1] += v * w1[0] * s1[1] * w1[2];
                xb[2] += v * w1[0] * w1[1] * s1[2];
            }
    const double fac = a.inv_cell / a.rho_bar;
    for (int d = 0; d < 3; ++d) a.sb[d][i] += (T)(fac * xb[d]);
}

// Transposed finite-difference stencil along one axis (unscaled) at index k of mk points.
template <typename T>
__device__ __forceinline__ double fd_t(const T *g, int i, int k, int mk, int stride) {
    double s = 0.0;
    if (k - 1 >= 1 && k - 1 <= mk - 2) s += g[i - stride];
    if (k + 1 >= 1 && k + 1 <= mk - 2) s -= g[i + stride];
    if (k == 0) s += -3.0 * g[i];
    if (k == 1) s += 4.0 * g[i - stride];
    if (k == 2) s += -1.0 * g[i - 2 * stride];
    if (k == mk - 1) s += 3.0 * g[i];
    if (k == mk - 2) s += -4.0 * g[i + stride];
    if (k == mk - 3) s += 1.0 * g[i + 2 * stride];
    return s;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void convergence_vjp_kernel(const T *__restrict__ kb,
                                                                   T *__restrict__ dbx,
                                                                   T *__restrict__ dby, int mx,
                                                                   int my, double inv2mux,
                                                                   double inv2muy) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= mx * my) return;
    const int ix = i % mx, iy = i / mx;
    dbx[i] += (T)(-0.5 * inv2mux * fd_t(kb, i, ix, mx, 1));
    dby[i] += (T)(-0.5 * inv2muy * fd_t(kb, i, iy, my, mx));
}

template <typename T>
AdjArgs<T> adj_args(hrt_ctx *c, int k, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                    const hrt_rays *rc, int step, AdjScratch &sc) {
    const Real &re = c->re[k];
    AdjArgs<T> a{};
    for (int d = 0; d < 3; ++d) {
        a.s[d] = static_cast<const T *>(m->s[d]);
        a.sb[d] = static_cast<T *>(mc->s[d]);
    }
    if (r) {
        for (int d = 0; d < 2; ++d) {
            a.dth[d] = static_cast<const T *>(r->dth[d]);
            a.db[d] = static_cast<T *>(rc->dth[d]);
            a.prb[d] = static_cast<T *>(rc->p[d]);
        }
    }
    const size_t n3 = (size_t)re.n * re.n * re.n;
    const size_t P = (size_t)re.np * re.np * re.np;
    a.grad = reinterpret_cast<const v4<T> *>(re.ws + re.lay.grad);
    a.gout = reinterpret_cast<v4<T> *>(re.ws + re.lay.grad);
    a.gbar = reinterpret_cast<unsigned long long *>(re.ws + re.lay.adj);
    a.maxbits = a.gbar + 2 * n3;
    a.div = reinterpret_cast<T *>(re.ws + re.lay.mesh_r);
    a.phi = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r) + n3;
    a.planes = reinterpret_cast<const PlaneEntry *>(re.ws + re.lay.planes);
    a.begin = re.tab.plane_begin[step];
    a.count = re.tab.plane_count[step];
    a.n = re.n;
    a.lnp = ilog2(re.np);
    a.lratio = ilog2(re.n / re.np);
    a.P = (int)P;
    a.mx = re.mx;
    a.my = re.my;
    a.nrays = re.mx * re.my;
    a.patch = (re.mx % 16 == 0 && re.my % 16 == 0) ? 1 : 0;
    a.inv_cell = 1.0 / re.cell;
    a.d = re.tab.d[step];
    double wmax = 0.0;
    for (int e = a.begin; e < a.begin + a.count; ++e) wmax = std::max(wmax, std::fabs(re.tab.plane_w[e]));
    a.wmax = wmax;
    // most contributions to one node: every particle, plus every ray on every plane entry
    const double bound = (double)a.P + (double)a.nrays * std::max(a.count, 1) + 1.0;
    a.hbits = (int)std::ceil(std::log2(bound)) + 1;
    a.rho_bar = (double)a.P / (double)n3;
    a.obsx = re.cfg.observer[0];
    a.obsy = re.cfg.observer[1];
    a.mux = re.cfg.fov_x / std::max(re.mx, 1);
    a.muy = re.cfg.fov_y / std::max(re.my, 1);
    a.half_mx = 0.5 * re.mx;
    a.half_my = 0.5 * re.my;
    sc.gbar = a.gbar;
    sc.maxbits = a.maxbits;
    sc.wsorted = re.ws + re.lay.adj + 2 * n3 * 8 + 256;
    a.tbpart = reinterpret_cast<double *>(re.ws + re.lay.adj + 2 * n3 * 8 + 256 + P * 4 * sizeof(T));
    a.parts = std::max(1, std::min(kRayVjpParts, a.count));
    a.chunk = (a.count + a.parts - 1) / a.parts;
    sc.hbits = a.hbits;
    return a;
}

inline int nb(int64_t count) { return (int)((count + kThreads - 1) / kThreads); }

// Reverse of step `step` for realisation k (m, r, mc, rc point to that realisation's
// state and cotangents; r and rc are NULL without the ray part, matter = false leaves out
// the matter kick-drift).
template <typename T>
hipError_t step_vjp_one(hrt_ctx *c, int k, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                        const hrt_rays *rc, int step, bool matter) {
    AdjScratch sc{};
    const AdjArgs<T> a = adj_args<T>(c, k, m, r, mc, rc, step, sc);
    const bool rays = r != nullptr;
    hipStream_t st = c->stream;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    const bool zero_gbar = rays || !matter;
    adj_zero_kernel<T><<<zero_gbar ? nb(2 * n3) : 1, kThreads, 0, st>>>(a, zero_gbar ? 1 : 0);
    if (rays) ray_vjp_prep_kernel<T><<<nb(a.nrays), kThreads, 0, st>>>(a);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && matter) e = launch_matter_vjp(c, k, m, mc, step, sc);
    if (e != hipSuccess) return e;
    if (rays) {
        ray_vjp_kernel<T><<<dim3(nb(a.nrays), a.parts), kThreads, 0, st>>>(a);
        ray_vjp_sum_kernel<T><<<nb(a.nrays), kThreads, 0, st>>>(a);
    }
    if (matter) e = launch_gbar_tiles(c, k, rays, sc);
    else gbar_convert_kernel<T><<<nb(n3), kThreads, 0, st>>>(a);
    if (e != hipSuccess) return e;
    fd4_div_kernel<T><<<nb(n3), kThreads, 0, st>>>(a);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_poisson(c, k);
    if (e == hipSuccess) paint_vjp_kernel<T><<<nb(a.P), kThreads, 0, st>>>(a);
    return e == hipSuccess ? hipGetLastError() : e;
}

// Every realisation of the context in turn (the force meshes were recomputed for all of
// them together; each realisation's reverse-mode scratch is its own).
template <typename T>
hipError_t step_vjp_impl(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                         const hrt_rays *rc, int step, bool matter) {
    for (int k = 0; k < (int)c->re.size(); ++k)
        if (hipError_t e = step_vjp_one<T>(c, k, &m[k], r ? &r[k] : nullptr, &mc[k], rc ? &rc[k] : nullptr,
                                           step, matter))
            return e;
    return hipSuccess;
}

}  // namespace

hipError_t launch_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                           const hrt_rays *rc, int step, bool matter) {
    return c->f64 ? step_vjp_impl<double>(c, m, r, mc, rc, step, matter)
                  : step_vjp_impl<float>(c, m, r, mc, rc, step, matter);
}

hipError_t launch_convergence_vjp(hrt_ctx *c, int realisation, const void *kappa_bar,
                                  const hrt_rays *rc) {
    const Real &re = c->re[realisation];
    const int nrays = re.mx * re.my;
    const double i2x = 0.5 * re.mx / re.cfg.fov_x, i2y = 0.5 * re.my / re.cfg.fov_y;
    if (c->f64)
        convergence_vjp_kernel<double><<<nb(nrays), kThreads, 0, c->stream>>>(
            static_cast<const double *>(kappa_bar), static_cast<double *>(rc->dth[0]),
            static_cast<double *>(rc->dth[1]), re.mx, re.my, i2x, i2y);
    else
        convergence_vjp_kernel<float><<<nb(nrays), kThreads, 0, c->stream>>>(
            static_cast<const float *>(kappa_bar), static_cast<float *>(rc->dth[0]),
            static_cast<float *>(rc->dth[1]), re.mx, re.my, i2x, i2y);
    return hipGetLastError();
}

}  // namespace hrt
