// Reverse mode of the co-evolution step and of the convergence map (vector-Jacobian
// products). The paper leaves gradients through HRT to future work (Sec. 6: the adjoint
// method of its ref. LiEtAl2024); this is the hand-written adjoint of the discretisation
// the forward kernels compute.
//
// Step n, forward: G = D L paint(q + s); p' = p + K readout(G, q + s); s' = s + D_n p';
// p_r' = p_r + sum_j w_j B_j(G, X_obs + chi_j theta); dth' = dth + d_n p_r'.
// Reverse, from the cotangents after the step (in place):
//   1. recompute G for the state before the step (pm_force);
//   2. p_bar += D s_bar, p_r_bar += d dth_bar                         (prep kernels)
//   3. rays: dth_bar += sum_j w_j chi_j / cell (dB_j/du)^T p_r_bar; G_bar += bilinear
//      scatter of w_j p_r_bar                                          (ray_vjp_kernel)
//   4. matter: s_bar += K (d readout / dx)^T p_bar; G_bar += trilinear scatter of K p_bar
//                                                                      (matter_vjp_kernel)
//   5. phi_bar = -sum_d D_d G_bar_d (4th-order differences are antisymmetric), delta_bar =
//      L phi_bar (the Poisson operator is symmetric), s_bar += (d paint / dx)^T delta_bar
//      / rho_bar                                                       (paint_vjp_kernel)
// G_bar is accumulated in 64-bit fixed point with a scale set on the device from the
// largest contribution: one unit is 2^-(62 - h) of it, h = log2 of the most contributions
// a node can receive (particles plus ray-plane crossings), so no sum overflows. The sum is
// exact and order-independent: reruns are bit-identical and no floating-point atomics are
// used.
#include <algorithm>
#include <cmath>

#include "device_common.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;

template <typename T>
struct AdjArgs {
    // state before the step
    const T *s[3];
    const T *dth[2];
    // cotangents (in place)
    T *sb[3], *pb[3], *db[2], *prb[2];
    const v4<T> *grad;          // G of the step (forward), later reused for G_bar
    v4<T> *gout;
    unsigned long long *gbar;   // 3 x n^3 fixed-point accumulators
    unsigned long long *maxbits;// largest |contribution| (double bits)
    const T *phi;               // delta_bar after the Poisson solve
    T *div;                     // phi_bar
    const PlaneEntry *planes;
    int begin, count;
    int n, lnp, ratio, P, mx, my, nrays;
    int hbits;                  // log2 bound of the contributions per node
    double inv_cell, K, D, d, wmax, rho_bar;
    double obsx, obsy, mux, muy, half_mx, half_my;
};

__device__ __forceinline__ void atomic_max_abs(unsigned long long *slot, double v) {
    atomicMax(slot, (unsigned long long)__double_as_longlong(fabs(v)));
}

__device__ __forceinline__ double fixed_scale(const unsigned long long *maxbits, int hbits) {
    const double m = __longlong_as_double((long long)*maxbits);
    if (!(m > 0.0)) return 1.0;
    int e;
    frexp(m, &e);                                   // m < 2^e
    return ldexp(1.0, 62 - hbits - e);
}

__device__ __forceinline__ void add_fixed(unsigned long long *slot, double v, double scale) {
    atomicAdd(slot, (unsigned long long)llrint(v * scale));
}

template <typename T>
__global__ void adj_zero_kernel(AdjArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    if (i < 3 * n3) a.gbar[i] = 0ull;
    if (i == 0) *a.maxbits = 0ull;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void matter_vjp_prep_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.P) return;
    double m = 0.0;
    for (int d = 0; d < 3; ++d) {
        const T pt = a.pb[d][i] + (T)a.D * a.sb[d][i];
        a.pb[d][i] = pt;
        m = fmax(m, fabs(a.K * (double)pt));
    }
    atomic_max_abs(a.maxbits, m);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void ray_vjp_prep_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nrays) return;
    double m = 0.0;
    for (int d = 0; d < 2; ++d) {
        const T pt = a.prb[d][i] + (T)a.d * a.db[d][i];
        a.prb[d][i] = pt;
        m = fmax(m, fabs(a.wmax * (double)pt));
    }
    atomic_max_abs(a.maxbits, m);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void ray_vjp_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.nrays) return;
    const double scale = fixed_scale(a.maxbits, a.hbits);
    const int ix = i % a.mx, iy = i / a.mx;
    const double thx = ((ix + 0.5) - a.half_mx) * a.mux + (double)a.dth[0][i];
    const double thy = ((iy + 0.5) - a.half_my) * a.muy + (double)a.dth[1][i];
    const int n = a.n, m = n - 1;
    const double ptx = a.prb[0][i], pty = a.prb[1][i];
    double tbx = 0.0, tby = 0.0;
    const size_t n3 = (size_t)n * n * n;
    for (int e = a.begin; e < a.begin + a.count; ++e) {
        const PlaneEntry pe = a.planes[e];
        const double X = (a.obsx + pe.chi * thx) * a.inv_cell;
        const double Y = (a.obsy + pe.chi * thy) * a.inv_cell;
        const double flx = floor(X), fly = floor(Y);
        const T fx = (T)(X - flx), fy = (T)(Y - fly);
        const int x0 = (int)((int64_t)flx & m), y0 = (int)((int64_t)fly & m);
        const int x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
        const size_t base = (size_t)pe.mesh * n * n;
        const size_t i00 = base + (size_t)y0 * n + x0, i01 = base + (size_t)y0 * n + x1;
        const size_t i10 = base + (size_t)y1 * n + x0, i11 = base + (size_t)y1 * n + x1;
        const v4<T> g00 = a.grad[i00], g01 = a.grad[i01], g10 = a.grad[i10], g11 = a.grad[i11];
        // d bilinear / du (cell units) for the two components
        const T dxa = (T(1) - fy) * (g01.x - g00.x) + fy * (g11.x - g10.x);
        const T dya = (T(1) - fx) * (g10.x - g00.x) + fx * (g11.x - g01.x);
        const T dxb = (T(1) - fy) * (g01.y - g00.y) + fy * (g11.y - g10.y);
        const T dyb = (T(1) - fx) * (g10.y - g00.y) + fx * (g11.y - g01.y);
        const double f = pe.w * pe.chi * a.inv_cell;
        tbx += f * (ptx * (double)dxa + pty * (double)dxb);
        tby += f * (ptx * (double)dya + pty * (double)dyb);
        const double wx0 = 1.0 - (double)fx, wx1 = fx, wy0 = 1.0 - (double)fy, wy1 = fy;
        const double cw[4] = {wx0 * wy0, wx1 * wy0, wx0 * wy1, wx1 * wy1};
        const size_t id[4] = {i00, i01, i10, i11};
        for (int c = 0; c < 4; ++c) {
            add_fixed(a.gbar + id[c], pe.w * cw[c] * ptx, scale);
            add_fixed(a.gbar + n3 + id[c], pe.w * cw[c] * pty, scale);
        }
    }
    a.db[0][i] += (T)tbx;
    a.db[1][i] += (T)tby;
}

template <typename T>
__device__ __forceinline__ void cell_of(const AdjArgs<T> &a, int i, int c[3], double f[3]) {
    const int pmk = (1 << a.lnp) - 1;
    const int lat[3] = {i & pmk, (i >> a.lnp) & pmk, i >> (2 * a.lnp)};
    for (int d = 0; d < 3; ++d) {
        T fd;
        axis_cell<T>(a.s[d][i], lat[d], a.ratio, (T)a.inv_cell, a.n - 1, c[d], fd);
        f[d] = fd;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void matter_vjp_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= a.P) return;
    const double scale = fixed_scale(a.maxbits, a.hbits);
    int c[3];
    double f[3];
    cell_of(a, i, c, f);
    const int n = a.n;
    const size_t n3 = (size_t)n * n * n;
    const double pt[3] = {a.pb[0][i], a.pb[1][i], a.pb[2][i]};
    double xb[3] = {0.0, 0.0, 0.0};
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                const double w1[3] = {cx ? f[0] : 1.0 - f[0], cy ? f[1] : 1.0 - f[1], cz ? f[2] : 1.0 - f[2]};
                const double s1[3] = {cx ? 1.0 : -1.0, cy ? 1.0 : -1.0, cz ? 1.0 : -1.0};
                const size_t node = ((size_t)((c[2] + cz) & (n - 1)) * n + ((c[1] + cy) & (n - 1))) * n +
                                    ((c[0] + cx) & (n - 1));
                const v4<T> g = a.grad[node];
                const double gp = pt[0] * (double)g.x + pt[1] * (double)g.y + pt[2] * (double)g.z;
                xb[0] += gp * s1[0] * w1[1] * w1[2];
                xb[1] += gp * w1[0] * s1[1] * w1[2];
                xb[2] += gp * w1[0] * w1[1] * s1[2];
                const double w = w1[0] * w1[1] * w1[2];
                for (int d = 0; d < 3; ++d) add_fixed(a.gbar + d * n3 + node, a.K * w * pt[d], scale);
            }
    for (int d = 0; d < 3; ++d) a.sb[d][i] += (T)(a.K * a.inv_cell * xb[d]);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void gbar_convert_kernel(AdjArgs<T> a) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    if (i >= n3) return;
    const double inv = 1.0 / fixed_scale(a.maxbits, a.hbits);
    v4<T> o;
    o.x = (T)((double)(long long)a.gbar[i] * inv);
    o.y = (T)((double)(long long)a.gbar[n3 + i] * inv);
    o.z = (T)((double)(long long)a.gbar[2 * n3 + i] * inv);
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
__global__ __launch_bounds__(kThreads) void paint_vjp_kernel(AdjArgs<T> a) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
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
AdjArgs<T> adj_args(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                    const hrt_rays *rc, int step) {
    const Real &re = c->re[0];
    AdjArgs<T> a{};
    for (int d = 0; d < 3; ++d) {
        a.s[d] = static_cast<const T *>(m->s[d]);
        a.sb[d] = static_cast<T *>(mc->s[d]);
        a.pb[d] = static_cast<T *>(mc->p[d]);
    }
    if (r) {
        for (int d = 0; d < 2; ++d) {
            a.dth[d] = static_cast<const T *>(r->dth[d]);
            a.db[d] = static_cast<T *>(rc->dth[d]);
            a.prb[d] = static_cast<T *>(rc->p[d]);
        }
    }
    const size_t n3 = (size_t)re.n * re.n * re.n;
    a.grad = reinterpret_cast<const v4<T> *>(re.ws + re.lay.grad);
    a.gout = reinterpret_cast<v4<T> *>(re.ws + re.lay.grad);
    a.gbar = reinterpret_cast<unsigned long long *>(re.ws + re.lay.adj);
    a.maxbits = a.gbar + 3 * n3;
    a.div = reinterpret_cast<T *>(re.ws + re.lay.mesh_r);
    a.phi = reinterpret_cast<const T *>(re.ws + re.lay.mesh_r) + n3;
    a.planes = reinterpret_cast<const PlaneEntry *>(re.ws + re.lay.planes);
    a.begin = re.tab.plane_begin[step];
    a.count = re.tab.plane_count[step];
    a.n = re.n;
    a.lnp = ilog2(re.np);
    a.ratio = re.n / re.np;
    a.P = re.np * re.np * re.np;
    a.mx = re.mx;
    a.my = re.my;
    a.nrays = re.mx * re.my;
    a.inv_cell = 1.0 / re.cell;
    a.K = re.tab.K[step];
    a.D = re.tab.D[step];
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
    return a;
}

inline int nb(int64_t count) { return (int)((count + kThreads - 1) / kThreads); }

template <typename T>
hipError_t step_vjp_before_poisson(hrt_ctx *c, const AdjArgs<T> &a, bool matter, bool rays) {
    hipStream_t st = c->stream;
    const int64_t n3 = (int64_t)a.n * a.n * a.n;
    adj_zero_kernel<T><<<nb(3 * n3), kThreads, 0, st>>>(a);
    if (matter) matter_vjp_prep_kernel<T><<<nb(a.P), kThreads, 0, st>>>(a);
    if (rays) ray_vjp_prep_kernel<T><<<nb(a.nrays), kThreads, 0, st>>>(a);
    if (rays) ray_vjp_kernel<T><<<nb(a.nrays), kThreads, 0, st>>>(a);
    if (matter) matter_vjp_kernel<T><<<nb(a.P), kThreads, 0, st>>>(a);
    gbar_convert_kernel<T><<<nb(n3), kThreads, 0, st>>>(a);
    fd4_div_kernel<T><<<nb(n3), kThreads, 0, st>>>(a);
    return hipGetLastError();
}

template <typename T>
hipError_t step_vjp_after_poisson(hrt_ctx *c, const AdjArgs<T> &a) {
    paint_vjp_kernel<T><<<nb(a.P), kThreads, 0, c->stream>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                           const hrt_rays *rc, int step, bool matter) {
    hipError_t e;
    if (c->f64) {
        const AdjArgs<double> a = adj_args<double>(c, m, r, mc, rc, step);
        e = step_vjp_before_poisson<double>(c, a, matter, r != nullptr);
        if (e == hipSuccess) e = launch_poisson(c);
        if (e == hipSuccess) e = step_vjp_after_poisson<double>(c, a);
    } else {
        const AdjArgs<float> a = adj_args<float>(c, m, r, mc, rc, step);
        e = step_vjp_before_poisson<float>(c, a, matter, r != nullptr);
        if (e == hipSuccess) e = launch_poisson(c);
        if (e == hipSuccess) e = step_vjp_after_poisson<float>(c, a);
    }
    return e;
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
