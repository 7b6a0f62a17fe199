// Ray side of the co-evolution step.
//
// ray_step_kernel (paper Eqs. symp_1-3, kick, drift; Sec. 4.2): one lane per ray. The
// kick over lens shell n sums, for every mesh z-plane j in the shell,
//     w_j * bilinear(G_x, G_y on mesh plane j mod n)(X_obs + chi_j * theta),
// where theta = theta0 + dth is the ray's current angle and w_j carries the line-of-sight
// element, r_j, the Poisson prefactor and the growth correction of Eq. kick. Then
// p += dp and dth += d_n p (drift with the midpoint radius, Eq. drift). Positions on a
// plane are formed in FP64 (chi_j * theta reaches hundreds of Mpc/h) and the fractions
// handed to the FP32 bilinear weights. Rays are independent (Sec. 4.1), so neighbouring
// lanes are neighbouring pixels and read neighbouring mesh nodes of the same plane.
//
// convergence_kernel (Eqs. A, obs_first_set, obs_second_set): finite differences of the
// deflections over the pixel grid, central inside and second-order one-sided on the
// edges; kappa, gamma1, gamma2, omega with omega kept to first order.
#include "device_common.h"
#include "hrt_internal.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void ray_step_kernel(
    T *__restrict__ dthx, T *__restrict__ dthy, T *__restrict__ px, T *__restrict__ py,
    const PlaneEntry *__restrict__ planes, int begin, int count, const v4<T> *__restrict__ g,
    int n, double inv_cell, double obsx, double obsy, int mx, int nrays, double mux, double muy,
    double half_mx, double half_my, T d) {
    const int i = xcd_block(gridDim.x) * kThreads + threadIdx.x;
    if (i >= nrays) return;
    const int ix = i % mx, iy = i / mx;
    const double thx = ((ix + 0.5) - half_mx) * mux + (double)dthx[i];
    const double thy = ((iy + 0.5) - half_my) * muy + (double)dthy[i];
    const int m = n - 1;
    T ax = 0, ay = 0;
    for (int e = begin; e < begin + count; ++e) {
        const PlaneEntry pe = planes[e];
        const double X = (obsx + pe.chi * thx) * inv_cell;
        const double Y = (obsy + pe.chi * thy) * inv_cell;
        const double flx = floor(X), fly = floor(Y);
        const T fx = (T)(X - flx), fy = (T)(Y - fly);
        const int x0 = (int)((int64_t)flx & m), y0 = (int)((int64_t)fly & m);
        const int x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
        const v4<T> *plane = g + (size_t)pe.mesh * n * n;
        const v4<T> g00 = plane[(size_t)y0 * n + x0], g01 = plane[(size_t)y0 * n + x1];
        const v4<T> g10 = plane[(size_t)y1 * n + x0], g11 = plane[(size_t)y1 * n + x1];
        const T w00 = (T(1) - fx) * (T(1) - fy), w01 = fx * (T(1) - fy);
        const T w10 = (T(1) - fx) * fy, w11 = fx * fy;
        const T gx = w00 * g00.x + w01 * g01.x + w10 * g10.x + w11 * g11.x;
        const T gy = w00 * g00.y + w01 * g01.y + w10 * g10.y + w11 * g11.y;
        const T w = (T)pe.w;
        ax += w * gx;
        ay += w * gy;
    }
    const T npx = px[i] + ax, npy = py[i] + ay;
    px[i] = npx;
    py[i] = npy;
    dthx[i] += d * npx;
    dthy[i] += d * npy;
}

template <typename T>
__device__ __forceinline__ T fd(const T *f, int i, int k, int mk, int stride) {
    if (k == 0) return T(-3) * f[i] + T(4) * f[i + stride] - f[i + 2 * stride];
    if (k == mk - 1) return T(3) * f[i] - T(4) * f[i - stride] + f[i - 2 * stride];
    return f[i + stride] - f[i - stride];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void convergence_kernel(
    const T *__restrict__ dthx, const T *__restrict__ dthy, T *__restrict__ kappa,
    T *__restrict__ g1, T *__restrict__ g2, T *__restrict__ om, int mx, int my, T inv2mux,
    T inv2muy) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= mx * my) return;
    const int ix = i % mx, iy = i / mx;
    const T dxx = fd(dthx, i, ix, mx, 1) * inv2mux;    // d dth_x / d theta0_x = A11 - 1
    const T dxy = fd(dthx, i, iy, my, mx) * inv2muy;   // A12
    const T dyx = fd(dthy, i, ix, mx, 1) * inv2mux;    // A21
    const T dyy = fd(dthy, i, iy, my, mx) * inv2muy;   // A22 - 1
    const T k = T(-0.5) * (dxx + dyy);                 // kappa = 1 - (A11 + A22)/2
    kappa[i] = k;
    if (g1 || g2 || om) {
        const T c2v = T(0.5) * (dxy - dyx), c3 = T(0.5) * (dyy - dxx), c4 = T(0.5) * (dxy + dyx);
        const T w = c2v / (T(1) - k);
        if (om) om[i] = w;
        if (g1) g1[i] = c3 + c4 * w;
        if (g2) g2[i] = -c4 + c3 * w;
    }
}

template <typename T>
hipError_t ray_impl(hrt_ctx *c, const hrt_rays *r, int begin, int count, double d) {
    const int nrays = c->mx * c->my;
    prof_begin(c);
    ray_step_kernel<T><<<(nrays + kThreads - 1) / kThreads, kThreads, 0, c->stream>>>(
        static_cast<T *>(r->dth[0]), static_cast<T *>(r->dth[1]), static_cast<T *>(r->p[0]),
        static_cast<T *>(r->p[1]), reinterpret_cast<const PlaneEntry *>(c->ws + c->lay.planes), begin,
        count, reinterpret_cast<const v4<T> *>(c->ws + c->lay.grad), c->n, 1.0 / c->cell,
        c->cfg.observer[0], c->cfg.observer[1], c->mx, nrays, c->cfg.fov_x / c->mx,
        c->cfg.fov_y / c->my, 0.5 * c->mx, 0.5 * c->my, (T)d);
    prof_end(c, K_RAY_STEP);
    return hipGetLastError();
}

template <typename T>
hipError_t conv_impl(hrt_ctx *c, const hrt_rays *r, void *kappa, void *g1, void *g2, void *om) {
    const int nrays = c->mx * c->my;
    prof_begin(c);
    convergence_kernel<T><<<(nrays + kThreads - 1) / kThreads, kThreads, 0, c->stream>>>(
        static_cast<const T *>(r->dth[0]), static_cast<const T *>(r->dth[1]), static_cast<T *>(kappa),
        static_cast<T *>(g1), static_cast<T *>(g2), static_cast<T *>(om), c->mx, c->my,
        (T)(0.5 * c->mx / c->cfg.fov_x), (T)(0.5 * c->my / c->cfg.fov_y));
    prof_end(c, K_CONVERGENCE);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ray_step(hrt_ctx *c, const hrt_rays *r, int begin, int count, double d) {
    return c->f64 ? ray_impl<double>(c, r, begin, count, d) : ray_impl<float>(c, r, begin, count, d);
}

hipError_t launch_convergence(hrt_ctx *c, const hrt_rays *r, void *kappa, void *g1, void *g2,
                              void *om) {
    return c->f64 ? conv_impl<double>(c, r, kappa, g1, g2, om)
                  : conv_impl<float>(c, r, kappa, g1, g2, om);
}

}  // namespace hrt
