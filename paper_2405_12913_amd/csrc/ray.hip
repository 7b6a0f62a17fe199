// Ray side of the co-evolution step.
//
// ray_step_kernel (paper Eqs. symp_1-3, kick, drift; Sec. 5.2): one lane per ray. The
// kick over lens shell n sums, for every line-of-sight plane j in the shell,
//     w_j * bilinear(G_u, G_v on lens plane j)(X_obs + chi_j * theta),
// the lens plane being the transverse gradient in the frame of plane j's replica (built for
// the step by plane_gradient_kernel; 8 or 16 bytes per node),
// where theta = theta0 + dth is the ray's current angle and w_j carries the line-of-sight
// element, r_j, the Poisson prefactor and the growth correction of Eq. kick. Then
// p += dp and dth += d_n p (drift with the midpoint radius, Eq. drift). Positions on a
// plane are formed in FP64 (chi_j * theta reaches hundreds of Mpc/h) and the fractions
// handed to the FP32 bilinear weights. Rays are independent (Sec. 5.1), so neighbouring
// lanes are neighbouring pixels and read neighbouring mesh nodes of the same plane.
//
// convergence_kernel (Eqs. A, obs_first_set, obs_second_set): finite differences of the
// deflections over the pixel grid, central inside and second-order one-sided on the
// edges, or the forward-mode distortion A carried by the rays (HRT_JACOBIAN); kappa,
// gamma1, gamma2, omega with omega kept to first order.
// Both kernels cover all realisations of a context (uneven ray grids) in one launch.
#include "device_common.h"

namespace hrt {
namespace {

constexpr int kThreads = 256;

template <typename T>
struct RayR {                  // one realisation, as the ray kernels see it
    T *dthx, *dthy, *px, *py;
    T *jac[8];                 // (A - I)_xx, _xy, _yx, _yy, B_xx, _xy, _yx, _yy (HRT_JACOBIAN)
    const PlaneEntry *planes;
    const c2<T> *stack;        // the step's lens planes: (G_u, G_v) [e - begin][v][u]
    const T *sphi, *sq;        // scalar lens planes: phi (time delay), Q (line-of-sight field)
    T *delay, *los;            // accumulated per ray (HRT_TIME_DELAY, los_field)
    const c2<T> *rm;           // the step's filtered ray-mesh kick (HRT_RAY_MESH), N x N
    int rm_n;
    double rm_mu;
    T *kappa, *g1, *g2, *om;
    T *akappa, *ag1, *ag2, *aom;   // n_g-weighted sums over the source planes (Eq. obs_accum)
    T aw;                          // weight of this source plane
    int amode;                     // 0: none, 1: write aw * map, 2: add aw * map
    int begin, count, n, mx, my, nrays;
    double inv_cell, obsx, obsy, mux, muy, half_mx, half_my;
    T d, inv2mux, inv2muy;
};

template <typename T>
struct RayBatch {
    BlockMap map;
    RayR<T> r[kMaxBatch];
    int rmap, xcd;             // launch-shape variant: ray map, XCD block grouping
};

// Ray of (logical block b, thread t). Variants (identical results, each ray is
// independent): 0 = rows of the pixel grid, 1 = 16 x 16 pixel patches, 2 = 32 x 8 patches;
// a patch map falls back to rows when the grid sides are not multiples of the patch.
__device__ __forceinline__ int ray_of(int b, int t, int mx, int my, int map) {
    if (map == 1 && (mx & 15) == 0 && (my & 15) == 0) {
        const int pw = mx >> 4, bx = b % pw, by = b / pw;
        return ((by << 4) + (t >> 4)) * mx + (bx << 4) + (t & 15);
    }
    if (map == 2 && (mx & 31) == 0 && (my & 7) == 0) {
        const int pw = mx >> 5, bx = b % pw, by = b / pw;
        return ((by << 3) + (t >> 5)) * mx + (bx << 5) + (t & 31);
    }
    return b * kThreads + t;
}

// XT: the time delay (phi planes, weight w_j / chi_j: the Shapiro term -2 Phi_j/c^2 cell)
// and/or the line-of-sight integral (Q planes, weight los_w_j) are accumulated too; the
// delay also gets the drift's geometric term p^2 d / 2 with the drift momentum.
template <typename T, bool JAC, bool XT>
__global__ __launch_bounds__(kThreads) void ray_step_kernel(RayBatch<T> b) {
    const int blk = logical_block(b.xcd);
    const int r = real_of(b.map, blk);
    const RayR<T> &a = b.r[r];
    const int i = ray_of(blk - b.map.start[r], threadIdx.x, a.mx, a.my, b.rmap);
    if (i >= a.nrays) return;
    const int ix = i % a.mx, iy = i / a.mx;
    const double thx = ((ix + 0.5) - a.half_mx) * a.mux + (double)a.dthx[i];
    const double thy = ((iy + 0.5) - a.half_my) * a.muy + (double)a.dthy[i];
    const int n = a.n, m = n - 1;
    T ax = 0, ay = 0;
    T j00 = 0, j01 = 0, j10 = 0, j11 = 0;        // d kick / d theta (JAC)
    T shap = 0, losacc = 0;                      // Shapiro and line-of-sight sums (XT)
    // The kick reads every plane at the step's starting angles, so the planes are
    // independent: kChunk of them have their gathers in flight together, then are added in
    // plane order (the same sums as one plane at a time).
    constexpr int kChunk = 4;
    struct Sample {
        c2<T> g00, g01, g10, g11;
        T fx, fy, w, wj;
        T p00, p01, p10, p11, wd;                // phi corners, w_j / chi_j (XT)
        T q00, q01, q10, q11, lw;                // Q corners, los_w_j (XT)
    };
    auto fetch = [&](int e, Sample &q) {
        const PlaneEntry pe = a.planes[e];
        double flx, fly, frx, fry;
        plane_cell(a.obsx, pe.chi, thx, a.inv_cell, flx, frx);
        plane_cell(a.obsy, pe.chi, thy, a.inv_cell, fly, fry);
        q.fx = (T)frx;
        q.fy = (T)fry;
        q.w = (T)pe.w;
        if (JAC) q.wj = (T)(pe.w * pe.chi * a.inv_cell);
        const int x0 = (int)((int64_t)flx & m), y0 = (int)((int64_t)fly & m);
        const int x1 = (x0 + 1) & m, y1 = (y0 + 1) & m;
        const c2<T> *plane = a.stack + (size_t)(e - a.begin) * n * n;
        q.g00 = plane[(size_t)y0 * n + x0];
        q.g01 = plane[(size_t)y0 * n + x1];
        q.g10 = plane[(size_t)y1 * n + x0];
        q.g11 = plane[(size_t)y1 * n + x1];
        if (XT) {
            const size_t off = (size_t)(e - a.begin) * n * n;
            if (a.sphi) {
                const T *ph = a.sphi + off;
                q.p00 = ph[(size_t)y0 * n + x0];
                q.p01 = ph[(size_t)y0 * n + x1];
                q.p10 = ph[(size_t)y1 * n + x0];
                q.p11 = ph[(size_t)y1 * n + x1];
                q.wd = (T)(pe.w / pe.chi);
            }
            if (a.sq) {
                const T *qp = a.sq + off;
                q.q00 = qp[(size_t)y0 * n + x0];
                q.q01 = qp[(size_t)y0 * n + x1];
                q.q10 = qp[(size_t)y1 * n + x0];
                q.q11 = qp[(size_t)y1 * n + x1];
                q.lw = (T)pe.los_w;
            }
        }
    };
    auto add = [&](const Sample &q) {
        const T fx = q.fx, fy = q.fy;
        const T w00 = (T(1) - fx) * (T(1) - fy), w01 = fx * (T(1) - fy);
        const T w10 = (T(1) - fx) * fy, w11 = fx * fy;
        const T gx = w00 * q.g00.x + w01 * q.g01.x + w10 * q.g10.x + w11 * q.g11.x;
        const T gy = w00 * q.g00.y + w01 * q.g01.y + w10 * q.g10.y + w11 * q.g11.y;
        ax += q.w * gx;
        ay += q.w * gy;
        if (XT) {
            if (a.delay) shap += q.wd * (w00 * q.p00 + w01 * q.p01 + w10 * q.p10 + w11 * q.p11);
            if (a.los) losacc += q.lw * (w00 * q.q00 + w01 * q.q01 + w10 * q.q10 + w11 * q.q11);
        }
        if (JAC) {
            // gradient of the bilinear interpolant: differences of the corner values
            const T dxu = (T(1) - fy) * (q.g01.x - q.g00.x) + fy * (q.g11.x - q.g10.x);
            const T dyu = (T(1) - fx) * (q.g10.x - q.g00.x) + fx * (q.g11.x - q.g01.x);
            const T dxv = (T(1) - fy) * (q.g01.y - q.g00.y) + fy * (q.g11.y - q.g10.y);
            const T dyv = (T(1) - fx) * (q.g10.y - q.g00.y) + fx * (q.g11.y - q.g01.y);
            j00 += q.wj * dxu;
            j01 += q.wj * dyu;
            j10 += q.wj * dxv;
            j11 += q.wj * dyv;
        }
    };
    const int e_end = a.begin + a.count;
    int e = a.begin;
    for (; e + kChunk <= e_end; e += kChunk) {
        Sample q[kChunk];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) fetch(e + k, q[k]);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) add(q[k]);
    }
    for (; e < e_end; ++e) {
        Sample q;
        fetch(e, q);
        add(q);
    }
    const T npx = a.px[i] + ax, npy = a.py[i] + ay;
    a.px[i] = npx;
    a.py[i] = npy;
    a.dthx[i] += a.d * npx;
    a.dthy[i] += a.d * npy;
    if (XT) {
        if (a.delay) a.delay[i] += shap + T(0.5) * a.d * (npx * npx + npy * npy);
        if (a.los) a.los[i] += losacc;
    }
    if (JAC) {
        // B += J (I + dA), then dA += d B (Eqs. obsv_recurse1-3, half-kicks merged)
        const T d00 = a.jac[0][i], d01 = a.jac[1][i], d10 = a.jac[2][i], d11 = a.jac[3][i];
        const T b00 = a.jac[4][i] + (j00 * (T(1) + d00) + j01 * d10);
        const T b01 = a.jac[5][i] + (j00 * d01 + j01 * (T(1) + d11));
        const T b10 = a.jac[6][i] + (j10 * (T(1) + d00) + j11 * d10);
        const T b11 = a.jac[7][i] + (j10 * d01 + j11 * (T(1) + d11));
        a.jac[4][i] = b00;
        a.jac[5][i] = b01;
        a.jac[6][i] = b10;
        a.jac[7][i] = b11;
        a.jac[0][i] = d00 + a.d * b00;
        a.jac[1][i] = d01 + a.d * b01;
        a.jac[2][i] = d10 + a.d * b10;
        a.jac[3][i] = d11 + a.d * b11;
    }
}

// The kick read from the step's ray mesh (HRT_RAY_MESH, Sec. 5.2: CIC readout at the rays'
// current angles), then the drift; JAC: J is the derivative of that bilinear readout
// (differences of the corner values / mu). Rays stay inside the mesh by its padding; the
// cell index is clamped to the mesh all the same. A step without lens planes adds no kick.
template <typename T, bool JAC>
__global__ __launch_bounds__(kThreads) void ray_mesh_step_kernel(RayBatch<T> b) {
    const int blk = logical_block(b.xcd);
    const int r = real_of(b.map, blk);
    const RayR<T> &a = b.r[r];
    const int i = ray_of(blk - b.map.start[r], threadIdx.x, a.mx, a.my, b.rmap);
    if (i >= a.nrays) return;
    T ax = 0, ay = 0, j00 = 0, j01 = 0, j10 = 0, j11 = 0;
    if (a.count > 0) {
        const int ix = i % a.mx, iy = i / a.mx, N = a.rm_n;
        const double thx = ((ix + 0.5) - a.half_mx) * a.mux + (double)a.dthx[i];
        const double thy = ((iy + 0.5) - a.half_my) * a.muy + (double)a.dthy[i];
        const double ux = (thx + 0.5 * N * a.rm_mu) / a.rm_mu, uy = (thy + 0.5 * N * a.rm_mu) / a.rm_mu;
        const int kx = min(max((int)floor(ux), 0), N - 2), ky = min(max((int)floor(uy), 0), N - 2);
        const T fx = (T)fmin(fmax(ux - kx, 0.0), 1.0), fy = (T)fmin(fmax(uy - ky, 0.0), 1.0);
        const c2<T> c00 = a.rm[(size_t)ky * N + kx], c01 = a.rm[(size_t)ky * N + kx + 1];
        const c2<T> c10 = a.rm[(size_t)(ky + 1) * N + kx], c11 = a.rm[(size_t)(ky + 1) * N + kx + 1];
        const T w00 = (T(1) - fx) * (T(1) - fy), w01 = fx * (T(1) - fy);
        const T w10 = (T(1) - fx) * fy, w11 = fx * fy;
        ax = w00 * c00.x + w01 * c01.x + w10 * c10.x + w11 * c11.x;
        ay = w00 * c00.y + w01 * c01.y + w10 * c10.y + w11 * c11.y;
        if (JAC) {
            const T inv = (T)(1.0 / a.rm_mu);
            j00 = ((T(1) - fy) * (c01.x - c00.x) + fy * (c11.x - c10.x)) * inv;
            j01 = ((T(1) - fx) * (c10.x - c00.x) + fx * (c11.x - c01.x)) * inv;
            j10 = ((T(1) - fy) * (c01.y - c00.y) + fy * (c11.y - c10.y)) * inv;
            j11 = ((T(1) - fx) * (c10.y - c00.y) + fx * (c11.y - c01.y)) * inv;
        }
    }
    const T npx = a.px[i] + ax, npy = a.py[i] + ay;
    a.px[i] = npx;
    a.py[i] = npy;
    a.dthx[i] += a.d * npx;
    a.dthy[i] += a.d * npy;
    if (JAC) {
        const T d00 = a.jac[0][i], d01 = a.jac[1][i], d10 = a.jac[2][i], d11 = a.jac[3][i];
        const T b00 = a.jac[4][i] + (j00 * (T(1) + d00) + j01 * d10);
        const T b01 = a.jac[5][i] + (j00 * d01 + j01 * (T(1) + d11));
        const T b10 = a.jac[6][i] + (j10 * (T(1) + d00) + j11 * d10);
        const T b11 = a.jac[7][i] + (j10 * d01 + j11 * (T(1) + d11));
        a.jac[4][i] = b00;
        a.jac[5][i] = b01;
        a.jac[6][i] = b10;
        a.jac[7][i] = b11;
        a.jac[0][i] = d00 + a.d * b00;
        a.jac[1][i] = d01 + a.d * b01;
        a.jac[2][i] = d10 + a.d * b10;
        a.jac[3][i] = d11 + a.d * b11;
    }
}

template <typename T>
__device__ __forceinline__ T fd(const T *f, int i, int k, int mk, int stride) {
    if (k == 0) return T(-3) * f[i] + T(4) * f[i + stride] - f[i + 2 * stride];
    if (k == mk - 1) return T(3) * f[i] - T(4) * f[i - stride] + f[i - 2 * stride];
    return f[i + stride] - f[i - stride];
}

// FROM_A: the derivatives are the forward-mode distortion dA = A - I carried by the rays
// (HRT_JACOBIAN) instead of finite differences of the deflections.
template <typename T, bool FROM_A>
__global__ __launch_bounds__(kThreads) void convergence_kernel(RayBatch<T> b) {
    const int r = real_of(b.map, blockIdx.x);
    const RayR<T> &a = b.r[r];
    const int i = (blockIdx.x - b.map.start[r]) * kThreads + threadIdx.x;
    if (i >= a.nrays) return;
    const int mx = a.mx, my = a.my, ix = i % mx, iy = i / mx;
    T dxx, dxy, dyx, dyy;
    if (FROM_A) {
        dxx = a.jac[0][i];
        dxy = a.jac[1][i];
        dyx = a.jac[2][i];
        dyy = a.jac[3][i];
    } else {
        dxx = fd<T>(a.dthx, i, ix, mx, 1) * a.inv2mux;    // d dth_x / d theta0_x = A11 - 1
        dxy = fd<T>(a.dthx, i, iy, my, mx) * a.inv2muy;   // A12
        dyx = fd<T>(a.dthy, i, ix, mx, 1) * a.inv2mux;    // A21
        dyy = fd<T>(a.dthy, i, iy, my, mx) * a.inv2muy;   // A22 - 1
    }
    const T k = T(-0.5) * (dxx + dyy);                        // kappa = 1 - (A11 + A22)/2
    if (a.kappa) a.kappa[i] = k;
    const bool acc = a.amode != 0;
    if (a.g1 || a.g2 || a.om || (acc && (a.ag1 || a.ag2 || a.aom))) {
        const T c2v = T(0.5) * (dxy - dyx), c3 = T(0.5) * (dyy - dxx), c4 = T(0.5) * (dxy + dyx);
        const T w = c2v / (T(1) - k);
        const T g1 = c3 + c4 * w, g2 = -c4 + c3 * w;
        if (a.om) a.om[i] = w;
        if (a.g1) a.g1[i] = g1;
        if (a.g2) a.g2[i] = g2;
        if (acc) {
            if (a.aom) a.aom[i] = (a.amode == 2 ? a.aom[i] : T(0)) + a.aw * w;
            if (a.ag1) a.ag1[i] = (a.amode == 2 ? a.ag1[i] : T(0)) + a.aw * g1;
            if (a.ag2) a.ag2[i] = (a.amode == 2 ? a.ag2[i] : T(0)) + a.aw * g2;
        }
    }
    if (acc && a.akappa) a.akappa[i] = (a.amode == 2 ? a.akappa[i] : T(0)) + a.aw * k;
}

template <typename T>
void fill_rays(hrt_ctx *c, int r, const StepArgs &s, int k, RayR<T> &a) {
    const Real &re = c->re[r];
    const hrt_rays &rays = s.r[r];
    a = RayR<T>{};
    a.dthx = static_cast<T *>(rays.dth[0]);
    a.dthy = static_cast<T *>(rays.dth[1]);
    a.px = static_cast<T *>(rays.p[0]);
    a.py = static_cast<T *>(rays.p[1]);
    for (int q = 0; q < 8; ++q) a.jac[q] = c->jacobian ? static_cast<T *>(rays.jac[q]) : nullptr;
    a.planes = reinterpret_cast<const PlaneEntry *>(re.ws + re.lay.planes);
    a.stack = reinterpret_cast<const c2<T> *>(re.ws + re.lay.stack);
    if (c->ray_mesh) {
        a.rm = reinterpret_cast<const c2<T> *>(re.ws + re.lay.rm_mesh);
        a.rm_n = re.tab.rm_n;
        a.rm_mu = re.tab.rm_mu[s.step];
    }
    if (c->delay) {
        a.delay = static_cast<T *>(rays.delay);
        a.sphi = reinterpret_cast<const T *>(re.ws + re.lay.stack_phi);
    }
    if (c->los) {
        a.los = static_cast<T *>(rays.los);
        a.sq = reinterpret_cast<const T *>(re.ws + (c->los == HRT_LOS_DENSITY ? re.lay.stack_delta
                                                                            : re.lay.stack_phi));
    }
    if (s.src_maps) {
        const hrt_maps &sm = s.src_maps[r], &am = s.acc_maps[r];
        a.kappa = static_cast<T *>(sm.kappa);
        a.g1 = static_cast<T *>(sm.gamma1);
        a.g2 = static_cast<T *>(sm.gamma2);
        a.om = static_cast<T *>(sm.omega);
        a.amode = s.acc_mode[r];
        if (a.amode) {
            a.akappa = static_cast<T *>(am.kappa);
            a.ag1 = static_cast<T *>(am.gamma1);
            a.ag2 = static_cast<T *>(am.gamma2);
            a.aom = static_cast<T *>(am.omega);
            a.aw = (T)s.acc_w[r];
        }
    } else if (s.kappa) {
        a.kappa = static_cast<T *>(s.kappa[r]);
        a.g1 = s.g1 ? static_cast<T *>(s.g1[r]) : nullptr;
        a.g2 = s.g2 ? static_cast<T *>(s.g2[r]) : nullptr;
        a.om = s.om ? static_cast<T *>(s.om[r]) : nullptr;
    }
    a.begin = re.tab.plane_begin[s.step];
    a.count = re.tab.plane_count[s.step];
    a.n = re.n;
    a.mx = re.mx;
    a.my = re.my;
    a.nrays = re.mx * re.my;
    a.inv_cell = 1.0 / re.cell;
    a.obsx = re.cfg.observer[0];
    a.obsy = re.cfg.observer[1];
    a.mux = re.cfg.fov_x / re.mx;
    a.muy = re.cfg.fov_y / re.my;
    a.half_mx = 0.5 * re.mx;
    a.half_my = 0.5 * re.my;
    a.d = (T)re.tab.d[s.step];
    a.inv2mux = (T)(0.5 * re.mx / re.cfg.fov_x);
    a.inv2muy = (T)(0.5 * re.my / re.cfg.fov_y);
    (void)k;
}

// MODE: 0 = ray step, 1 = maps from finite differences, 2 = maps from A, 3 = ray step with
// the ray-mesh kick
template <typename T, int MODE>
hipError_t rays_impl(hrt_ctx *c, const StepArgs &s) {
    constexpr bool CONV = MODE == 1 || MODE == 2;
    const int nre = (int)c->re.size();
    for (int r0 = 0; r0 < nre; r0 += kMaxBatch) {
        const int R = std::min(kMaxBatch, nre - r0);
        RayBatch<T> b{};
        b.map.R = R;
        b.map.start[0] = 0;
        for (int k = 0; k < R; ++k) {
            fill_rays<T>(c, r0 + k, s, k, b.r[k]);
            const RayR<T> &q = b.r[k];
            // a source-plane map launch skips realisations with nothing to write here
            const bool idle = CONV && !q.kappa && !q.g1 && !q.g2 && !q.om && q.amode == 0;
            b.map.start[k + 1] = b.map.start[k] + (idle ? 0 : (q.nrays + kThreads - 1) / kThreads);
        }
        if (b.map.start[R] == 0) continue;
        const int v = c->variant[K_RAY_STEP];
        b.rmap = v % 3;
        b.xcd = v >= 3 ? 0 : 1;
        prof_begin(c);
        if (MODE == 1) convergence_kernel<T, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        else if (MODE == 2) convergence_kernel<T, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        else if (MODE == 3 && c->jacobian) ray_mesh_step_kernel<T, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        else if (MODE == 3) ray_mesh_step_kernel<T, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        else {
            const bool xt = c->delay || c->los;
            if (c->jacobian && xt) ray_step_kernel<T, true, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
            else if (c->jacobian) ray_step_kernel<T, true, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
            else if (xt) ray_step_kernel<T, false, true><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
            else ray_step_kernel<T, false, false><<<b.map.start[R], kThreads, 0, c->stream>>>(b);
        }
        prof_end(c, CONV ? K_CONVERGENCE : K_RAY_STEP);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_ray_step(hrt_ctx *c, const StepArgs &s) {
    return c->f64 ? rays_impl<double, 0>(c, s) : rays_impl<float, 0>(c, s);
}

hipError_t launch_ray_mesh_step(hrt_ctx *c, const StepArgs &s) {
    return c->f64 ? rays_impl<double, 3>(c, s) : rays_impl<float, 3>(c, s);
}

hipError_t launch_convergence(hrt_ctx *c, const StepArgs &s, bool from_a) {
    if (from_a) return c->f64 ? rays_impl<double, 2>(c, s) : rays_impl<float, 2>(c, s);
    return c->f64 ? rays_impl<double, 1>(c, s) : rays_impl<float, 1>(c, s);
}

}  // namespace hrt
