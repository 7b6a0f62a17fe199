// Host FP64 step tables: background cosmology, matter kick/drift factors, ray drift
// factors and the lens-shell plane lists with their kick weights.
//
// Paper passages: Poisson prefactor (3/2) Omega_m H0^2 / a (Sec. 2); flat universe,
// r = chi (Sec. 2); KDK ray integrator with kick and drift operators (Sec. 3.1,
// Eqs. symp_1-3, kick_notimecor, drift); growth correction of the potential inside a
// shell (Sec. 3.2, Eq. kick); mesh points of the 3D mesh inside the lens shell
// chi_a <= chi < chi_b carry the kick (Sec. 5.2).
//
// Readings (fused leapfrog, half points, shell membership) are stated next to each
// function. Integrals use adaptive Gauss-Kronrod (7/15) on substituted integrands
// a = t^2 that are smooth down to a = 0.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <functional>
#include <vector>

#include "hrt_internal.h"

namespace hrt {
namespace {

constexpr double kC = 299792.458;             // km/s
constexpr double kCH0 = kC / 100.0;           // c/H0 [Mpc/h]
constexpr double kG = 4.30091e-9;             // Mpc (km/s)^2 / Msun
constexpr double kGoverC2 = kG / (kC * kC);   // Mpc/h per Msun/h
constexpr double kPi = 3.14159265358979323846;

// Gauss-Kronrod 15-point nodes and weights (the 7-point Gauss rule is embedded).
const double kXgk[8] = {0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
                        0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
                        0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
                        0.207784955007898467600689403773245, 0.0};
const double kWgk[8] = {0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
                        0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
                        0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
                        0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
const double kWg[4] = {0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
                       0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

double gk15(const std::function<double(double)> &f, double a, double b, double *err) {
    double c = 0.5 * (a + b), h = 0.5 * (b - a);
    double fc = f(c);
    double rk = fc * kWgk[7], rg = fc * kWg[3];
    for (int j = 0; j < 7; ++j) {
        double x = h * kXgk[j];
        double f1 = f(c - x), f2 = f(c + x);
        rk += kWgk[j] * (f1 + f2);
        if (j % 2 == 1) rg += kWg[j / 2] * (f1 + f2);
    }
    *err = std::fabs((rk - rg) * h);
    return rk * h;
}

// Global adaptive quadrature: keep bisecting the sub-interval with the largest error
// estimate (a heap) until the summed error is below 1e-14 of the result (or 1e-300
// absolute) or the worst estimate is at rounding level, with at most 2000 bisections, so
// the cost is bounded whatever the integrand. Pieces are summed in order of position.
double integrate(const std::function<double(double)> &f, double a, double b, int n_init = 1) {
    if (a == b) return 0.0;
    struct Piece { double a, b, val, err; };
    auto less = [](const Piece &x, const Piece &y) { return x.err < y.err; };
    std::vector<Piece> heap;         // max-heap on the error estimate
    heap.reserve(4096 + n_init);
    double total = 0.0, total_err = 0.0;
    for (int i = 0; i < n_init; ++i) {       // optional initial equal partition
        const double lo = a + (b - a) * i / n_init, hi = a + (b - a) * (i + 1) / n_init;
        double err;
        const double val = gk15(f, lo, hi, &err);
        heap.push_back({lo, hi, val, err});
        total += val;
        total_err += err;
    }
    std::make_heap(heap.begin(), heap.end(), less);
    for (int it = 0; it < 2000; ++it) {
        if (total_err <= std::max(1e-14 * std::fabs(total), 1e-300)) break;
        const Piece p = heap.front();
        // the worst piece's estimate is at rounding level: no bisection can improve it
        if (p.err <= 1e-15 * std::fabs(p.val)) break;
        std::pop_heap(heap.begin(), heap.end(), less);
        heap.pop_back();
        const double m = 0.5 * (p.a + p.b);
        double e1, e2;
        const double v1 = gk15(f, p.a, m, &e1), v2 = gk15(f, m, p.b, &e2);
        heap.push_back({p.a, m, v1, e1});
        std::push_heap(heap.begin(), heap.end(), less);
        heap.push_back({m, p.b, v2, e2});
        std::push_heap(heap.begin(), heap.end(), less);
        total += v1 + v2 - p.val;
        total_err += e1 + e2 - p.err;
    }
    std::sort(heap.begin(), heap.end(), [](const Piece &x, const Piece &y) { return x.a < y.a; });
    double sum = 0.0;
    for (const Piece &p : heap) sum += p.val;
    return sum;
}

struct Cosmo {
    double om, ol;
    double E(double a) const { return std::sqrt(om / (a * a * a) + ol); }
    // int_{a0}^{a1} da / (a^2 E) with a = t^2:  2 dt / sqrt(om + ol t^6)
    double kick(double a0, double a1) const {
        return integrate([this](double t) { return 2.0 / std::sqrt(om + ol * std::pow(t, 6)); },
                         std::sqrt(a0), std::sqrt(a1));
    }
    // int_{a0}^{a1} da / (a^3 E) with a = t^2:  2 dt / (t^2 sqrt(om + ol t^6))
    double drift(double a0, double a1) const {
        return integrate(
            [this](double t) { return 2.0 / (t * t * std::sqrt(om + ol * std::pow(t, 6))); },
            std::sqrt(a0), std::sqrt(a1));
    }
    double chi(double a) const { return kCH0 * kick(a, 1.0); }
    // a(chi): Newton on chi(a) - chi (d chi/da = -c/H0 / (a^2 E)), safeguarded by bisection.
    double a_of_chi(double x) const {
        if (x == 0.0) return 1.0;
        double lo = 1e-8, hi = 1.0, a = 0.5;
        for (int it = 0; it < 200; ++it) {
            double g = chi(a) - x;          // decreasing in a
            if (g > 0) lo = a; else hi = a;
            double an = a + g / (kCH0 / (a * a * E(a)));
            if (!(an > lo && an < hi)) an = 0.5 * (lo + hi);
            if (std::fabs(an - a) <= 1e-16 * a) { a = an; break; }
            a = an;
        }
        return a;
    }
    // D1(a) = (5 om / 2) E(a) int_0^a da'/(a' E)^3, with a' = t^2: 2 t^4 (om + ol t^6)^(-3/2)
    double D1(double a) const {
        double I = integrate([this](double t) {
            double t2 = t * t;
            return 2.0 * t2 * t2 / std::pow(om + ol * t2 * t2 * t2, 1.5);
        }, 0.0, std::sqrt(a));
        return 2.5 * om * E(a) * I;
    }
};

// Planes j with lo <= j*cell - z_obs < hi (lo/hi sorted): shells are half-open in
// absolute chi, so a schedule run backwards selects exactly the same planes.
void shell_planes(double x0, double x1, double cell, double z_obs, std::vector<int64_t> &out) {
    double a = std::min(x0, x1), b = std::max(x0, x1);
    int64_t j0 = (int64_t)std::floor((a + z_obs) / cell) - 1;
    int64_t j1 = (int64_t)std::ceil((b + z_obs) / cell) + 1;
    out.clear();
    for (int64_t j = j0; j <= j1; ++j) {
        double c = (double)j * cell - z_obs;
        if (a <= c && c < b) out.push_back(j);
    }
}

// Growth ODEs in ln a (' = d/dln a, Om(a) = om a^-3 / E^2):
//   D1'' + (2 + dlnE/dlna) D1' - 1.5 Om(a) D1 = 0
//   D2'' + (2 + dlnE/dlna) D2' - 1.5 Om(a) D2 = -1.5 Om(a) D1^2
// from deep matter domination (D1 = a, D2 = -3/7 a^2), classical RK4 in ln a.
void growth_rk4(double om, double a_end, double out[4]) {
    const double ol = 1.0 - om;
    auto rhs = [&](double lna, const double *y, double *dy) {
        const double a = std::exp(lna);
        const double e2 = om / (a * a * a) + ol;
        const double oma = om / (a * a * a) / e2;
        const double dlnE = -1.5 * oma;
        dy[0] = y[1];
        dy[1] = -(2.0 + dlnE) * y[1] + 1.5 * oma * y[0];
        dy[2] = y[3];
        dy[3] = -(2.0 + dlnE) * y[3] + 1.5 * oma * y[2] - 1.5 * oma * y[0] * y[0];
    };
    const double a0 = 1e-5;
    double y[4] = {a0, a0, -3.0 / 7.0 * a0 * a0, -6.0 / 7.0 * a0 * a0};
    const double x0 = std::log(a0), x1 = std::log(a_end);
    const int steps = 20000;
    const double h = (x1 - x0) / steps;
    double k1[4], k2[4], k3[4], k4[4], t[4];
    for (int s = 0; s < steps; ++s) {
        const double x = x0 + s * h;
        rhs(x, y, k1);
        for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k1[i];
        rhs(x + 0.5 * h, t, k2);
        for (int i = 0; i < 4; ++i) t[i] = y[i] + 0.5 * h * k2[i];
        rhs(x + 0.5 * h, t, k3);
        for (int i = 0; i < 4; ++i) t[i] = y[i] + h * k3[i];
        rhs(x + h, t, k4);
        for (int i = 0; i < 4; ++i) y[i] += h / 6.0 * (k1[i] + 2 * k2[i] + 2 * k3[i] + k4[i]);
    }
    out[0] = y[0];
    out[1] = y[1] / y[0];
    out[2] = y[2];
    out[3] = y[3] / y[2];
}

}  // namespace

// Eisenstein & Hu (1998) no-wiggle transfer function parameters (their Eqs. 26, 31),
// sigma_8 normalisation (top-hat of 8 Mpc/h at a = 1) and the 2LPT growth factors.
int ic_params(const hrt_config &c, const hrt_ic_params &in, IcParams &p, std::string &err) {
    if (c.flags & HRT_STATIC) { err = "initial conditions need a cosmological configuration"; return HRT_ESTATE; }
    if (!(in.a > 0 && in.a <= 1) || !(in.h > 0) || !(in.sigma8 > 0) || !(in.omega_b >= 0) ||
        !(in.omega_b < c.omega_m) || !(in.t_cmb > 0) || !std::isfinite(in.n_s)) {
        err = "invalid initial-condition parameters";
        return HRT_EINVAL;
    }
    const double om = c.omega_m, h = in.h;
    const double theta = in.t_cmb / 2.7, om_h2 = om * h * h, ob_h2 = in.omega_b * h * h;
    const double fb = in.omega_b / om;
    p.omega_m = om;
    p.h = h;
    p.n_s = in.n_s;
    p.s_sound = 44.5 * std::log(9.83 / om_h2) / std::sqrt(1.0 + 10.0 * std::pow(ob_h2, 0.75));
    p.alpha = 1.0 - 0.328 * std::log(431.0 * om_h2) * fb + 0.38 * std::log(22.3 * om_h2) * fb * fb;
    p.theta2 = theta * theta;
    auto transfer = [&](double k) {
        const double ks = 0.43 * k * h * p.s_sound;
        const double ge = om * h * (p.alpha + (1.0 - p.alpha) / (1.0 + ks * ks * ks * ks));
        const double q = k * p.theta2 / ge;
        const double l0 = std::log(2.0 * 2.718281828459045 + 1.8 * q);
        const double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
        return l0 / (l0 + c0 * q * q);
    };
    const double R = 8.0;
    auto integrand = [&](double lnk) {
        const double k = std::exp(lnk), x = k * R;
        const double w = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
        const double tk = transfer(k);
        return k * k * k * std::pow(k, in.n_s) * tk * tk * w * w;
    };
    // start from 64 pieces so the adaptive rule sees the top-hat's oscillations
    double s2 = integrate(integrand, std::log(1e-5), std::log(1e3), 64);
    s2 /= 2.0 * kPi * kPi;
    p.amp = in.sigma8 * in.sigma8 / s2;
    const double box = c.box;
    p.kf = 2.0 * kPi / box;
    p.cell_volume = std::pow(box / c.ptcl_n, 3);
    double ga[4], g0[4];
    growth_rk4(om, in.a, ga);
    growth_rk4(om, 1.0, g0);
    p.D1 = ga[0];
    p.f1 = ga[1];
    p.D2 = ga[2];
    p.f2 = ga[3];
    p.D1_today = g0[0];
    p.g1 = ga[0] / g0[0];
    p.g2 = ga[2] / (g0[0] * g0[0]);
    const double mom = in.a * in.a * std::sqrt(om / (in.a * in.a * in.a) + 1.0 - om);
    p.m1 = mom * ga[1] * p.g1;
    p.m2 = mom * ga[3] * p.g2;
    return HRT_OK;
}

int validate_config(const hrt_config &c, std::string &err) {
    auto bad = [&](const char *m) { err = m; return HRT_EINVAL; };
    if (c.mesh_n < 16 || c.mesh_n > 1024 || (c.mesh_n & (c.mesh_n - 1)))
        return bad("mesh_n must be a power of two in [16, 1024]");
    if (c.ptcl_n < 1 || c.mesh_n % c.ptcl_n) return bad("ptcl_n must be >= 1 and divide mesh_n");
    if (!((c.ray_nx == 0 && c.ray_ny == 0) || (c.ray_nx >= 3 && c.ray_ny >= 3)))
        return bad("ray_nx and ray_ny must both be 0 or both >= 3");
    if ((int64_t)c.ray_nx * c.ray_ny > (int64_t)1 << 26) return bad("too many rays");
    if (c.n_steps < 1 || c.n_steps > 100000) return bad("n_steps out of range");
    if (c.dtype != HRT_F32 && c.dtype != HRT_F64) return bad("dtype must be HRT_F32 or HRT_F64");
    if (c.flags & ~(HRT_STATIC | HRT_ADJOINT | HRT_JACOBIAN | HRT_TIME_DELAY | HRT_RAY_MESH | HRT_FORCE_SLOTS_MASK))
        return bad("unknown flag");
    if ((c.flags & HRT_FORCE_SLOTS_MASK) && !(c.flags & HRT_ADJOINT))
        return bad("HRT_FORCE_SLOTS needs HRT_ADJOINT");
    if (c.flags & HRT_RAY_MESH) {
        if (c.ray_nx == 0) return bad("HRT_RAY_MESH needs rays");
        if (!(c.ray_mesh_iota > 0 && c.ray_mesh_iota <= 1)) return bad("ray_mesh_iota must be in (0, 1]");
        if (!(c.ray_mesh_pmin >= 0) || !std::isfinite(c.ray_mesh_pmin)) return bad("ray_mesh_pmin must be >= 0");
        if ((c.flags & (HRT_ADJOINT | HRT_TIME_DELAY)) || c.los_field != HRT_LOS_NONE) {
            err = "HRT_RAY_MESH with HRT_ADJOINT, HRT_TIME_DELAY or a line-of-sight integral is not supported";
            return HRT_EUNSUPPORTED;
        }
    }
    if ((c.flags & HRT_TIME_DELAY) && c.ray_nx == 0) return bad("HRT_TIME_DELAY needs rays");
    if (c.los_field < HRT_LOS_NONE || c.los_field > HRT_LOS_POTENTIAL) return bad("unknown los_field");
    if (c.los_field != HRT_LOS_NONE) {
        if (c.ray_nx == 0) return bad("a line-of-sight integral needs rays");
        if (c.los_n < 2 || !c.los_chi || !c.los_p) return bad("los_n >= 2 knots with los_chi and los_p needed");
        for (int i = 0; i < c.los_n; ++i) {
            if (!std::isfinite(c.los_chi[i]) || !std::isfinite(c.los_p[i])) return bad("los knots must be finite");
            if (i > 0 && !(c.los_chi[i] > c.los_chi[i - 1])) return bad("los_chi must increase");
        }
    }
    if ((c.flags & HRT_ADJOINT) && ((c.flags & HRT_TIME_DELAY) || c.los_field != HRT_LOS_NONE)) {
        err = "time delay and line-of-sight integrals with HRT_ADJOINT are not supported";
        return HRT_EUNSUPPORTED;
    }
    if ((c.flags & HRT_JACOBIAN) && c.ray_nx == 0) return bad("HRT_JACOBIAN needs rays");
    if ((c.flags & HRT_JACOBIAN) && (c.flags & HRT_ADJOINT)) {
        err = "HRT_JACOBIAN with HRT_ADJOINT is not supported";
        return HRT_EUNSUPPORTED;
    }
    if (c.n_replicas < 0 || c.n_replicas > HRT_MAX_REPLICAS) return bad("n_replicas out of range");
    if ((c.n_replicas > 0) != (c.replicas != nullptr)) return bad("replicas and n_replicas disagree");
    for (int k = 0; k < c.n_replicas; ++k) {
        const int32_t *row = c.replicas + 9 * k;
        int seen = 0;
        for (int a = 0; a < 3; ++a) {
            if (row[a] < 0 || row[a] > 2) return bad("replica perm entries must be 0, 1 or 2");
            seen |= 1 << row[a];
            if (row[3 + a] != 1 && row[3 + a] != -1) return bad("replica signs must be +1 or -1");
            if (row[6 + a] < 0 || row[6 + a] >= c.mesh_n) return bad("replica shifts must be in [0, mesh_n)");
        }
        if (seen != 7) return bad("replica perm must be a permutation of 0, 1, 2");
        const bool ident = row[0] == 0 && row[1] == 1 && row[2] == 2 && row[3] == 1 && row[4] == 1 &&
                           row[5] == 1 && row[6] == 0 && row[7] == 0 && row[8] == 0;
        if (!ident && (c.flags & HRT_ADJOINT)) {
            err = "replica transforms with HRT_ADJOINT are not supported";
            return HRT_EUNSUPPORTED;
        }
    }
    if (c.n_src < 0 || c.n_src > HRT_MAX_SOURCES) return bad("n_src out of range [0, HRT_MAX_SOURCES]");
    if (c.n_src > 0 && !c.src) return bad("src is NULL with n_src > 0");
    if (c.n_src > 0 && c.ray_nx == 0) return bad("source planes need rays");
    for (int i = 0; i < c.n_src; ++i) {
        if (!std::isfinite(c.src[i]) || !(c.src[i] > 0)) return bad("source planes must be positive and finite");
        if (c.src_w && !std::isfinite(c.src_w[i])) return bad("source weights must be finite");
    }
    if (!(c.box > 0) || !std::isfinite(c.box)) return bad("box must be positive");
    if (c.ray_nx > 0 && (!(c.fov_x > 0) || !(c.fov_y > 0) || c.fov_x > 1.0 || c.fov_y > 1.0))
        return bad("fov must be in (0, 1] rad");
    if (!c.sched) return bad("sched is NULL");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(c.observer[i])) return bad("observer must be finite");
    if (c.flags & HRT_STATIC) {
        if (!(c.static_mass > 0)) return bad("static_mass must be positive");
        for (int i = 0; i <= c.n_steps; ++i)
            if (!(c.sched[i] >= 0) || !std::isfinite(c.sched[i])) return bad("chi schedule must be >= 0");
    } else {
        if (!(c.omega_m > 0 && c.omega_m <= 1)) return bad("omega_m must be in (0, 1]");
        for (int i = 0; i <= c.n_steps; ++i)
            if (!(c.sched[i] > 0 && c.sched[i] <= 1)) return bad("a schedule must be in (0, 1]");
    }
    return HRT_OK;
}

// P(chi) of the line-of-sight integral: linear between the knots, 0 outside them.
static double los_profile(const hrt_config &c, double chi) {
    if (chi < c.los_chi[0] || chi > c.los_chi[c.los_n - 1]) return 0.0;
    for (int i = 1; i < c.los_n; ++i)
        if (chi <= c.los_chi[i]) {
            const double t = (chi - c.los_chi[i - 1]) / (c.los_chi[i] - c.los_chi[i - 1]);
            return c.los_p[i - 1] + t * (c.los_p[i] - c.los_p[i - 1]);
        }
    return 0.0;
}

// Fused leapfrog tables (step n runs boundary n -> n+1; step N is the closing
// half-kick). Half points are arithmetic means clipped at both ends.
int build_tables(const hrt_config &c, StepTables &t, std::string &err) {
    int rc = validate_config(c, err);
    if (rc) return rc;
    const int N = c.n_steps;
    const double cell = c.box / c.mesh_n;
    const double z_obs = c.observer[2];
    const bool stat = (c.flags & HRT_STATIC) != 0;
    t = StepTables();
    t.a.assign(N + 1, 1.0);
    t.chi.assign(N + 1, 0.0);
    t.K.assign(N + 1, 0.0);
    t.D.assign(N + 1, 0.0);
    t.d.assign(N + 1, 0.0);
    t.plane_begin.assign(N + 1, 0);
    t.plane_count.assign(N + 1, 0);
    Cosmo cos{c.omega_m, 1.0 - c.omega_m};
    std::vector<double> D1n;
    if (stat) {
        for (int i = 0; i <= N; ++i) t.chi[i] = c.sched[i];
    } else {
        for (int i = 0; i <= N; ++i) {
            t.a[i] = c.sched[i];
            t.chi[i] = cos.chi(t.a[i]);
        }
        for (int n = 0; n <= N; ++n) {
            double alo = n == 0 ? t.a[0] : 0.5 * (t.a[n - 1] + t.a[n]);
            double ahi = n == N ? t.a[N] : 0.5 * (t.a[n] + t.a[n + 1]);
            t.K[n] = -1.5 * c.omega_m * cos.kick(alo, ahi);
            t.D[n] = n < N ? cos.drift(t.a[n], t.a[n + 1]) : 0.0;
        }
        if (c.ray_nx > 0) {
            D1n.resize(N + 1);
            for (int n = 0; n <= N; ++n) D1n[n] = cos.D1(t.a[n]);
        }
    }
    if (c.ray_nx == 0) return HRT_OK;
    // ray mesh (Sec. 5.2-5.3, App. C): per step lam = max(2 cell / (r_a + r_b), mu_2D) over
    // the kick's shell [chi_{n-1/2}, chi_{n+1/2}], spacing iota lam, and one mesh size for the
    // run: the smallest power of two with N mu >= field + p_min lam at every step
    if (c.flags & HRT_RAY_MESH) {
        const double mu2d = std::max(c.fov_x / c.ray_nx, c.fov_y / c.ray_ny);
        const double field = std::max(c.fov_x, c.fov_y);
        t.rm_lam.assign(N + 1, 0.0);
        t.rm_mu.assign(N + 1, 0.0);
        int64_t size = 16;
        for (int n = 0; n <= N; ++n) {
            const double lo = std::fabs(n == 0 ? t.chi[0] : 0.5 * (t.chi[n - 1] + t.chi[n]));
            const double hi = std::fabs(n == N ? t.chi[N] : 0.5 * (t.chi[n] + t.chi[n + 1]));
            const double lam = lo + hi > 0 ? std::max(2.0 * cell / (lo + hi), mu2d) : mu2d;
            t.rm_lam[n] = lam;
            t.rm_mu[n] = c.ray_mesh_iota * lam;
            const double need = field / t.rm_mu[n] + c.ray_mesh_pmin / c.ray_mesh_iota;
            if (!(need <= 2048.0)) {
                err = "the ray mesh would need more than 2048 points per side";
                return HRT_EUNSUPPORTED;
            }
            while ((double)size < need) size *= 2;
        }
        t.rm_n = (int32_t)size;
    }
    // source planes: each must sit on a step boundary 1..N of the schedule (Alg. 1 observes
    // the rays at the end of a step)
    t.src_step.assign(c.n_src, -1);
    t.src_w.assign(c.n_src, 0.0);
    t.has_src_w = c.src_w != nullptr;
    for (int i = 0; i < c.n_src; ++i) {
        const double v = stat ? c.src[i] : 1.0 / (1.0 + c.src[i]);
        for (int k = 1; k <= N; ++k) {
            const double b = stat ? t.chi[k] : t.a[k];
            if (std::fabs(b - v) <= 1e-9 * std::max(std::fabs(b), stat ? 1.0 : 0.0)) {
                t.src_step[i] = k;
                break;
            }
        }
        if (t.src_step[i] < 0) {
            err = std::string("source plane ") + std::to_string(c.src[i]) +
                  (stat ? " (chi)" : " (z)") + " is not a step boundary of the schedule";
            return HRT_EINVAL;
        }
        for (int j = 0; j < i; ++j)
            if (t.src_step[j] == t.src_step[i]) {
                err = "two source planes on the same step boundary";
                return HRT_EINVAL;
            }
        if (c.src_w) t.src_w[i] = c.src_w[i];
    }
    const double rho_bar = std::pow((double)c.ptcl_n, 3) / std::pow((double)c.mesh_n, 3);
    const double static_pref = -8.0 * kPi * kGoverC2 * c.static_mass * rho_bar / (cell * cell);
    std::vector<int64_t> js;
    for (int n = 0; n <= N; ++n) {
        double rmid = n < N ? 0.5 * (t.chi[n] + t.chi[n + 1]) : 0.0;
        t.d[n] = n < N ? (t.chi[n + 1] - t.chi[n]) / (rmid * rmid) : 0.0;
        double lo = n == 0 ? t.chi[0] : 0.5 * (t.chi[n - 1] + t.chi[n]);
        double hi = n == N ? t.chi[N] : 0.5 * (t.chi[n] + t.chi[n + 1]);
        double sgn = hi >= lo ? 1.0 : -1.0;
        shell_planes(lo, hi, cell, z_obs, js);
        t.plane_begin[n] = (int32_t)t.plane_chi.size();
        for (int64_t j : js) {
            double cj = (double)j * cell - z_obs;
            if (!(cj > 0.0)) continue;            // r = 0 carries no weight
            double w, growth = 1.0;               // growth: D1(a_j) / D1(a_n)
            if (stat) {
                w = sgn * static_pref * cj;
            } else {
                double aj = cos.a_of_chi(cj);
                growth = cos.D1(aj) / D1n[n];
                w = sgn * (-3.0 * c.omega_m * cell * cj * cos.D1(aj)) / (kCH0 * kCH0 * D1n[n] * aj);
            }
            int64_t m = j % c.mesh_n;
            if (m < 0) m += c.mesh_n;
            int64_t rep = 0;                      // table row of replica floor(j / n)
            if (c.n_replicas > 0) {
                const int64_t k = (j - m) / c.mesh_n;
                rep = k % c.n_replicas;
                if (rep < 0) rep += c.n_replicas;
            }
            // line-of-sight weight: P(chi_j) cell times the field's growth correction to
            // the plane's time (density D1(a_j)/D1(a_n); potential -w_j / (2 chi_j cell), the
            // kick's Phi/c^2 per unit phi)
            double lw = 0.0;
            if (c.los_field != HRT_LOS_NONE) {
                const double P = los_profile(c, cj);
                if (c.los_field == HRT_LOS_POTENTIAL) lw = -P * w / (2.0 * cj);
                else lw = sgn * P * cell * growth;
            }
            t.plane_mesh.push_back((int32_t)m);
            t.plane_rep.push_back((int32_t)rep);
            t.plane_los.push_back(lw);
            t.plane_chi.push_back(cj);
            t.plane_w.push_back(w);
        }
        t.plane_count[n] = (int32_t)t.plane_chi.size() - t.plane_begin[n];
        t.max_count = std::max(t.max_count, t.plane_count[n]);
        if (t.plane_chi.size() > (size_t)1 << 28) {
            err = "too many shell planes";
            return HRT_EINVAL;
        }
    }
    return HRT_OK;
}

}  // namespace hrt
