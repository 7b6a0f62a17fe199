// C ABI of the HRT library: configuration, workspace layout, step sequencing and
// launches. Declarations and argument contracts are in include/hrt.h.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "hrt_internal.h"

namespace hrt {
namespace {

thread_local std::string g_init_error;

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

Layout make_layout(const hrt_config &cfg, int64_t n_plane_entries) {
    Layout L{};
    const size_t T = cfg.dtype == HRT_F64 ? 8 : 4;
    const size_t n = (size_t)cfg.mesh_n;
    const size_t n3 = n * n * n;
    const size_t P = (size_t)cfg.ptcl_n * cfg.ptcl_n * cfg.ptcl_n;
    L.nbins = (int64_t)(n3 / 64);          // (n/8)^3 tiles x 8 face masks
    const int64_t nblk = (L.nbins + 1023) / 1024;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t at = off; off = align_up(off + bytes); return at; };
    L.mesh_r = take(2 * n3 * T);                        // delta, then phi
    L.spec = take((n / 2 + 1) * n * n * 2 * T);
    const size_t np = (size_t)cfg.ptcl_n;
    L.spec2 = take((np / 2 + 1) * np * np * 2 * T);      // second spectrum for the initial conditions
    L.grad = take(n3 * 4 * T);                          // (G_x, G_y, G_z, 0) per node
    L.twiddle = take(n * 2 * T);
    L.bins = take((size_t)(L.nbins + L.nbins + 1 + nblk + 1) * 4);
    L.cursor = take((size_t)L.nbins * 4);
    L.sorted = take(P * 4 * T);
    L.planes = take((size_t)std::max<int64_t>(n_plane_entries, 1) * sizeof(PlaneEntry));
    L.total = off;
    return L;
}

}  // namespace hrt

using hrt::g_init_error;

namespace hrt {

static hipEvent_t pool_event(hrt_ctx *c) {
    if (!c->prof_pool.empty()) {
        hipEvent_t e = c->prof_pool.back();
        c->prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void prof_drain(hrt_ctx *c) {
    if (c->prof_pending.empty()) return;
    hipStreamSynchronize(c->stream);
    for (const ProfRecord &r : c->prof_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            c->prof_ms[r.id] += ms;
            c->prof_n[r.id] += 1;
        }
        c->prof_pool.push_back(r.start);
        c->prof_pool.push_back(r.stop);
    }
    c->prof_pending.clear();
}

void prof_begin(hrt_ctx *c) {
    if (!c->prof) return;
    c->prof_open = pool_event(c);
    if (c->prof_open) hipEventRecord(c->prof_open, c->stream);
}

void prof_end(hrt_ctx *c, int id) {
    if (!c->prof || !c->prof_open) return;
    hipEvent_t stop = pool_event(c);
    if (!stop) return;
    hipEventRecord(stop, c->stream);
    c->prof_pending.push_back(ProfRecord{id, c->prof_open, stop});
    c->prof_open = nullptr;
    if (c->prof_pending.size() > 20000) prof_drain(c);
}

}  // namespace hrt

hrt_ctx::~hrt_ctx() {
    for (const hrt::ProfRecord &r : prof_pending) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : prof_pool) hipEventDestroy(e);
}

static const char *kKernelNames[hrt::K_COUNT] = {
    "bin_count", "bin_scan", "bin_scatter", "paint_tiles", "fft_x_r2c", "fft_y_fwd",
    "fft_z_poisson", "fft_y_inv", "fft_x_c2r", "fd4_gradient", "matter_kd", "ray_step",
    "convergence"};

extern "C" const char *hrt_kernel_name(int id) {
    return (id >= 0 && id < hrt::K_COUNT) ? kKernelNames[id] : nullptr;
}

extern "C" int hrt_profile_enable(hrt_ctx *c, int on) {
    if (!c) return HRT_EINVAL;
    hrt::prof_drain(c);
    if (on) {
        for (int k = 0; k < hrt::K_COUNT; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
        }
    }
    c->prof = on != 0;
    return HRT_OK;
}

extern "C" int hrt_profile_read(hrt_ctx *c, double *total_ms, int64_t *launches, int n) {
    if (!c || n < 0) return HRT_EINVAL;
    hrt::prof_drain(c);
    for (int k = 0; k < n && k < hrt::K_COUNT; ++k) {
        if (total_ms) total_ms[k] = c->prof_ms[k];
        if (launches) launches[k] = c->prof_n[k];
    }
    return HRT_OK;
}

static int fail(hrt_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    else g_init_error = msg;
    return code;
}

static int check_hip(hrt_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return HRT_OK;
    return fail(c, HRT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

extern "C" int hrt_workspace_bytes(const hrt_config *cfg, size_t *bytes) {
    if (!cfg || !bytes) return fail(nullptr, HRT_EINVAL, "NULL argument");
    hrt::StepTables t;
    std::string err;
    int rc = hrt::build_tables(*cfg, t, err);
    if (rc) return fail(nullptr, rc, err);
    *bytes = hrt::make_layout(*cfg, (int64_t)t.plane_chi.size()).total;
    return HRT_OK;
}

extern "C" int hrt_tables(const hrt_config *cfg, double *a, double *chi, double *K, double *D,
                          double *d, int32_t *plane_begin, int32_t *plane_count,
                          int32_t *plane_mesh, double *plane_chi, double *plane_w,
                          int32_t max_planes, int32_t *n_planes) {
    if (!cfg) return fail(nullptr, HRT_EINVAL, "NULL config");
    hrt::StepTables t;
    std::string err;
    int rc = hrt::build_tables(*cfg, t, err);
    if (rc) return fail(nullptr, rc, err);
    const int N1 = cfg->n_steps + 1;
    auto put = [&](double *dst, const std::vector<double> &src) {
        if (dst) std::memcpy(dst, src.data(), src.size() * sizeof(double));
    };
    put(a, t.a);
    put(chi, t.chi);
    put(K, t.K);
    put(D, t.D);
    put(d, t.d);
    if (plane_begin) std::memcpy(plane_begin, t.plane_begin.data(), N1 * sizeof(int32_t));
    if (plane_count) std::memcpy(plane_count, t.plane_count.data(), N1 * sizeof(int32_t));
    const int64_t np = (int64_t)t.plane_chi.size();
    if (n_planes) *n_planes = (int32_t)np;
    if (np > max_planes) return fail(nullptr, HRT_ENOMEM, "max_planes too small");
    if (plane_mesh) std::memcpy(plane_mesh, t.plane_mesh.data(), np * sizeof(int32_t));
    put(plane_chi, t.plane_chi);
    put(plane_w, t.plane_w);
    return HRT_OK;
}

extern "C" int hrt_init(const hrt_config *cfg, void *workspace, size_t ws_bytes, void *stream,
                        hrt_ctx **out) {
    if (!cfg || !out) return fail(nullptr, HRT_EINVAL, "NULL argument");
    *out = nullptr;
    hrt_ctx *c = new (std::nothrow) hrt_ctx();
    if (!c) return fail(nullptr, HRT_ENOMEM, "host allocation failed");
    std::string err;
    int rc = hrt::build_tables(*cfg, c->tab, err);
    if (rc) {
        delete c;
        return fail(nullptr, rc, err);
    }
    c->cfg = *cfg;
    c->sched.assign(cfg->sched, cfg->sched + cfg->n_steps + 1);
    c->cfg.sched = c->sched.data();
    c->n = cfg->mesh_n;
    c->np = cfg->ptcl_n;
    c->mx = cfg->ray_nx;
    c->my = cfg->ray_ny;
    c->N = cfg->n_steps;
    c->f64 = cfg->dtype == HRT_F64;
    c->is_static = (cfg->flags & HRT_STATIC) != 0;
    c->box = cfg->box;
    c->cell = cfg->box / cfg->mesh_n;
    c->stream = static_cast<hipStream_t>(stream);
    c->lay = hrt::make_layout(*cfg, (int64_t)c->tab.plane_chi.size());
    if (!workspace || ws_bytes < c->lay.total) {
        delete c;
        return fail(nullptr, HRT_ENOMEM, "workspace missing or smaller than hrt_workspace_bytes()");
    }
    if (reinterpret_cast<uintptr_t>(workspace) % 256) {
        delete c;
        return fail(nullptr, HRT_EINVAL, "workspace must be 256-byte aligned");
    }
    c->ws = static_cast<char *>(workspace);
    const double P = std::pow((double)c->np, 3);
    // Fixed-point fraction bits for the paint: the largest node sum (all particles on
    // one node) must stay below 2^62.
    c->fixed_bits = std::min(52, 62 - (int)std::ceil(std::log2(std::max(P, 1.0))));

    // twiddles W_n^m = exp(-2 pi i m / n) and plane entries
    const int n = c->n;
    std::vector<double> twd(2 * n);
    for (int m = 0; m < n; ++m) {
        const double ang = -2.0 * 3.14159265358979323846 * m / n;
        twd[2 * m] = std::cos(ang);
        twd[2 * m + 1] = std::sin(ang);
    }
    std::vector<char> twbuf(2 * n * (c->f64 ? 8 : 4));
    if (c->f64) {
        std::memcpy(twbuf.data(), twd.data(), twbuf.size());
    } else {
        float *f = reinterpret_cast<float *>(twbuf.data());
        for (int k = 0; k < 2 * n; ++k) f[k] = (float)twd[k];
    }
    std::vector<hrt::PlaneEntry> pe(c->tab.plane_chi.size());
    for (size_t k = 0; k < pe.size(); ++k)
        pe[k] = hrt::PlaneEntry{c->tab.plane_chi[k], c->tab.plane_w[k], c->tab.plane_mesh[k], 0};
    hipError_t e = hipMemcpyAsync(c->ws + c->lay.twiddle, twbuf.data(), twbuf.size(),
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !pe.empty())
        e = hipMemcpyAsync(c->ws + c->lay.planes, pe.data(), pe.size() * sizeof(hrt::PlaneEntry),
                           hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("table upload failed: ") + hipGetErrorString(e);
        delete c;
        return fail(nullptr, HRT_EDEVICE, msg);
    }
    *out = c;
    return HRT_OK;
}

extern "C" int hrt_destroy(hrt_ctx *ctx) {
    delete ctx;
    return HRT_OK;
}

extern "C" const char *hrt_last_error(const hrt_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

static int check_matter(hrt_ctx *c, const hrt_matter *m, bool need_p) {
    if (!m) return fail(c, HRT_EINVAL, "NULL matter state");
    for (int d = 0; d < 3; ++d) {
        if (!m->s[d]) return fail(c, HRT_EINVAL, "NULL displacement array");
        if (need_p && !m->p[d]) return fail(c, HRT_EINVAL, "NULL momentum array");
    }
    return HRT_OK;
}

extern "C" int pm_force(hrt_ctx *c, const hrt_matter *m, int step) {
    if (!c) return HRT_EINVAL;
    if (step < 0 || step > c->N) return fail(c, HRT_EINVAL, "step out of range [0, n_steps]");
    if (int rc = check_matter(c, m, false)) return rc;
    if (int rc = check_hip(c, hrt::launch_paint(c, m), "paint")) return rc;
    if (int rc = check_hip(c, hrt::launch_poisson(c), "poisson")) return rc;
    if (int rc = check_hip(c, hrt::launch_gradient(c), "gradient")) return rc;
    c->force_step = step;
    return HRT_OK;
}

extern "C" int pm_step(hrt_ctx *c, const hrt_matter *m, int step) {
    if (!c) return HRT_EINVAL;
    if (c->is_static) return fail(c, HRT_ESTATE, "pm_step is not valid for a static run");
    if (int rc = check_matter(c, m, true)) return rc;
    if (int rc = pm_force(c, m, step)) return rc;
    return check_hip(c, hrt::launch_matter_kd(c, m, c->tab.K[step], c->tab.D[step]), "matter kick-drift");
}

extern "C" int ray_step(hrt_ctx *c, const hrt_rays *r, int step) {
    if (!c) return HRT_EINVAL;
    if (c->mx == 0) return fail(c, HRT_ESTATE, "configuration has no rays");
    if (step < 0 || step > c->N) return fail(c, HRT_EINVAL, "step out of range [0, n_steps]");
    if (!r || !r->dth[0] || !r->dth[1] || !r->p[0] || !r->p[1])
        return fail(c, HRT_EINVAL, "NULL ray array");
    if (c->force_step < 0) return fail(c, HRT_ESTATE, "no force mesh yet: call pm_force or pm_step first");
    if (!c->is_static && c->force_step != step)
        return fail(c, HRT_ESTATE, "ray_step must follow pm_step/pm_force of the same step");
    return check_hip(c, hrt::launch_ray_step(c, r, c->tab.plane_begin[step], c->tab.plane_count[step],
                                             c->tab.d[step]), "ray step");
}

extern "C" int ray_convergence(hrt_ctx *c, const hrt_rays *r, void *kappa, void *gamma1,
                               void *gamma2, void *omega) {
    if (!c) return HRT_EINVAL;
    if (c->mx == 0) return fail(c, HRT_ESTATE, "configuration has no rays");
    if (!r || !r->dth[0] || !r->dth[1] || !kappa) return fail(c, HRT_EINVAL, "NULL argument");
    return check_hip(c, hrt::launch_convergence(c, r, kappa, gamma1, gamma2, omega), "convergence");
}

extern "C" int hrt_ic_factors(const hrt_config *cfg, const hrt_ic_params *ic, double *out) {
    if (!cfg || !ic || !out) return fail(nullptr, HRT_EINVAL, "NULL argument");
    std::string err;
    int rc = hrt::validate_config(*cfg, err);
    if (rc) return fail(nullptr, rc, err);
    hrt::IcParams p;
    rc = hrt::ic_params(*cfg, *ic, p, err);
    if (rc) return fail(nullptr, rc, err);
    out[0] = p.amp;
    out[1] = p.D1;
    out[2] = p.f1;
    out[3] = p.D2;
    out[4] = p.f2;
    out[5] = p.D1_today;
    return HRT_OK;
}

extern "C" int hrt_ic_2lpt(hrt_ctx *c, const void *noise, const hrt_ic_params *ic, const hrt_matter *out) {
    if (!c) return HRT_EINVAL;
    if (!noise || !ic) return fail(c, HRT_EINVAL, "NULL argument");
    if (int rc = check_matter(c, out, true)) return rc;
    if (c->np < 16) return fail(c, HRT_EUNSUPPORTED, "initial conditions need ptcl_n >= 16");
    hrt::IcParams p;
    std::string err;
    if (int rc = hrt::ic_params(c->cfg, *ic, p, err)) return fail(c, rc, err);
    if (int rc = check_hip(c, hrt::launch_ic(c, noise, p, out), "initial conditions")) return rc;
    c->force_step = -1;          // the force mesh was used as scratch
    return HRT_OK;
}

extern "C" int hrt_mesh_ptr(const hrt_ctx *c, int which, void **ptr) {
    if (!c || !ptr) return HRT_EINVAL;
    const size_t T = c->f64 ? 8 : 4;
    const size_t n3 = (size_t)c->n * c->n * c->n;
    switch (which) {
        case HRT_MESH_DELTA: *ptr = c->ws + c->lay.mesh_r; return HRT_OK;
        case HRT_MESH_PHI: *ptr = c->ws + c->lay.mesh_r + n3 * T; return HRT_OK;
        case HRT_MESH_GRAD: *ptr = c->ws + c->lay.grad; return HRT_OK;
        default: return HRT_EINVAL;
    }
}
