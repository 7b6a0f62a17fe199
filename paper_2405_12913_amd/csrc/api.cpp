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

Layout make_layout(const hrt_config &cfg, int64_t n_plane_entries, int64_t max_count, int64_t rm_n) {
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
    // mover-list run (FP32 with moving particles): the records lie as [rec0 | S | rec1 | U]
    // in `sorted` (P, P, P, 2P entries) and the momenta as [mom0 | S | mom1 | U] in `state`
    // (3P, 3P, 3P, 6P values), all within 32-bit offsets of rec0 and mom0
    const bool list = !(cfg.flags & HRT_STATIC) && T == 4 && 15 * P < ((size_t)1 << 31);
    L.sorted = take(P * 4 * T * (list ? 5 : 1));
    // sorted-state run: the second record buffer (the first is `sorted`) and both momentum
    // buffers, P x (4 + 3 + 3) values; with the list, the momenta only (15P values); a static
    // run moves no particles
    L.state = (cfg.flags & HRT_STATIC) ? 0 : take(P * (list ? 15 : 10) * T);
    L.planes = take((size_t)std::max<int64_t>(n_plane_entries, 1) * sizeof(PlaneEntry));
    // reverse mode: 2 x n^3 64-bit fixed-point accumulators (rays' part of the force-mesh
    // cotangent), one 8-byte device scalar (256 bytes reserved), P x 4 kick weights and the
    // ray VJP's per-group partial sums (kRayVjpParts x rays x 2 doubles)
    const size_t M = (size_t)cfg.ray_nx * cfg.ray_ny;
    L.adj = (cfg.flags & HRT_ADJOINT) ? take(2 * n3 * 8 + 256 + P * 4 * T + kRayVjpParts * M * 16) : off;
    // lens-plane stack of one shell: (G_u, G_v) per node of each plane, replica frame
    L.stack = cfg.ray_nx > 0 ? take((size_t)std::max<int64_t>(max_count, 1) * n * n * 2 * T) : off;
    // scalar lens planes: phi (time delay, potential integrals), delta (density integrals)
    const bool want_phi = (cfg.flags & HRT_TIME_DELAY) || cfg.los_field == HRT_LOS_POTENTIAL;
    const bool want_delta = cfg.los_field == HRT_LOS_DENSITY;
    L.stack_phi = want_phi ? take((size_t)std::max<int64_t>(max_count, 1) * n * n * T) : off;
    L.stack_delta = want_delta ? take((size_t)std::max<int64_t>(max_count, 1) * n * n * T) : off;
    L.reps = take((size_t)std::max(cfg.n_replicas, 1) * 9 * 4);      // replica transform rows
    // ray mesh: the complex kick field (N^2) and its twiddles W_N^m (N)
    L.rm_mesh = rm_n > 0 ? take((size_t)rm_n * rm_n * 2 * T) : off;
    L.rm_tw = rm_n > 0 ? take((size_t)rm_n * 2 * T) : off;
    // mover-list run: control words, the mover histogram and list offsets, holes per bin and
    // the extents of the kick-drift workgroups' parts of U
    L.list = list ? take(list_offsets((size_t)L.nbins).total) : 0;
    // force slots (HRT_FORCE_SLOTS): per slot a copy of G and of the paint-bin offsets
    const int slots = (cfg.flags & HRT_FORCE_SLOTS_MASK) >> 8;
    L.fslot_g = align_up(n3 * 4 * T);
    L.fslot_bytes = L.fslot_g + align_up((size_t)(L.nbins + 1) * 4);
    L.fslots = slots ? take(slots * L.fslot_bytes) : off;
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
    if (graph) hipGraphExecDestroy(graph);
    for (const hrt::ProfRecord &r : prof_pending) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    for (hipEvent_t e : prof_pool) hipEventDestroy(e);
}

static const char *kKernelNames[hrt::K_COUNT] = {
    "bin_count", "bin_scan", "bin_scatter", "paint_tiles", "fft_x_r2c", "fft_y_fwd",
    "fft_z_poisson", "fft_y_inv", "fft_x_c2r", "fd4_gradient", "matter_kd", "ray_step",
    "convergence", "state_scatter", "kd_tiles", "plane_gradient", "state_gather", "ray_mesh",
    "list_settle"};

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

// Realisation r's part of a batched workspace starts at the sum of the previous parts.
static int batch_layouts(const hrt_config *cfg, int n_cfg, std::vector<hrt::StepTables> *tabs,
                         std::vector<hrt::Layout> &lays, std::string &err) {
    if (!cfg || n_cfg < 1) { err = "need at least one configuration"; return HRT_EINVAL; }
    lays.clear();
    if (tabs) tabs->assign(n_cfg, hrt::StepTables());
    for (int r = 0; r < n_cfg; ++r) {
        const hrt_config &c0 = cfg[0], &c = cfg[r];
        if (c.dtype != c0.dtype || c.n_steps != c0.n_steps || c.flags != c0.flags ||
            (c.ray_nx > 0) != (c0.ray_nx > 0) || c.n_src != c0.n_src ||
            (c.src_w == nullptr) != (c0.src_w == nullptr) || c.los_field != c0.los_field) {
            err = "batched configurations must share dtype, n_steps, flags, whether they have rays, "
                  "n_src, whether they have source weights and los_field";
            return HRT_EINVAL;
        }
        hrt::StepTables t;
        int rc = hrt::build_tables(c, t, err);
        if (rc) return rc;
        lays.push_back(hrt::make_layout(c, (int64_t)t.plane_chi.size(), t.max_count, t.rm_n));
        if (tabs) (*tabs)[r] = std::move(t);
    }
    return HRT_OK;
}

extern "C" int hrt_workspace_bytes(const hrt_config *cfg, int n_cfg, size_t *bytes) {
    if (!cfg || !bytes) return fail(nullptr, HRT_EINVAL, "NULL argument");
    std::vector<hrt::Layout> lays;
    std::string err;
    int rc = batch_layouts(cfg, n_cfg, nullptr, lays, err);
    if (rc) return fail(nullptr, rc, err);
    size_t total = 0;
    for (const hrt::Layout &L : lays) total += L.total;
    *bytes = total;
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

int hrt::init_context(const hrt_config *cfg, int n_cfg, void *workspace, size_t ws_bytes,
                      void *stream, hrt_ctx **out) {
    if (!cfg || !out) return fail(nullptr, HRT_EINVAL, "NULL argument");
    *out = nullptr;
    std::vector<hrt::StepTables> tabs;
    std::vector<hrt::Layout> lays;
    std::string err;
    int rc = batch_layouts(cfg, n_cfg, &tabs, lays, err);
    if (rc) return fail(nullptr, rc, err);
    size_t total = 0;
    for (const hrt::Layout &L : lays) total += L.total;
    if (!workspace || ws_bytes < total)
        return fail(nullptr, HRT_ENOMEM,
                    "workspace missing or smaller than hrt_workspace_bytes() (" + std::to_string(total) +
                        " bytes needed, " + std::to_string(ws_bytes) + " given)");
    if (reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(nullptr, HRT_EINVAL, "workspace must be 256-byte aligned");
    hrt_ctx *c = new (std::nothrow) hrt_ctx();
    if (!c) return fail(nullptr, HRT_ENOMEM, "host allocation failed");
    c->stream = static_cast<hipStream_t>(stream);
    c->N = cfg[0].n_steps;
    c->f64 = cfg[0].dtype == HRT_F64;
    c->is_static = (cfg[0].flags & HRT_STATIC) != 0;
    c->has_rays = cfg[0].ray_nx > 0;
    c->jacobian = (cfg[0].flags & HRT_JACOBIAN) != 0;
    c->delay = (cfg[0].flags & HRT_TIME_DELAY) != 0;
    c->ray_mesh = (cfg[0].flags & HRT_RAY_MESH) != 0;
    c->los = cfg[0].los_field;
    c->n_src = cfg[0].n_src;
    c->n_maps = cfg[0].n_src + (cfg[0].src_w ? 1 : 0);
    c->slot_step.assign((cfg[0].flags & HRT_FORCE_SLOTS_MASK) >> 8, -1);
    c->re.resize(n_cfg);
    char *ws = static_cast<char *>(workspace);
    hipError_t e = hipSuccess;
    for (int r = 0; r < n_cfg && e == hipSuccess; ++r) {
        hrt::Real &re = c->re[r];
        re.cfg = cfg[r];
        re.sched.assign(cfg[r].sched, cfg[r].sched + cfg[r].n_steps + 1);
        re.cfg.sched = re.sched.data();
        re.cfg.src = nullptr;            // copied into the tables (src_step, src_w)
        re.cfg.src_w = nullptr;
        re.cfg.replicas = nullptr;       // copied into the workspace
        re.cfg.los_chi = nullptr;        // folded into the plane weights
        re.cfg.los_p = nullptr;
        re.n = cfg[r].mesh_n;
        re.np = cfg[r].ptcl_n;
        re.mx = cfg[r].ray_nx;
        re.my = cfg[r].ray_ny;
        re.box = cfg[r].box;
        re.cell = cfg[r].box / cfg[r].mesh_n;
        re.tab = std::move(tabs[r]);
        re.lay = lays[r];
        re.ws = ws;
        ws += lays[r].total;
        // Fixed-point fraction bits for the paint: the largest node sum (all particles
        // on one node) must stay below 2^62.
        const double P = std::pow((double)re.np, 3);
        re.fixed_bits = std::min(52, 62 - (int)std::ceil(std::log2(std::max(P, 1.0))));
        // twiddles W_n^m = exp(-2 pi i m / n) and plane entries
        const int n = re.n;
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
        std::vector<hrt::PlaneEntry> pe(re.tab.plane_chi.size());
        for (size_t k = 0; k < pe.size(); ++k)
            pe[k] = hrt::PlaneEntry{re.tab.plane_chi[k], re.tab.plane_w[k], re.tab.plane_mesh[k],
                                    re.tab.plane_rep[k], re.tab.plane_los[k]};
        // replica rows (the identity when the configuration has none)
        static const int32_t kIdentity[9] = {0, 1, 2, 1, 1, 1, 0, 0, 0};
        std::vector<int32_t> reps(kIdentity, kIdentity + 9);
        if (cfg[r].n_replicas > 0) reps.assign(cfg[r].replicas, cfg[r].replicas + 9 * cfg[r].n_replicas);
        re.identity_reps = true;
        for (size_t k = 0; k < reps.size(); ++k)
            if (reps[k] != kIdentity[k % 9]) re.identity_reps = false;
        e = hipMemcpyAsync(re.ws + re.lay.twiddle, twbuf.data(), twbuf.size(), hipMemcpyHostToDevice,
                           c->stream);
        if (e == hipSuccess && !pe.empty())
            e = hipMemcpyAsync(re.ws + re.lay.planes, pe.data(), pe.size() * sizeof(hrt::PlaneEntry),
                               hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(re.ws + re.lay.reps, reps.data(), reps.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, c->stream);
        // ray-mesh twiddles W_N^m = exp(-2 pi i m / N)
        std::vector<char> rmtw;
        if (re.tab.rm_n > 0) {
            const int N = re.tab.rm_n;
            rmtw.resize((size_t)2 * N * (c->f64 ? 8 : 4));
            for (int m = 0; m < N; ++m) {
                const double ang = -2.0 * 3.14159265358979323846 * m / N;
                if (c->f64) {
                    reinterpret_cast<double *>(rmtw.data())[2 * m] = std::cos(ang);
                    reinterpret_cast<double *>(rmtw.data())[2 * m + 1] = std::sin(ang);
                } else {
                    reinterpret_cast<float *>(rmtw.data())[2 * m] = (float)std::cos(ang);
                    reinterpret_cast<float *>(rmtw.data())[2 * m + 1] = (float)std::sin(ang);
                }
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(re.ws + re.lay.rm_tw, rmtw.data(), rmtw.size(), hipMemcpyHostToDevice,
                                   c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    }
    if (e != hipSuccess) {
        std::string msg = std::string("table upload failed: ") + hipGetErrorString(e);
        delete c;
        return fail(nullptr, HRT_EDEVICE, msg);
    }
    *out = c;
    return HRT_OK;
}

extern "C" int hrt_init(const hrt_config *cfg, int n_cfg, void *workspace, size_t ws_bytes,
                        void *stream, hrt_ctx **out) {
    return hrt::init_context(cfg, n_cfg, workspace, ws_bytes, stream, out);
}

int hrt::set_init_error(int code, const std::string &msg) { return fail(nullptr, code, msg); }

// A context whose workspace is the static no-allocation array stays valid only until the
// next hrt_init_noalloc on the same device re-lays that array out for another context.
static int guard(hrt_ctx *c) {
    if (hrt::noalloc_superseded(c))
        return fail(c, HRT_ESTATE, "context superseded: a later hrt_init_noalloc on this device "
                                   "re-used the static workspace");
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
    for (size_t r = 0; r < c->re.size(); ++r)
        for (int d = 0; d < 3; ++d) {
            if (!m[r].s[d]) return fail(c, HRT_EINVAL, "NULL displacement array");
            if (need_p && !m[r].p[d]) return fail(c, HRT_EINVAL, "NULL momentum array");
        }
    return HRT_OK;
}

static int check_rays(hrt_ctx *c, const hrt_rays *r, bool need_p, bool need_jac = false) {
    if (!c->has_rays) return fail(c, HRT_ESTATE, "configuration has no rays");
    if (!r) return fail(c, HRT_EINVAL, "NULL ray state");
    for (size_t k = 0; k < c->re.size(); ++k) {
        for (int d = 0; d < 2; ++d) {
            if (!r[k].dth[d]) return fail(c, HRT_EINVAL, "NULL ray deflection array");
            if (need_p && !r[k].p[d]) return fail(c, HRT_EINVAL, "NULL ray momentum array");
        }
        // a ray step also accumulates the time delay / line-of-sight integral when configured
        if (need_p && c->delay && !r[k].delay) return fail(c, HRT_EINVAL, "NULL delay array (HRT_TIME_DELAY)");
        if (need_p && c->los && !r[k].los) return fail(c, HRT_EINVAL, "NULL line-of-sight array (los_field)");
        if (need_jac)
            for (int q = 0; q < 8; ++q)
                if (!r[k].jac[q]) return fail(c, HRT_EINVAL, "NULL distortion array (HRT_JACOBIAN)");
    }
    return HRT_OK;
}

extern "C" int pm_force(hrt_ctx *c, const hrt_matter *m, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (step < 0 || step > c->N) return fail(c, HRT_EINVAL, "step out of range [0, n_steps]");
    if (int rc = check_matter(c, m, false)) return rc;
    hrt::StepArgs a;
    a.m = m;
    a.step = step;
    if (int rc = check_hip(c, hrt::launch_paint(c, a), "paint")) return rc;
    if (int rc = check_hip(c, hrt::launch_poisson(c), "poisson")) return rc;
    if (int rc = check_hip(c, hrt::launch_gradient(c), "gradient")) return rc;
    c->force_step = step;
    c->mesh_g_stale = false;
    return HRT_OK;
}

extern "C" int pm_step(hrt_ctx *c, const hrt_matter *m, int step) {
    if (!c) return HRT_EINVAL;
    if (c->is_static) return fail(c, HRT_ESTATE, "pm_step is not valid for a static run");
    if (int rc = check_matter(c, m, true)) return rc;
    if (int rc = pm_force(c, m, step)) return rc;
    hrt::StepArgs a;
    a.m = m;
    a.step = step;
    return check_hip(c, hrt::launch_matter_kd(c, a), "matter kick-drift");
}

extern "C" int ray_step(hrt_ctx *c, const hrt_rays *r, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (step < 0 || step > c->N) return fail(c, HRT_EINVAL, "step out of range [0, n_steps]");
    if (int rc = check_rays(c, r, true, c->jacobian)) return rc;
    if (c->force_step < 0) return fail(c, HRT_ESTATE, "no force mesh yet: call pm_force or pm_step first");
    if (!c->is_static && c->force_step != step)
        return fail(c, HRT_ESTATE, "ray_step must follow pm_step/pm_force of the same step");
    hrt::StepArgs a;
    a.r = r;
    a.step = step;
    if (int rc = check_hip(c, hrt::launch_plane_gradient(c, step), "lens planes")) return rc;
    if (c->ray_mesh) {
        if (int rc = check_hip(c, hrt::launch_ray_mesh(c, step), "ray mesh")) return rc;
        return check_hip(c, hrt::launch_ray_mesh_step(c, a), "ray step (ray mesh)");
    }
    return check_hip(c, hrt::launch_ray_step(c, a), "ray step");
}

extern "C" int ray_observe(hrt_ctx *c, const hrt_rays *r, const hrt_maps *maps) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (!c->jacobian) return fail(c, HRT_ESTATE, "ray_observe needs a context created with HRT_JACOBIAN");
    if (int rc = check_rays(c, r, false, true)) return rc;
    if (!maps) return fail(c, HRT_EINVAL, "NULL maps");
    std::vector<hrt_maps> none(c->re.size(), hrt_maps{});
    std::vector<double> w(c->re.size(), 0.0);
    std::vector<int> mode(c->re.size(), 0);
    hrt::StepArgs a;
    a.r = r;
    a.src_maps = maps;
    a.acc_maps = none.data();
    a.acc_w = w.data();
    a.acc_mode = mode.data();
    return check_hip(c, hrt::launch_convergence(c, a, true), "observe");
}

extern "C" int ray_convergence(hrt_ctx *c, const hrt_rays *r, void *const *kappa,
                               void *const *gamma1, void *const *gamma2, void *const *omega) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (int rc = check_rays(c, r, false)) return rc;
    if (!kappa) return fail(c, HRT_EINVAL, "NULL kappa");
    for (size_t k = 0; k < c->re.size(); ++k)
        if (!kappa[k]) return fail(c, HRT_EINVAL, "NULL kappa array");
    hrt::StepArgs a;
    a.r = r;
    a.kappa = kappa;
    a.g1 = gamma1;
    a.g2 = gamma2;
    a.om = omega;
    return check_hip(c, hrt::launch_convergence(c, a), "convergence");
}

// After the ray step that ends on boundary b: the maps of every source plane at b (Alg. 1
// `observe`), and the n_g-weighted sum (Eq. obs_accum: the first source plane along the
// schedule writes it, the later ones add to it). One launch for all realisations that have
// a source plane at b.
static int observe(hrt_ctx *c, const hrt_rays *r, int b, const hrt_maps *maps) {
    if (!maps || c->n_src == 0 || b > c->N) return HRT_OK;
    const int R = (int)c->re.size();
    std::vector<hrt_maps> src(R), acc(R);
    std::vector<double> w(R, 0.0);
    std::vector<int> mode(R, 0);
    bool any = false;
    for (int k = 0; k < R; ++k) {
        const hrt::StepTables &t = c->re[k].tab;
        src[k] = hrt_maps{};
        acc[k] = hrt_maps{};
        int first = c->N + 1;
        for (int i = 0; i < c->n_src; ++i) first = std::min(first, (int)t.src_step[i]);
        for (int i = 0; i < c->n_src; ++i) {
            if (t.src_step[i] != b) continue;
            src[k] = maps[(size_t)k * c->n_maps + i];
            if (t.has_src_w) {
                acc[k] = maps[(size_t)k * c->n_maps + c->n_src];
                w[k] = t.src_w[i];
                mode[k] = b == first ? 1 : 2;
            }
            any = any || src[k].kappa || src[k].gamma1 || src[k].gamma2 || src[k].omega || mode[k];
        }
    }
    if (!any) return HRT_OK;
    hrt::StepArgs a;
    a.r = r;
    a.src_maps = src.data();
    a.acc_maps = acc.data();
    a.acc_w = w.data();
    a.acc_mode = mode.data();
    return check_hip(c, hrt::launch_convergence(c, a, c->jacobian), "source-plane maps");
}

// Steps first..first+n-1 with the matter drift of each step counting the particles into
// the next step's paint bins (the state is not touched by anyone else in between); rays
// observed at the source planes the steps reach (maps may be NULL).
static int run_steps(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, int first, int n,
                     const hrt_maps *maps) {
    if (c->is_static) {
        if (int rc = pm_force(c, m, first)) return rc;
        for (int k = first; k < first + n; ++k) {
            if (int rc = ray_step(c, r, k)) return rc;
            if (int rc = observe(c, r, k + 1, maps)) return rc;
        }
        return HRT_OK;
    }
    // Particle order of the sequence (kd_tiles variant): 1 = Lagrangian order (pm_step's
    // kernels), 2 = paint-bin order (sorted-state kernels, G formed per tile and on the lens
    // planes only), 3 = the same with the tile kick-drift as a persistent pipelined kernel,
    // 4 = paint-bin order with x-pairs of tiles per kick-drift workgroup (FP32; FP64 runs
    // variant 2), 5 = 4 with the particles that leave their paint bin moved through a side
    // list instead of re-binning the whole state every step (FP32; re-binned once the list
    // holds P/16 entries), 6 = 5 with a limit of P/64, 7 = 5 with G formed per particle from
    // the pair's phi block (256 lanes per pair; sparse particle sets), 0 = bin order (5 in
    // FP32, 2 in FP64)
    // for sequences of kSortedMinSteps steps or more, whose per-step saving outweighs the
    // one-off cost of entering and leaving the sorted state. All give the same bits.
    constexpr int kSortedMinSteps = 8;
    const int order = c->variant[hrt::K_KD_TILES];
    const bool sorted = order >= 2 || (order == 0 && n >= kSortedMinSteps);
    bool list = sorted && !c->f64 && (order == 5 || order == 6 || order == 7 || order == 0);
    for (const hrt::Real &re : c->re) list = list && re.lay.list != 0;
    bool counted = false;
    int cur = 0;
    if (list) {
        hrt::StepArgs a;
        a.m = m;
        a.par = first & 1;
        a.list_shift = order == 6 ? 6 : 4;
        if (int rc = check_hip(c, hrt::launch_list_init(c, a), "list init")) return rc;
    }
    for (int k = first; k < first + n; ++k) {
        hrt::StepArgs a;
        a.m = m;
        a.step = k;
        a.counts_ready = counted;
        if (sorted) {
            a.state = k == first ? hrt::STATE_FROM_CALLER : hrt::STATE_SORTED;
            a.cur = cur;
            a.list = list;
            a.par = k & 1;
        }
        if (int rc = check_hip(c, hrt::launch_paint(c, a), "paint")) return rc;
        if (int rc = check_hip(c, hrt::launch_poisson(c), "poisson")) return rc;
        if (!sorted)
            if (int rc = check_hip(c, hrt::launch_gradient(c), "gradient")) return rc;
        c->force_step = k;
        a.counts_ready = false;
        a.count_next = k + 1 < first + n;
        if (int rc = check_hip(c, hrt::launch_matter_kd(c, a), "matter kick-drift")) return rc;
        if (list && a.count_next)
            if (int rc = check_hip(c, hrt::launch_list_settle(c, a), "list settle")) return rc;
        counted = a.count_next;
        if (r) {
            if (int rc = ray_step(c, r, k)) return rc;
            if (int rc = observe(c, r, k + 1, maps)) return rc;
        }
        cur ^= 1;                        // sorted: the next paint bins into the other buffer
    }
    if (sorted) {
        hrt::StepArgs a;
        a.m = m;
        a.cur = cur ^ 1;                 // the buffer the last step moved
        a.list = list;
        a.par = (first + n - 1) & 1;     // list: the last step's control words
        if (int rc = check_hip(c, hrt::launch_state_gather(c, a), "state gather")) return rc;
        c->mesh_g_stale = true;          // G was formed per tile in LDS, not on the mesh
    }
    return HRT_OK;
}

static int check_maps(hrt_ctx *c, const hrt_rays *r, const hrt_maps *maps) {
    if (maps && !r) return fail(c, HRT_EINVAL, "maps need the rays");
    if (maps && c->n_src == 0) return fail(c, HRT_EINVAL, "maps given but the configuration has no source planes");
    return HRT_OK;
}

extern "C" int hrt_run(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, int first_step,
                       int n_steps, const hrt_maps *maps) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (n_steps < 1 || first_step < 0 || first_step + n_steps > c->N + 1)
        return fail(c, HRT_EINVAL, "steps out of range [0, n_steps]");
    if (int rc = check_matter(c, m, !c->is_static)) return rc;
    if (r)
        if (int rc = check_rays(c, r, true)) return rc;
    if (c->is_static && !r) return fail(c, HRT_EINVAL, "a static run needs rays");
    if (int rc = check_maps(c, r, maps)) return rc;
    return run_steps(c, m, r, first_step, n_steps, maps);
}

extern "C" int hrt_graph_capture(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r,
                                 int first_step, int n_steps, const hrt_maps *maps) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (c->prof) return fail(c, HRT_ESTATE, "switch profiling off before capturing a graph");
    if (n_steps < 1 || first_step < 0 || first_step + n_steps > c->N + 1)
        return fail(c, HRT_EINVAL, "captured steps out of range [0, n_steps]");
    if (int rc = check_matter(c, m, !c->is_static)) return rc;
    if (r)
        if (int rc = check_rays(c, r, true)) return rc;
    if (int rc = check_maps(c, r, maps)) return rc;
    if (c->graph) {
        hipGraphExecDestroy(c->graph);
        c->graph = nullptr;
    }
    hipStream_t cap = nullptr, user = c->stream;
    if (int rc = check_hip(c, hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "capture stream"))
        return rc;
    c->stream = cap;
    // nothing runs while capturing: the force mesh the sequence leaves behind becomes
    // current only when the graph is launched
    const int force_before = c->force_step;
    const bool stale_before = c->mesh_g_stale;
    int rc = check_hip(c, hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
    if (rc == HRT_OK) rc = (c->is_static && !r) ? pm_force(c, m, first_step)
                                                : run_steps(c, m, r, first_step, n_steps, maps);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cap, &graph);
    c->stream = user;
    c->graph_force_step = c->force_step;
    c->graph_g_stale = c->mesh_g_stale;
    c->force_step = force_before;
    c->mesh_g_stale = stale_before;
    if (rc == HRT_OK) rc = check_hip(c, e, "end capture");
    if (rc == HRT_OK) rc = check_hip(c, hipGraphInstantiate(&c->graph, graph, nullptr, nullptr, 0),
                                     "graph instantiate");
    if (graph) hipGraphDestroy(graph);
    hipStreamDestroy(cap);
    return rc;
}

extern "C" int hrt_graph_launch(hrt_ctx *c) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (!c->graph) return fail(c, HRT_ESTATE, "no captured graph");
    if (int rc = check_hip(c, hipGraphLaunch(c->graph, c->stream), "graph launch")) return rc;
    c->force_step = c->graph_force_step;
    c->mesh_g_stale = c->graph_g_stale;
    return HRT_OK;
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

extern "C" int hrt_ic_2lpt(hrt_ctx *c, int realisation, const void *noise, const hrt_ic_params *ic,
                           const hrt_matter *out) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (realisation < 0 || realisation >= (int)c->re.size())
        return fail(c, HRT_EINVAL, "realisation index out of range");
    if (!noise || !ic || !out) return fail(c, HRT_EINVAL, "NULL argument");
    for (int d = 0; d < 3; ++d)
        if (!out->s[d] || !out->p[d]) return fail(c, HRT_EINVAL, "NULL output array");
    const hrt::Real &re = c->re[realisation];
    if (re.np < 16) return fail(c, HRT_EUNSUPPORTED, "initial conditions need ptcl_n >= 16");
    hrt::IcParams p;
    std::string err;
    if (int rc = hrt::ic_params(re.cfg, *ic, p, err)) return fail(c, rc, err);
    if (int rc = check_hip(c, hrt::launch_ic(c, realisation, noise, p, out), "initial conditions"))
        return rc;
    c->force_step = -1;          // the force mesh was used as scratch
    return HRT_OK;
}

// Reverse of step `step` for every realisation: matter kick-drift (matter) and/or ray
// kick-drift (r, rc non-NULL), with the force mesh recomputed first and the force's
// transpose applied to the summed force-mesh cotangent.
static int force_copy(hrt_ctx *c, int slot, bool save);

// slot >= 0: the force comes from that force slot instead of a paint and Poisson solve.
static int step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                    const hrt_rays *rc, int step, bool matter, int slot = -1) {
    if (!(c->re[0].cfg.flags & HRT_ADJOINT))
        return fail(c, HRT_ESTATE, "context was created without HRT_ADJOINT");
    if (step < 0 || step > c->N) return fail(c, HRT_EINVAL, "step out of range [0, n_steps]");
    if (int rc0 = check_matter(c, m, false)) return rc0;
    if (!mc) return fail(c, HRT_EINVAL, "NULL matter cotangent");
    for (size_t k = 0; k < c->re.size(); ++k)
        for (int d = 0; d < 3; ++d) {
            if (!mc[k].s[d]) return fail(c, HRT_EINVAL, "NULL displacement cotangent array");
            if (matter && !mc[k].p[d]) return fail(c, HRT_EINVAL, "NULL momentum cotangent array");
        }
    if ((r == nullptr) != (rc == nullptr))
        return fail(c, HRT_EINVAL, "ray state and ray cotangent must both be given or both be NULL");
    if (r) {
        if (int rc0 = check_rays(c, r, false)) return rc0;
        if (int rc0 = check_rays(c, rc, true)) return rc0;
    }
    if (!matter && !r) return fail(c, HRT_EINVAL, "nothing to differentiate: no rays and no matter step");
    if (slot >= 0) {
        if (int rc0 = force_copy(c, slot, false)) return rc0;
        c->force_step = step;
        c->mesh_g_stale = false;
    } else if (int rc0 = pm_force(c, m, step)) {
        return rc0;
    }
    int rc0 = check_hip(c, hrt::launch_step_vjp(c, m, r, mc, rc, step, matter), "step vjp");
    c->force_step = -1;          // the force mesh now holds the cotangent
    return rc0;
}

extern "C" int hrt_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r,
                            const hrt_matter *mc, const hrt_rays *rc, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    return step_vjp(c, m, r, mc, rc, step, !c->is_static);
}

// Copies between the context's force (G mesh, paint-bin offsets) and force slot `slot`.
static int force_copy(hrt_ctx *c, int slot, bool save) {
    for (hrt::Real &re : c->re) {
        char *sl = re.ws + re.lay.fslots + (size_t)slot * re.lay.fslot_bytes;
        char *g = re.ws + re.lay.grad;
        char *offs = re.ws + re.lay.bins + (size_t)re.lay.nbins * 4;    // after the counts
        const size_t gb = (size_t)re.n * re.n * re.n * 4 * (c->f64 ? 8 : 4), ob = (size_t)(re.lay.nbins + 1) * 4;
        hipError_t e = hipMemcpyAsync(save ? sl : g, save ? g : sl, gb, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(save ? sl + re.lay.fslot_g : offs, save ? offs : sl + re.lay.fslot_g, ob,
                               hipMemcpyDeviceToDevice, c->stream);
        if (int rc = check_hip(c, e, "force slot copy")) return rc;
    }
    return HRT_OK;
}

extern "C" int hrt_force_save(hrt_ctx *c, int slot) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (c->slot_step.empty()) return fail(c, HRT_ESTATE, "context has no force slots (HRT_FORCE_SLOTS)");
    if (slot < 0 || slot >= (int)c->slot_step.size()) return fail(c, HRT_EINVAL, "force slot out of range");
    if (c->force_step < 0 || c->mesh_g_stale)
        return fail(c, HRT_ESTATE, "no current force mesh to save (pm_step or pm_force first)");
    if (int rc = force_copy(c, slot, true)) return rc;
    c->slot_step[slot] = c->force_step;
    return HRT_OK;
}

extern "C" int hrt_step_vjp_saved(hrt_ctx *c, int slot, const hrt_matter *m, const hrt_rays *r,
                                  const hrt_matter *mc, const hrt_rays *rc, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (c->slot_step.empty()) return fail(c, HRT_ESTATE, "context has no force slots (HRT_FORCE_SLOTS)");
    if (slot < 0 || slot >= (int)c->slot_step.size()) return fail(c, HRT_EINVAL, "force slot out of range");
    if (c->slot_step[slot] != step) return fail(c, HRT_ESTATE, "force slot does not hold this step's force");
    return step_vjp(c, m, r, mc, rc, step, !c->is_static, slot);
}

extern "C" int pm_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_matter *mc, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (c->is_static) return fail(c, HRT_ESTATE, "pm_step_vjp is not valid for a static run");
    return step_vjp(c, m, nullptr, mc, nullptr, step, true);
}

extern "C" int ray_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                            const hrt_rays *rc, int step) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (!r || !rc) return fail(c, HRT_EINVAL, "ray_step_vjp needs the ray state and its cotangent");
    return step_vjp(c, m, r, mc, rc, step, false);
}

extern "C" int ray_convergence_vjp(hrt_ctx *c, void *const *kappa_bar, const hrt_rays *rc) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (int rc0 = check_rays(c, rc, false)) return rc0;
    if (!kappa_bar) return fail(c, HRT_EINVAL, "NULL kappa_bar");
    for (size_t k = 0; k < c->re.size(); ++k)
        if (!kappa_bar[k]) return fail(c, HRT_EINVAL, "NULL kappa_bar array");
    for (size_t k = 0; k < c->re.size(); ++k)
        if (int rc0 = check_hip(c, hrt::launch_convergence_vjp(c, (int)k, kappa_bar[k], &rc[k]),
                                "convergence vjp"))
            return rc0;
    return HRT_OK;
}

extern "C" int hrt_ic_2lpt_vjp(hrt_ctx *c, int realisation, const void *noise,
                               const hrt_ic_params *ic, const hrt_matter *cot, void *noise_bar) {
    if (!c) return HRT_EINVAL;
    if (int g = guard(c)) return g;
    if (realisation < 0 || realisation >= (int)c->re.size())
        return fail(c, HRT_EINVAL, "realisation index out of range");
    if (!noise || !ic || !cot || !noise_bar) return fail(c, HRT_EINVAL, "NULL argument");
    for (int d = 0; d < 3; ++d) {
        if (!cot->s[d] || !cot->p[d]) return fail(c, HRT_EINVAL, "NULL cotangent array");
        if (cot->s[d] == noise_bar || cot->p[d] == noise_bar)
            return fail(c, HRT_EINVAL, "noise_bar aliases a cotangent array");
    }
    if (noise == noise_bar) return fail(c, HRT_EINVAL, "noise_bar aliases noise");
    const hrt::Real &re = c->re[realisation];
    if (re.np < 16) return fail(c, HRT_EUNSUPPORTED, "initial conditions need ptcl_n >= 16");
    hrt::IcParams p;
    std::string err;
    if (int rc = hrt::ic_params(re.cfg, *ic, p, err)) return fail(c, rc, err);
    if (int rc = check_hip(c, hrt::launch_ic_vjp(c, realisation, noise, p, cot, noise_bar),
                           "initial conditions vjp"))
        return rc;
    c->force_step = -1;
    return HRT_OK;
}

extern "C" int hrt_mesh_ptr(const hrt_ctx *c, int realisation, int which, void **ptr) {
    if (!c || !ptr || realisation < 0 || realisation >= (int)c->re.size()) return HRT_EINVAL;
    const hrt::Real &re = c->re[realisation];
    const size_t T = c->f64 ? 8 : 4;
    const size_t n3 = (size_t)re.n * re.n * re.n;
    switch (which) {
        case HRT_MESH_DELTA: *ptr = re.ws + re.lay.mesh_r; return HRT_OK;
        case HRT_MESH_PHI: *ptr = re.ws + re.lay.mesh_r + n3 * T; return HRT_OK;
        case HRT_MESH_GRAD:
            if (c->mesh_g_stale) return HRT_ESTATE;   // paint-bin-order hrt_run: G only in LDS
            *ptr = re.ws + re.lay.grad;
            return HRT_OK;
        case HRT_MESH_LIST_CTL:
            if (!re.lay.list) return HRT_EINVAL;
            *ptr = re.ws + re.lay.list + hrt::list_offsets(0).ctl;
            return HRT_OK;
        default: return HRT_EINVAL;
    }
}
