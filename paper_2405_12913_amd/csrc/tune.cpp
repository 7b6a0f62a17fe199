// Launch-shape variants and their autotuner (C ABI in include/hrt.h).
//
// A variant only changes how particles or rays are mapped onto workgroups and lanes (patch
// shapes, particles per lane) and whether workgroups are grouped per XCD; the arithmetic of
// every particle, ray and mesh node is the same, so all variants give bit-identical results. The tuner times each variant on
// the context's own shapes and keeps the fastest; choices persist in a small JSON file
// keyed by device architecture, kernel, dtype and sizes.
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>

#include "hrt_internal.h"

namespace {

using hrt::K_BIN_COUNT;
using hrt::K_BIN_SCATTER;
using hrt::K_COUNT;
using hrt::K_MATTER_KD;
using hrt::K_PAINT;
using hrt::K_RAY_STEP;

int variants_of(int id) {
    switch (id) {
        case K_MATTER_KD: return 16;
        case K_BIN_COUNT: case K_BIN_SCATTER: return 8;
        case K_RAY_STEP: return 6;
        case K_PAINT: return 14;
        case hrt::K_KD_TILES: return 8;      // run order: 0 automatic, 1 Lagrangian, 2 sorted state,
                                             // 3 sorted state with a pipelined persistent kick-drift,
                                             // 4 sorted state with x-pairs of tiles per workgroup,
                                             // 5 as 4 with the movers in a side list (FP32),
                                             // 6 as 5 with re-binnings eight times as often,
                                             // 7 as 5 with G formed per particle from phi
        default: return (id >= 0 && id < K_COUNT) ? 1 : 0;
    }
}

struct Entry {
    int variant;
    double us;
};

// Reads the entries of a cache file written by write_cache; a missing or unreadable file
// gives no entries.
std::map<std::string, Entry> read_cache(const char *path) {
    std::map<std::string, Entry> out;
    std::ifstream f(path);
    if (!f) return out;
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    const std::string kk = "\"key\": \"", kv = "\"variant\": ", ku = "\"us\": ";
    while ((pos = s.find(kk, pos)) != std::string::npos) {
        pos += kk.size();
        const size_t end = s.find('"', pos);
        if (end == std::string::npos) break;
        const std::string key = s.substr(pos, end - pos);
        const size_t v = s.find(kv, end), u = s.find(ku, end), next = s.find(kk, end);
        if (v == std::string::npos || (next != std::string::npos && v > next)) { pos = end; continue; }
        Entry e{std::atoi(s.c_str() + v + kv.size()), 0.0};
        if (u != std::string::npos && (next == std::string::npos || u < next))
            e.us = std::atof(s.c_str() + u + ku.size());
        out[key] = e;
        pos = end;
    }
    return out;
}

bool write_cache(const char *path, const std::map<std::string, Entry> &m) {
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp);
        if (!f) return false;
        f << "{\n  \"hrt_tuning\": 1,\n  \"entries\": [\n";
        size_t k = 0;
        for (const auto &kv : m) {
            char us[64];
            std::snprintf(us, sizeof us, "%.3f", kv.second.us);
            f << "    {\"key\": \"" << kv.first << "\", \"variant\": " << kv.second.variant
              << ", \"us\": " << us << "}" << (++k < m.size() ? ",\n" : "\n");
        }
        f << "  ]\n}\n";
        if (!f) return false;
    }
    return std::rename(tmp.c_str(), path) == 0;
}

std::string shape_key(const hrt_ctx *c, int id) {
    hipDeviceProp_t prop{};
    int dev = 0;
    std::string arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    std::string k = arch + "|" + hrt_kernel_name(id) + "|" + (c->f64 ? "f64" : "f32") + "|";
    for (size_t r = 0; r < c->re.size(); ++r) {
        const hrt::Real &re = c->re[r];
        char buf[96];
        std::snprintf(buf, sizeof buf, "%s%d/%d/%dx%d", r ? "," : "", re.n, re.np, re.mx, re.my);
        k += buf;
    }
    return k;
}

}  // namespace

extern "C" int hrt_num_variants(int kernel_id) { return variants_of(kernel_id); }

extern "C" int hrt_set_variant(hrt_ctx *c, int kernel_id, int variant) {
    if (!c) return HRT_EINVAL;
    if (variant < 0 || variant >= variants_of(kernel_id)) {
        c->err = "variant out of range for this kernel";
        return HRT_EINVAL;
    }
    c->variant[kernel_id] = variant;
    return HRT_OK;
}

extern "C" int hrt_get_variant(const hrt_ctx *c, int kernel_id, int *variant) {
    if (!c || !variant || kernel_id < 0 || kernel_id >= K_COUNT) return HRT_EINVAL;
    *variant = c->variant[kernel_id];
    return HRT_OK;
}

extern "C" int hrt_autotune(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, int step,
                            const char *cache_path) {
    if (!c) return HRT_EINVAL;
    if (c->is_static) {
        c->err = "autotuning needs a cosmological configuration";
        return HRT_ESTATE;
    }
    if (r && !c->has_rays) {
        c->err = "configuration has no rays";
        return HRT_ESTATE;
    }
    if (int rc = pm_force(c, m, step)) return rc;            // checks m and step, sets G
    for (size_t k = 0; k < c->re.size(); ++k)
        for (int d = 0; d < 3; ++d)
            if (!m[k].p[d]) {
                c->err = "autotuning needs the momenta (scratch)";
                return HRT_EINVAL;
            }
    if (r)
        for (size_t k = 0; k < c->re.size(); ++k) {
            for (int d = 0; d < 2; ++d)
                if (!r[k].dth[d] || !r[k].p[d]) {
                    c->err = "NULL ray array";
                    return HRT_EINVAL;
                }
            if (c->jacobian)
                for (int q = 0; q < 8; ++q)
                    if (!r[k].jac[q]) {
                        c->err = "NULL distortion array (HRT_JACOBIAN)";
                        return HRT_EINVAL;
                    }
            if ((c->delay && !r[k].delay) || (c->los && !r[k].los)) {
                c->err = "NULL delay or line-of-sight array";
                return HRT_EINVAL;
            }
        }
    std::map<std::string, Entry> cache;
    if (cache_path) cache = read_cache(cache_path);
    bool dirty = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        c->err = "event creation failed";
        return HRT_EDEVICE;
    }
    hrt::StepArgs sa;
    sa.m = m;
    sa.r = r;
    sa.step = step;
    const int ids[] = {K_BIN_COUNT, K_BIN_SCATTER, K_PAINT, K_MATTER_KD, K_RAY_STEP};
    hipError_t err = hipSuccess;
    for (int id : ids) {
        if (id == K_RAY_STEP && !r) continue;
        if (id == K_RAY_STEP) err = hrt::launch_plane_gradient(c, step);   // the lens planes it reads
        if (err != hipSuccess) break;
        const std::string key = shape_key(c, id);
        auto it = cache.find(key);
        if (it != cache.end() && it->second.variant >= 0 && it->second.variant < variants_of(id)) {
            c->variant[id] = it->second.variant;
            continue;
        }
        auto run = [&]() -> hipError_t {
            if (id == K_MATTER_KD) return hrt::launch_matter_kd(c, sa);
            if (id == K_RAY_STEP) return hrt::launch_ray_step(c, sa);
            return hrt::launch_paint(c, sa);
        };
        int best = 0;
        double best_us = 0.0;
        for (int v = 0; v < variants_of(id) && err == hipSuccess; ++v) {
            c->variant[id] = v;
            const int reps = 5;
            err = run();                                         // warm-up
            if (err == hipSuccess) err = hipEventRecord(e0, c->stream);
            for (int k = 0; k < reps && err == hipSuccess; ++k) err = run();
            if (err == hipSuccess) err = hipEventRecord(e1, c->stream);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            const double us = 1e3 * ms / reps;
            if (v == 0 || us < best_us) {
                best = v;
                best_us = us;
            }
        }
        if (err != hipSuccess) break;
        c->variant[id] = best;
        cache[key] = Entry{best, best_us};
        dirty = true;
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (err != hipSuccess) {
        c->err = std::string("autotune: ") + hipGetErrorString(err);
        return HRT_EDEVICE;
    }
    c->force_step = -1;            // the tuning runs moved the state the mesh was made from
    if (cache_path && dirty && !write_cache(cache_path, cache)) {
        c->err = std::string("autotune: cannot write ") + cache_path;
        return HRT_EINVAL;
    }
    return HRT_OK;
}
