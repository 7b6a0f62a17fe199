// hrt_init_noalloc: a context whose workspace is a static device array of the library,
// for callers that cannot allocate device memory (declaration and contract in
// include/hrt.h). The array is sized HRT_NOALLOC_MAX_BYTES; every device the library runs
// on holds its own copy until the process ends. Its address is looked up once per device
// with hipGetSymbolAddress (the array's name in host code is not a device address) and the
// context's realisations are laid out inside it exactly as in a caller's workspace, so
// every entry point runs the same kernels on it. Nothing in the workspace needs to start
// at zero: the kernels clear what they accumulate into (bin counts, reverse-mode sums).
#include <atomic>
#include <mutex>

#include "hrt_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[HRT_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices] = {};                  // device address of `scratch` per device
std::atomic<uint64_t> g_gen[kMaxDevices] = {};  // layouts handed out per device

}  // namespace

bool hrt::noalloc_superseded(const hrt_ctx *c) {
    if (!c || c->noalloc_dev < 0) return false;
    return g_gen[c->noalloc_dev].load() != c->noalloc_gen;
}

extern "C" int hrt_init_noalloc(const hrt_config *cfg, int n_cfg, void *stream, hrt_ctx **out) {
    if (!cfg || !out) return hrt::set_init_error(HRT_EINVAL, "NULL argument");
    *out = nullptr;
    size_t need = 0;
    if (int rc = hrt_workspace_bytes(cfg, n_cfg, &need)) return rc;
    if (need > (size_t)HRT_NOALLOC_MAX_BYTES)
        return hrt::set_init_error(HRT_ENOMEM, "configuration needs " + std::to_string(need) +
                                                   " bytes of workspace; the static no-allocation "
                                                   "workspace holds " +
                                                   std::to_string((size_t)HRT_NOALLOC_MAX_BYTES));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return hrt::set_init_error(HRT_EDEVICE, "no current HIP device");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!g_ptr[dev]) {
            // the current device is `dev`: the symbol resolves to that device's copy
            hipError_t e = hipGetSymbolAddress(&g_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_ptr[dev]) {
                g_ptr[dev] = nullptr;
                return hrt::set_init_error(HRT_EDEVICE, std::string("hipGetSymbolAddress: ") +
                                                            hipGetErrorString(e));
            }
        }
        ptr = g_ptr[dev];
    }
    // Contexts laid out earlier in this device's array are superseded from here on, also if
    // this initialisation fails part way (the tables upload may have overwritten them).
    const uint64_t gen = g_gen[dev].fetch_add(1) + 1;
    hrt_ctx *c = nullptr;
    if (int rc = hrt::init_context(cfg, n_cfg, ptr, (size_t)HRT_NOALLOC_MAX_BYTES, stream, &c)) return rc;
    c->noalloc_dev = dev;
    c->noalloc_gen = gen;
    *out = c;
    return HRT_OK;
}
