// Internal declarations of the HRT library (not part of the public ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/hrt.h"

namespace hrt {

// Per-step scalars and shell plane lists, all FP64 on the host (see tables.cpp).
struct StepTables {
    std::vector<double> a, chi, K, D, d;     // N+1 each
    std::vector<int32_t> plane_begin, plane_count;   // N+1 each
    std::vector<int32_t> plane_mesh;         // mesh plane index (j mod n) per entry
    std::vector<int32_t> plane_rep;          // replica transform row per entry
    std::vector<double> plane_los;           // line-of-sight weight per entry
    int32_t max_count = 0;                   // most planes in one shell
    std::vector<double> plane_chi, plane_w;  // chi_j and weight w_j per entry
    std::vector<double> rm_lam, rm_mu;       // ray mesh (HRT_RAY_MESH): resolution limit and
    int32_t rm_n = 0;                        //   spacing per step; the run's mesh size
    std::vector<int32_t> src_step;           // step boundary of each source plane
    std::vector<double> src_w;               // n_g weights (Eq. obs_accum), if has_src_w
    bool has_src_w = false;
};

// Fills t for cfg; returns HRT_OK or an error with a message in err.
int build_tables(const hrt_config &cfg, StepTables &t, std::string &err);
int validate_config(const hrt_config &cfg, std::string &err);

// Everything the device needs for the 2LPT initial conditions (host FP64, see tables.cpp).
struct IcParams {
    double kf;              // 2 pi / box
    double cell_volume;     // (box / np)^3
    double amp, n_s;        // P(k) = amp k^n_s T(k)^2, sigma_8 normalised at a = 1
    double omega_m, h, s_sound, alpha, theta2;   // Eisenstein-Hu no-wiggle parameters
    double g1, g2, m1, m2;  // s = g1 s1 + g2 s2, p = m1 s1 + m2 s2 at the requested a
    double D1, f1, D2, f2, D1_today;   // growth factors (reported by hrt_ic_factors)
};
int ic_params(const hrt_config &cfg, const hrt_ic_params &in, IcParams &out, std::string &err);

// Device-side plane entry (one per shell plane).
struct PlaneEntry {
    double chi;        // comoving distance of the plane [Mpc/h]
    double w;          // kick weight
    int32_t mesh;      // mesh plane index (line-of-sight node index inside its replica)
    int32_t rep;       // replica transform row (0 without a replica table)
    double los_w;      // weight of the line-of-sight field on this plane (0 without one)
};

// Workspace carve-up of one realisation, identical in hrt_workspace_bytes and hrt_init.
struct Layout {
    size_t mesh_r, spec, spec2, grad, twiddle, bins, cursor, sorted, planes, adj, state, stack, reps,
        stack_phi, stack_delta, rm_mesh, rm_tw, list, fslots, total;
    size_t fslot_g, fslot_bytes;   // force slot: its G part's size, the whole slot's stride
    int64_t nbins;
};

// Mover-list run (kd_tiles variants 5 and 6, FP32): between re-binnings the particles that
// stay in their paint bin keep their slot in the bin-ordered record buffer (the bins'
// "fronts"); a particle that leaves its bin leaves a hole (record index -1) and goes, with
// every particle of the side list, to the list U, which is then sorted by bin into the side
// list S read by the next step. Every particle outside the fronts is in the list, so the
// holes number exactly the list's entries. Control words per step parity: a step with
// parity q reads ctl[q] and its settle writes ctl[1 - q].
struct ListCtl {
    unsigned int cur;        // record buffer holding the fronts
    unsigned int nlist;      // entries of S
    unsigned int holes;      // holes in the fronts (= entries of the list)
    unsigned int ucount;     // unused (0)
    unsigned int rebuilds;   // re-binnings so far in this run
    unsigned int limit;      // a step that starts with more list entries than this re-bins
    unsigned int pad[2];
};

// Byte offsets of the mover-list region of one realisation (P particles, nbins paint bins),
// used by the host layout and by the kernels that carve the region. The particle data of
// the run lie in the sorted-state regions as records [rec0 | S | rec1 | U] (P, P, P and 2P
// entries) and momenta [mom0 | S | mom1 | U] (3P, 3P, 3P values, then 3 x 2P: U's axes are
// 2P apart), so every list kernel indexes them from rec0 and mom0 with non-negative 32-bit
// offsets (host-checked: 15P < 2^31). U has room for 2P entries: kick-drift workgroup w
// appends to [ubase[w], ubase[w] + ucnt[w]), ubase[w] being the start of its inputs in the
// fronts plus in S (disjoint ranges below 2P).
struct ListOffsets {
    size_t ctl, lcount, lcursor, loffs, lsums, ubase, ucnt, total;
};
__host__ __device__ inline size_t list_al(size_t x) { return (x + 255) & ~(size_t)255; }
__host__ __device__ inline ListOffsets list_offsets(size_t nbins) {
    ListOffsets o{};
    const size_t nblk = (nbins + 1023) / 1024, npairs = nbins / 16;
    size_t at = 0;
    o.ctl = at;     at += list_al(2 * sizeof(ListCtl));
    o.lcount = at;  at += list_al(nbins * 4);
    o.lcursor = at; at += list_al(nbins * 4);
    o.loffs = at;   at += list_al((nbins + 1) * 4);
    o.lsums = at;   at += list_al((nblk + 1) * 4);
    o.ubase = at;   at += list_al(npairs * 4);
    o.ucnt = at;    at += list_al(npairs * 4);
    o.total = at;
    return o;
}

// Kernel ids for the optional per-kernel HIP-event timing (hrt_profile_*).
enum KernelId {
    K_BIN_COUNT = 0, K_BIN_SCAN, K_BIN_SCATTER, K_PAINT, K_FFT_X_R2C, K_FFT_Y_FWD, K_FFT_Z_POISSON,
    K_FFT_Y_INV, K_FFT_X_C2R, K_GRADIENT, K_MATTER_KD, K_RAY_STEP, K_CONVERGENCE,
    K_STATE_SCATTER, K_KD_TILES, K_PLANE_GRADIENT, K_STATE_GATHER, K_RAY_MESH, K_LIST_SETTLE, K_COUNT
};
struct ProfRecord {
    int id;
    hipEvent_t start, stop;
};

// Realisations per kernel launch: their pointers and scalars travel in the kernel's
// by-value argument block (well under the 4 KB limit); larger batches launch in chunks.
constexpr int kMaxBatch = 16;

// The ray part of the step VJP splits a step's lens planes over this many groups of
// workgroups (more waves than one per 64 rays); each group's per-ray partial sums of the
// deflection cotangent are added in group order afterwards (reverse-mode scratch).
constexpr int kRayVjpParts = 8;

// One realisation of a (possibly batched) context.
struct Real {
    hrt_config cfg;
    std::vector<double> sched;
    int n = 0, np = 0, mx = 0, my = 0;
    double cell = 0, box = 0;
    StepTables tab;
    Layout lay;
    char *ws = nullptr;          // this realisation's part of the workspace
    int fixed_bits = 0;          // paint fixed-point fraction bits
    bool identity_reps = true;   // every replica uses the identity transform
};

// Per-call state handed to the launchers: one entry per realisation.
struct StepArgs {
    const hrt_matter *m = nullptr;
    const hrt_rays *r = nullptr;
    int step = 0;
    void *const *kappa = nullptr;
    void *const *g1 = nullptr;
    void *const *g2 = nullptr;
    void *const *om = nullptr;
    // Source-plane observation (hrt_run maps): per realisation, the maps of this source
    // plane (entries may be NULL), the accumulated n_g-weighted maps, their weight and mode
    // (0 = none, 1 = write w * map, 2 = add w * map). A realisation with nothing to write is
    // skipped. Unused (NULL) for ray_convergence, which writes kappa for every realisation.
    const hrt_maps *src_maps = nullptr;
    const hrt_maps *acc_maps = nullptr;
    const double *acc_w = nullptr;
    const int *acc_mode = nullptr;
    // Fused bin histogram (hrt_run): the matter kick-drift also counts the drifted
    // particles into the paint bins of the next step, whose paint then skips its own count.
    bool count_next = false;     // launch_matter_kd: zero the counts, count the new positions
    bool counts_ready = false;   // launch_paint: the counts already hold these positions
    // Where the particle kernels find the state (hrt_run keeps it in paint-bin order between
    // its first and last step). The paint bins it into sorted-state buffer `cur` from the
    // caller's arrays (STATE_FROM_CALLER) or from buffer 1 - cur (STATE_SORTED); the
    // kick-drift then works on buffer cur in place.
    int state = 0;               // STATE_LAGRANGIAN, STATE_FROM_CALLER or STATE_SORTED
    int cur = 0;
    // Mover-list run (FP32 kd_tiles variants 0, 5, 6): the record buffer and the list sizes live in
    // the device control words ctl[par] (par = step parity) instead of `cur`.
    bool list = false;
    int par = 0;
    int list_shift = 4;          // list_init: re-bin beyond P >> list_shift list entries
};
enum { STATE_LAGRANGIAN = 0, STATE_FROM_CALLER = 1, STATE_SORTED = 2 };

// Blocks of realisation r are [start[r], start[r+1]); start[R] is the grid size.
struct BlockMap {
    int R;
    int start[kMaxBatch + 1];
};

}  // namespace hrt

struct hrt_ctx {
    std::vector<hrt::Real> re;   // realisations (a plain run is a batch of one)
    hipStream_t stream = nullptr;
    int N = 0;                   // shared number of steps
    bool f64 = false, is_static = false, has_rays = false, jacobian = false;
    bool delay = false;          // HRT_TIME_DELAY
    bool ray_mesh = false;       // HRT_RAY_MESH
    int los = 0;                 // line-of-sight field (HRT_LOS_*)
    int n_src = 0, n_maps = 0;   // source planes; map sets per realisation (+1 with weights)
    int force_step = -1;         // boundary of the phi (and G) currently in the workspaces
    std::vector<int> slot_step;  // force slots (HRT_FORCE_SLOTS): the step each holds, or -1
    bool mesh_g_stale = false;   // after a paint-bin-order hrt_run the G mesh is not current
    std::string err;
    // captured step sequence (hrt_graph_capture / hrt_graph_launch)
    hipGraphExec_t graph = nullptr;
    int graph_force_step = -1;   // force_step after the captured sequence has run
    bool graph_g_stale = false;  // mesh_g_stale after it
    // per-kernel timing (off unless hrt_profile_enable)
    bool prof = false;
    std::vector<hrt::ProfRecord> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    hipEvent_t prof_open = nullptr;
    double prof_ms[hrt::K_COUNT] = {};
    int64_t prof_n[hrt::K_COUNT] = {};
    // launch-shape variant per kernel id (hrt_autotune / hrt_set_variant; 0 = default)
    int variant[hrt::K_COUNT] = {};
    // workspace in the static no-allocation array (hrt_init_noalloc): its device and the
    // generation of that device's array this context was laid out in (-1: caller workspace)
    int noalloc_dev = -1;
    uint64_t noalloc_gen = 0;
    ~hrt_ctx();
};

namespace hrt {
// hrt_init on an explicit workspace (shared by hrt_init and hrt_init_noalloc).
int init_context(const hrt_config *cfg, int n_cfg, void *workspace, size_t ws_bytes, void *stream,
                 hrt_ctx **out);
// Records the message returned by hrt_last_error(NULL) and returns code.
int set_init_error(int code, const std::string &msg);
// True if c lives in the static no-allocation array of its device and a later
// hrt_init_noalloc on that device has laid the array out for another context.
bool noalloc_superseded(const hrt_ctx *c);
}  // namespace hrt

// Kernel launchers (defined in the .hip files); each covers every realisation of the
// context with one launch per kernel type (per mesh-size class for the FFT passes) and
// returns hipSuccess or the error.
namespace hrt {
void prof_begin(hrt_ctx *c);           // record a start event when profiling is on
void prof_end(hrt_ctx *c, int id);     // record the stop event of kernel `id`
hipError_t launch_paint(hrt_ctx *c, const StepArgs &a);
hipError_t launch_poisson(hrt_ctx *c, int only = -1);   // every realisation, or only `only`
hipError_t launch_gradient(hrt_ctx *c);
hipError_t launch_plane_gradient(hrt_ctx *c, int step);      // the step's lens-plane stack
hipError_t launch_state_gather(hrt_ctx *c, const StepArgs &a);   // sorted state -> caller
// Mover-list run: list_init before the first step (control words of parity a.par, empty S);
// list_settle after a step's kick-drift: scan of the mover histogram and sort of U into S,
// or (once the holes or the list pass their limit) a full re-binning into the other buffer.
hipError_t launch_list_init(hrt_ctx *c, const StepArgs &a);
hipError_t launch_list_settle(hrt_ctx *c, const StepArgs &a);
hipError_t launch_matter_kd(hrt_ctx *c, const StepArgs &a);
hipError_t launch_ray_step(hrt_ctx *c, const StepArgs &a);
// HRT_RAY_MESH: the step's kick on the 2D ray mesh (projection of the lens-plane stack,
// FFT deconvolution and smoothing), then the readout / drift kernel for the rays
hipError_t launch_ray_mesh(hrt_ctx *c, int step);
hipError_t launch_ray_mesh_step(hrt_ctx *c, const StepArgs &a);
hipError_t launch_convergence(hrt_ctx *c, const StepArgs &a, bool from_a = false);
hipError_t launch_ic(hrt_ctx *c, int realisation, const void *noise, const IcParams &p,
                     const hrt_matter *m);
// Reverse-mode scratch of one realisation (HRT_ADJOINT): fixed-point ray contributions to
// the cotangent of G_x, G_y (2 n^3), the largest contribution (double bits), and the
// particles' kick weights K p_bar in paint-bin order (P x 4 values of the dtype).
struct AdjScratch {
    unsigned long long *gbar;
    unsigned long long *maxbits;
    void *wsorted;
    int hbits;
};
// Matter part of the step VJP of realisation k: p_bar += D s_bar; s_bar += K (d readout/dx)^T p_bar; the
// particles re-binned with their weights; the largest weight into *maxbits.
hipError_t launch_matter_vjp(hrt_ctx *c, int k, const hrt_matter *m, const hrt_matter *mc, int step,
                             const AdjScratch &s);
// Force-mesh cotangent: per tile, the particles' CIC-weighted K p_bar summed in LDS plus
// the rays' part from s.gbar (if rays), converted into the G mesh slot.
hipError_t launch_gbar_tiles(hrt_ctx *c, int k, bool rays, const AdjScratch &s);
// Reverse mode (every realisation of a context created with HRT_ADJOINT, see adjoint.hip).
hipError_t launch_step_vjp(hrt_ctx *c, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                           const hrt_rays *rc, int step, bool matter);
hipError_t launch_convergence_vjp(hrt_ctx *c, int realisation, const void *kappa_bar,
                                  const hrt_rays *rc);
hipError_t launch_ic_vjp(hrt_ctx *c, int realisation, const void *noise, const IcParams &p,
                         const hrt_matter *cot, void *noise_bar);
}  // namespace hrt
