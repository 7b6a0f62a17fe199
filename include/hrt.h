/*
 * hrt.h - C ABI of the MI355X (gfx950) Hamiltonian ray tracing hot path.
 *
 * One particle-mesh (PM) gravity step co-evolved with light rays, following
 * Zhou et al., "A Hamiltonian, post-Born, three-dimensional, on-the-fly ray
 * tracing algorithm for gravitational lensing" (arXiv:2405.12913):
 *   pm_force        CIC paint + FFT Poisson solve + gradient   (Sec. 2 Poisson eq.; Sec. 5.1-5.2)
 *   pm_step         pm_force + matter kick and drift           (Alg. 1, nbody_reverse_step)
 *   ray_step        ray kick over one lens shell + ray drift   (Eqs. symp_1-3, kick, drift)
 *   ray_convergence kappa (gamma1, gamma2, omega) from finite  (Eqs. A, obs_first_set,
 *                   differences of the ray deflections          obs_second_set)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All device pointers are caller-owned. The library never allocates device memory:
 *   its scratch (meshes, FFT buffers, sort bins, step tables) lives in one
 *   caller-allocated workspace of hrt_workspace_bytes() bytes that must stay alive and
 *   untouched until hrt_destroy().
 * - Every GPU entry point only enqueues work on the stream given to hrt_init and
 *   returns without synchronising the host. Calls on one context are not thread-safe
 *   and must be issued in order; results are ready after the stream synchronises.
 * - Return value: HRT_OK (0) or a negative hrt_status; hrt_last_error() gives a text.
 *   Invalid arguments are reported before anything is enqueued.
 * - Floating point type of every state array and output is the config's dtype
 *   (HRT_F32 -> float, HRT_F64 -> double).
 * - Mesh layout: n^3 nodes at x = i * box/n, row-major [z][y][x], the line of sight is
 *   +z. Particle i = (iz*np + iy)*np + ix has Lagrangian position
 *   q = (ix, iy, iz) * box/np; the state stores the displacement s = x - q and the
 *   momentum p = a^2 dx/dt / H0 (Mpc/h). Ray i = iy*Mx + ix sits at the pixel centre
 *   theta0 = ((ix + 1/2) - Mx/2, (iy + 1/2) - My/2) * fov/M (radians); the state stores
 *   dth = theta - theta0 and the canonical momentum p with d theta/d chi = p / chi^2.
 * - Determinism: no floating-point atomics anywhere; two runs give identical bits.
 * - Batches: a context holds n_cfg >= 1 realisations (different seeds, cosmologies, mesh
 *   sizes and ray grids; they must share dtype, n_steps, flags and whether they have
 *   rays). Every step entry point then takes arrays of n_cfg state structs and launches
 *   each kernel type once for all realisations (once per mesh size for the FFT passes).
 *   Results per realisation are bit-identical to running it alone.
 */
#ifndef HRT_H
#define HRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HRT_OK = 0,
    HRT_EINVAL = -1,        /* invalid argument or configuration                    */
    HRT_ENOMEM = -2,        /* workspace too small                                   */
    HRT_EDEVICE = -3,       /* a HIP call or kernel launch failed                    */
    HRT_ESTATE = -4,        /* call not valid in the context's state                 */
    HRT_EUNSUPPORTED = -5   /* valid request this build does not implement           */
} hrt_status;

enum { HRT_F32 = 0, HRT_F64 = 1 };

/* flags */
enum {
    HRT_STATIC = 1,         /* static point-lens run: a = 1, sched holds chi_n, the mesh
                               source is unit-weight particles of mass static_mass each */
    HRT_ADJOINT = 2,        /* reserve the reverse-mode scratch (hrt_step_vjp) in the
                               workspace: 16 n^3 + 256 + 4 np^3 sizeof(dtype) bytes more */
    HRT_TIME_DELAY = 8,     /* the rays accumulate c times the arrival-time delay (Sec. 2,
                               Eq. eom3: geometric p^2/(2 r^2) and Shapiro -2 Phi/c^2 per
                               unit chi) in hrt_rays.delay [Mpc/h]; not with HRT_ADJOINT   */
    HRT_RAY_MESH = 16,      /* the paper's kick operator (Sec. 5.2, 5.3, App. C): each
                               step's shell is projected onto an adaptive 2D ray mesh
                               (CIC), deconvolved (sinc^-4), smoothed at the resolution limit
                               of Eq. reslim (Gaussian, negative exponent) and read at the
                               rays (CIC), instead of the plane-sum readout; mesh spacing
                               ray_mesh_iota * lam per step, size the smallest power of two
                               (<= 2048, else HRT_EUNSUPPORTED) that holds the field plus
                               ray_mesh_pmin * lam of padding at every step. Not with
                               HRT_ADJOINT, HRT_TIME_DELAY or a line-of-sight integral    */
    HRT_JACOBIAN = 4        /* the rays carry the forward-mode distortion recursion of
                               Sec. 4 (Eqs. A, B, obsv_recurse1-3; Alg. 1 iterate_A,
                               iterate_B): hrt_rays.jac required by ray_step; source-plane
                               maps are formed from A instead of finite differences.
                               Not combinable with HRT_ADJOINT (HRT_EUNSUPPORTED)       */
};

/* HRT_FORCE_SLOTS(k), 1 <= k <= 15, or'ed into flags together with HRT_ADJOINT: reserve k
 * force slots for hrt_force_save / hrt_step_vjp_saved, k (16 n^3 sizeof(dtype) +
 * 4 (n^3/64 + 1)) bytes more per realisation (each slot rounded up to 256 bytes per part). */
#define HRT_FORCE_SLOTS(k) ((int32_t)(k) << 8)
#define HRT_FORCE_SLOTS_MASK 0xf00

typedef struct {
    int32_t mesh_n;         /* n: power of two, 16 <= n <= 1024                         */
    int32_t ptcl_n;         /* np particles per side, n % np == 0 (np = 1: one particle) */
    int32_t ray_nx, ray_ny; /* Mx, My >= 3 (0 = no rays)                                */
    int32_t n_steps;        /* N >= 1                                                    */
    int32_t dtype;          /* HRT_F32 or HRT_F64                                        */
    int32_t flags;          /* HRT_STATIC and/or HRT_ADJOINT, or 0                      */
    int32_t n_src;          /* number of source planes, 0 <= n_src <= HRT_MAX_SOURCES    */
    double box;             /* periodic box side L [Mpc/h]                               */
    double fov_x, fov_y;    /* field of view [rad]                                       */
    double observer[3];     /* observer position in box coordinates [Mpc/h]              */
    double omega_m;         /* matter density (flat LambdaCDM, no radiation)             */
    double static_mass;     /* M [Msun/h] per particle when HRT_STATIC                   */
    const double *sched;    /* N+1 host values: a_0..a_N (cosmological, any direction,
                               0 < a <= 1) or chi_0..chi_N [Mpc/h] when HRT_STATIC;
                               copied at hrt_init                                        */
    const double *src;      /* n_src host values (NULL if n_src = 0), each a step boundary
                               1..N of sched: the source redshift z (a = 1/(1+z) must equal
                               some a_k to 1e-9 relative) or, with HRT_STATIC, the source
                               distance chi [Mpc/h] (equal to some chi_k to 1e-9 relative);
                               distinct boundaries; rays required. Alg. 1 observes the rays
                               at these planes (hrt_run / hrt_graph_capture maps).
                               HRT_EINVAL if a value is not a boundary. Copied at init.  */
    const double *src_w;    /* NULL, or n_src weights n_g(chi_i) of the source distribution
                               (Eq. obs_accum): the maps then also accumulate
                               sum_i src_w[i] * map_i into one more map set              */
    const int32_t *replicas;/* NULL (plain periodic replication), or n_replicas rows of 9
                               values: the light cone is the box replicated along the line
                               of sight (Sec. 6.2), replica k holding the planes j with
                               k n <= j < (k+1) n and using row k mod n_replicas =
                               (perm0, perm1, perm2, sign0, sign1, sign2, shift0, shift1,
                               shift2): replica axis a (x, y, z = line of sight) runs along
                               box axis perm[a] (a permutation of 0, 1, 2) with orientation
                               sign[a] = +-1, and replica node u sits on box node
                               x[perm[a]] = sign[a] u[a] + shift[perm[a]] (mod n), 0 <=
                               shift < n. Copied at init. Not combinable with HRT_ADJOINT
                               unless every row is the identity (HRT_EUNSUPPORTED)       */
    int32_t n_replicas;     /* rows in replicas (0 when NULL), <= HRT_MAX_REPLICAS       */
    int32_t los_field;      /* line-of-sight integral O = int dchi P(chi) Q along the ray
                               (Sec. 4, Eq. integral), accumulated in hrt_rays.los:
                               HRT_LOS_NONE, HRT_LOS_DENSITY (Q = delta) or
                               HRT_LOS_POTENTIAL (Q = Phi/c^2); Q of the step's mesh carried
                               to each plane's time with the kick's linear-growth
                               correction (Eq. kick). Not with HRT_ADJOINT                */
    int32_t los_n;          /* knots of P (>= 2 when los_field != 0)                      */
    const double *los_chi;  /* los_n increasing chi [Mpc/h]; P is linear between knots and
                               0 outside them                                             */
    const double *los_p;    /* los_n values of P; both copied at init                      */
    double ray_mesh_iota;   /* HRT_RAY_MESH: accuracy parameter iota, 0 < iota <= 1       */
    double ray_mesh_pmin;   /* HRT_RAY_MESH: minimum padding p_min >= 0 in units of lam   */
} hrt_config;

enum { HRT_LOS_NONE = 0, HRT_LOS_DENSITY = 1, HRT_LOS_POTENTIAL = 2 };

enum { HRT_MAX_SOURCES = 256, HRT_MAX_REPLICAS = 4096 };

/* Output maps of one source plane (or of the weighted sum over the source planes): device
 * arrays of Mx*My values of the config's dtype, caller-owned; any may be NULL (not
 * written). */
typedef struct { void *kappa, *gamma1, *gamma2, *omega; } hrt_maps;

typedef struct { void *s[3]; void *p[3]; } hrt_matter;   /* device SoA, np^3 each (x, y, z) */
/* device SoA, Mx*My values each: deflection dth = theta - theta0 (x, y), canonical momentum
 * p (x, y), and with HRT_JACOBIAN the distortion recursion jac = (A - I)_xx, (A - I)_xy,
 * (A - I)_yx, (A - I)_yy, B_xx, B_xy, B_yx, B_yy with A = d theta / d theta0, B = d p /
 * d theta0 (A_ab: component a, derivative along b); all zero at the observer (A_0 = I,
 * B_0 = 0). jac entries are ignored (may be NULL) without HRT_JACOBIAN; delay (with
 * HRT_TIME_DELAY) and los (with a line-of-sight integral) are accumulated in place (zero at
 * the observer) and ignored otherwise. A quantity read at boundary k holds the planes of the
 * kicks applied so far: the closing half-kick (step N) adds the last half shell, as it does
 * for the momentum. */
typedef struct { void *dth[2]; void *p[2]; void *jac[8]; void *delay; void *los; } hrt_rays;

typedef struct hrt_ctx hrt_ctx;

/* Bytes of device workspace needed for the n_cfg configurations cfg[0..n_cfg-1].
 * Pure host function. */
int hrt_workspace_bytes(const hrt_config *cfg, int n_cfg, size_t *bytes);

/* Validates cfg[0..n_cfg-1], builds the FP64 step tables on the host and uploads them
 * into the workspace (synchronously). stream is a hipStream_t (NULL = default stream).
 * The context keeps no pointer to cfg or cfg->sched. */
int hrt_init(const hrt_config *cfg, int n_cfg, void *workspace, size_t ws_bytes, void *stream,
             hrt_ctx **out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): hrt_init without a caller workspace.
 * The workspace is a static device array of the library, HRT_NOALLOC_MAX_BYTES bytes on
 * every device the library runs on (held until the process ends); the context is laid
 * out in the array of the device current at the call, which must also be the device of
 * `stream` and of every state array. The call allocates no device memory (it uploads the
 * step tables into the array and synchronises the stream, as hrt_init does). Returns
 * HRT_ENOMEM, with the size needed in hrt_last_error(NULL), if hrt_workspace_bytes(cfg,
 * n_cfg) exceeds HRT_NOALLOC_MAX_BYTES. All contexts created this way on one device share
 * that one array: a context stays valid until the next hrt_init_noalloc on its device
 * (after which its GPU entry points return HRT_ESTATE; hrt_destroy is still required),
 * and work of two such contexts that overlaps in time on one device races. Everything
 * else (entry points, results, bits) is as for a context from hrt_init. */
#define HRT_NOALLOC_MAX_BYTES 67108864
int hrt_init_noalloc(const hrt_config *cfg, int n_cfg, void *stream, hrt_ctx **out);

/* Frees the host-side context (does not touch the caller's device memory). */
int hrt_destroy(hrt_ctx *ctx);

/* Text of the last error of ctx, or of the last failed hrt_init when ctx is NULL. */
const char *hrt_last_error(const hrt_ctx *ctx);

/* Paint the matter at boundary `step` (0 <= step <= N) onto the mesh, solve
 * grad^2 phi = delta (delta = rho/rho_bar - 1, Sec. 2 Poisson equation without its
 * prefactor, which the step tables carry) and store G = grad(phi) in the workspace.
 * m points to n_cfg states; their p arrays may be NULL. */
int pm_force(hrt_ctx *ctx, const hrt_matter *m, int step);

/* pm_force, then the matter kick p += K_step * G(q + s) and drift s += D_step * p
 * (fused leapfrog; step N is the closing half-kick with no drift). Not valid with
 * HRT_STATIC (returns HRT_ESTATE). */
int pm_step(hrt_ctx *ctx, const hrt_matter *m, int step);

/* Kick the rays over lens shell `step` with the potential left by the last pm_force /
 * pm_step / hrt_run of that step, evaluated at the current angles, then drift (step N:
 * closing half-kick, no drift). The step's lens planes are first formed from phi: plane j
 * holds the transverse gradient (G_u, G_v) in the frame of its replica (fourth-order
 * differences, mesh plane j mod n without replica transforms); each contributes
 * w_j * bilinear(G_u, G_v)(X_obs + chi_j * theta). With HRT_JACOBIAN also
 * B += J (I + dA), dA += d_step B with J = d kick / d theta (the plane sum of w_j chi_j
 * times the gradient of the bilinear interpolant). */
int ray_step(hrt_ctx *ctx, const hrt_rays *r, int step);

/* Finite-difference distortion matrix of the deflections over the pixel grid
 * (central inside, second-order one-sided on the edges) and kappa, gamma1, gamma2,
 * omega of Eq. obs_first_set. Each output is an array of n_cfg device pointers to
 * Mx*My values of the realisation; gamma1, gamma2 and omega may be NULL (the ray
 * momenta in r may be NULL too). */
int ray_convergence(hrt_ctx *ctx, const hrt_rays *r, void *const *kappa, void *const *gamma1,
                    void *const *gamma2, void *const *omega);

/* The same maps from the forward-mode distortion A = I + dA of a context created with
 * HRT_JACOBIAN (Alg. 1 `observe`, Eqs. obs_first_set, obs_second_set): maps points to
 * n_cfg entries (members may be NULL). HRT_ESTATE without HRT_JACOBIAN. */
int ray_observe(hrt_ctx *ctx, const hrt_rays *r, const hrt_maps *maps);

/* Runs steps first_step .. first_step+n_steps-1: pm_step then ray_step for every
 * realisation (r may be NULL for matter only); with HRT_STATIC one pm_force then the ray
 * steps (r required). Results are bit-identical to calling pm_step / ray_step step by step.
 * maps (NULL, or n_cfg * n_maps entries, realisation-major, n_maps = n_src + 1 with source
 * weights, else n_src): when a step ends on the boundary of source plane i, the maps of
 * ray_convergence at that plane go to maps[r * n_maps + i] (NULL members are skipped), and
 * with src_w the weighted sum of Eq. obs_accum to maps[r * n_maps + n_src] (written at the
 * first source plane along the schedule, added to at the later ones; every member of that
 * entry that is not NULL). Requires rays and n_src > 0 (else HRT_EINVAL).
 * Particle order (variant of kernel id kd_tiles): 2 keeps the particles in paint-bin order
 * in the workspace from the call's first step to its last: the first step reads the state
 * arrays, the last writes them back, and each drift counts the particles into the next
 * step's bins. The force is then formed per 8^3 tile inside the kick-drift (the rays read
 * their lens planes, formed from phi, as always), so after such a call no G mesh is kept
 * (hrt_mesh_ptr(HRT_MESH_GRAD) returns HRT_ESTATE; phi of the last step is there, and a
 * ray_step of that step may follow). 3 is 2 with the tile kick-drift run as a
 * persistent, software-pipelined grid (each workgroup loads its next tile while it moves
 * the current one). 4 is 2 with one kick-drift workgroup per x-pair of tiles (one phi
 * block of 24 x 13 x 13 for both; FP32 only, FP64 runs 2). 5 (FP32; FP64 runs 2) is 4
 * without re-binning the whole state every step: a particle that stays in its paint bin
 * keeps its slot, one that leaves it leaves a hole and joins a side list sorted by bin,
 * which the paint and the kick-drift read beside the bins; the whole state is re-binned only
 * at the end of a step that starts with more than P/16 listed particles. 6 is 5 with a limit
 * of P/64. 7 is 5 with G formed per particle from the pair's phi block (no G block; 256 lanes
 * per pair), faster when particles are sparse (np <= n/2). 1 runs pm_step's Lagrangian-order
 * kernels (with the same fused counting). 0 (default) takes, for calls of 8 steps or more,
 * 5 in FP32 (7 when every realisation has np <= n/2) and 2 in FP64, and 1 otherwise. Either way the state arrays must not be modified by anyone else while the
 * call's work runs. */
int hrt_run(hrt_ctx *ctx, const hrt_matter *m, const hrt_rays *r, int first_step, int n_steps,
            const hrt_maps *maps);

/* Captures steps first_step .. first_step+n_steps-1 (pm_step then ray_step for every
 * realisation, as hrt_run does, with the same source-plane maps; with HRT_STATIC one
 * pm_force then ray_steps; r may be NULL for matter only) into a HIP graph held by the
 * context, replacing any previous one. Nothing runs during capture; hrt_graph_launch
 * replays the whole sequence with one launch on the context's stream. The state arrays,
 * map arrays and workspace must stay the same between capture and replays. Profiling must
 * be off while capturing. */
int hrt_graph_capture(hrt_ctx *ctx, const hrt_matter *m, const hrt_rays *r, int first_step,
                      int n_steps, const hrt_maps *maps);
int hrt_graph_launch(hrt_ctx *ctx);

/* Device pointer to an internal mesh of realisation `realisation`, valid until
 * hrt_destroy: HRT_MESH_DELTA (n^3, after pm_force: delta), HRT_MESH_PHI (n^3: phi),
 * HRT_MESH_GRAD (n^3 interleaved quadruples (G_x, G_y, G_z, 0); HRT_ESTATE after an hrt_run
 * in paint-bin order, which forms G per tile and keeps no G mesh, until the next
 * pm_force / pm_step). HRT_MESH_LIST_CTL: the control words of the mover-list run (kd_tiles
 * variants 0, 5 and 6 in FP32), two records of 8 uint32 (one per step parity: record buffer
 * holding the bins' fronts, side-list entries, holes, 0, re-binnings so far in the call,
 * re-binning limit, 2 unused), for tests and statistics; HRT_EINVAL for FP64 and static
 * contexts, which have none. */
enum { HRT_MESH_DELTA = 0, HRT_MESH_PHI = 1, HRT_MESH_GRAD = 2, HRT_MESH_LIST_CTL = 3 };
int hrt_mesh_ptr(const hrt_ctx *ctx, int realisation, int which, void **ptr);

/* Host-only step tables for cfg (no GPU use), for checking the table builder.
 * Sizes: a, chi, K, D, d: N+1 doubles each; plane_begin, plane_count: N+1 ints;
 * plane_mesh (int), plane_chi, plane_w (double): up to max_planes entries.
 * *n_planes receives the total number of shell-plane entries; HRT_ENOMEM if it
 * exceeds max_planes (then only *n_planes is written). Any array may be NULL. */
int hrt_tables(const hrt_config *cfg, double *a, double *chi, double *K, double *D,
               double *d, int32_t *plane_begin, int32_t *plane_count, int32_t *plane_mesh,
               double *plane_chi, double *plane_w, int32_t max_planes, int32_t *n_planes);

/* Initial conditions (support for the cosmological runs; the paper starts from 2LPT at
 * a = 1/64, Sec. 6.2, without giving the recipe). Linear spectrum at a = 1:
 * P(k) = A k^n_s T(k)^2 with the Eisenstein & Hu (1998) no-wiggle transfer function and A
 * fixed by sigma8 (top-hat of 8 Mpc/h); field on the particle lattice
 * delta_k = FFT(noise)_k sqrt(P(k) / (box/np)^3) (k = 0 removed); second-order Lagrangian
 * displacement s = D1 s1 + D2 s2 with s1 = -grad phi1, grad^2 phi1 = delta,
 * s2 = grad phi2, grad^2 phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij^2), growth factors from
 * the growth ODEs normalised to D1(1) = 1, and p = a^2 E(a) (f1 D1 s1 + f2 D2 s2). */
typedef struct {
    double omega_b;         /* baryon density parameter (transfer-function shape only) */
    double h;               /* H0 / (100 km/s/Mpc)                                      */
    double n_s;             /* primordial spectral index                                */
    double sigma8;          /* rms linear density contrast in 8 Mpc/h spheres at a = 1  */
    double t_cmb;           /* CMB temperature [K]                                      */
    double a;               /* scale factor of the returned state, 0 < a <= 1           */
} hrt_ic_params;

/* Writes the 2LPT state of realisation `realisation` at scale factor ic->a into out (all
 * six arrays) from the unit white noise `noise` (device, np^3 values of the config's
 * dtype, layout [z][y][x]). Uses that realisation's workspace as scratch (it overwrites
 * the force mesh). Needs 16 <= np. */
int hrt_ic_2lpt(hrt_ctx *ctx, int realisation, const void *noise, const hrt_ic_params *ic,
                const hrt_matter *out);

/* Host-only: out[0..5] = amplitude A, D1(a), f1(a), D2(a), f2(a), D1(1) (growth factors
 * with D1 -> a deep in matter domination) for cfg and ic. */
int hrt_ic_factors(const hrt_config *cfg, const hrt_ic_params *ic, double *out);

/* Reverse mode (vector-Jacobian products). The paper names gradients through the ray
 * tracer as future work (Sec. 7, via the adjoint method of its ref. LiEtAl2024); these are
 * the exact transposes of the forward discretisation above. A cotangent array has the
 * shape, layout and dtype of the state array it belongs to; the functions update the
 * cotangents in place (device, caller-owned). m, r, mc, rc point to n_cfg entries (batched
 * contexts are supported; their realisations are processed one after another). All of them
 * need a context created with HRT_ADJOINT (else HRT_ESTATE), recompute the force mesh of
 * the step from m (so they overwrite it: the next ray_step needs a new pm_force/pm_step),
 * and sum the force-mesh cotangent in 64-bit fixed point, so results are deterministic.
 *
 * hrt_step_vjp: the whole co-evolution step (pm_step then ray_step). m (s; p may be NULL)
 * and r (dth; p may be NULL) are the state BEFORE step `step`; on entry mc and rc hold the
 * cotangents of the state AFTER the step, on return those of the state before it. It runs
 * the transposed ray kick-drift and the transposed matter kick-drift, and the transposed
 * force (fourth-order difference, Poisson solve, CIC paint) once on the summed cotangent of
 * the force mesh. r and rc are both NULL for matter only; with HRT_STATIC the matter does
 * not move, mc->p may be NULL and mc->s receives the lens-position cotangent.
 *
 * pm_step_vjp and ray_step_vjp are the same step split along the contract's two forward
 * calls: pm_step_vjp is the transpose of pm_step (mc after -> before; not valid with
 * HRT_STATIC), ray_step_vjp that of ray_step: rc after -> before, and the rays' dependence
 * on the matter through the force mesh added to mc->s (mc->p untouched, may be NULL).
 * Applying pm_step_vjp and then ray_step_vjp to the same cotangents gives hrt_step_vjp's
 * result up to rounding (the force's transpose then runs twice, on each part of the
 * force-mesh cotangent; hrt_step_vjp sums them first and is the cheaper call). */
int hrt_step_vjp(hrt_ctx *ctx, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                 const hrt_rays *rc, int step);

/* Reverse mode without forming the force a second time, for callers that recompute a
 * checkpoint segment forward (pm_step of each step but the last, then the VJPs of the
 * segment's steps in reverse). hrt_force_save copies the force the last pm_step / pm_force
 * formed (the G mesh and the paint-bin offsets of every realisation) into slot `slot`
 * (0 <= slot < k of HRT_FORCE_SLOTS(k): HRT_EINVAL otherwise, or HRT_ESTATE for a context
 * without slots) and records its step; HRT_ESTATE if there is no current force (none formed
 * yet, or a paint-bin-order hrt_run, which keeps no G mesh). hrt_step_vjp_saved is
 * hrt_step_vjp with the force copied back from slot `slot`, which must hold the force of
 * `step` (HRT_ESTATE otherwise), instead of painted and solved again; m must be the state
 * that force was formed from (not checked: the caller keeps the two together). Given that,
 * its results equal hrt_step_vjp's bit for bit. A slot keeps its content until the next
 * hrt_force_save to it; saving and the VJP overwrite the context's force meshes only. */
int hrt_force_save(hrt_ctx *ctx, int slot);
int hrt_step_vjp_saved(hrt_ctx *ctx, int slot, const hrt_matter *m, const hrt_rays *r,
                       const hrt_matter *mc, const hrt_rays *rc, int step);
int pm_step_vjp(hrt_ctx *ctx, const hrt_matter *m, const hrt_matter *mc, int step);
int ray_step_vjp(hrt_ctx *ctx, const hrt_matter *m, const hrt_rays *r, const hrt_matter *mc,
                 const hrt_rays *rc, int step);

/* Adds the cotangent of the deflections from kappa_bar (n_cfg device pointers to Mx*My
 * values: the cotangent of ray_convergence's kappa) to rc[k].dth (rc[k].p may be NULL). */
int ray_convergence_vjp(hrt_ctx *ctx, void *const *kappa_bar, const hrt_rays *rc);

/* Cotangent of the white noise of hrt_ic_2lpt: from the cotangents cot->s, cot->p of the
 * 2LPT state (read only) writes noise_bar (np^3 values, layout of the noise; it must not
 * alias noise or any cotangent array: it serves as scratch before the result is written;
 * HRT_EINVAL if it is one of them). Uses the realisation's workspace as scratch (it
 * overwrites the force mesh). */
int hrt_ic_2lpt_vjp(hrt_ctx *ctx, int realisation, const void *noise, const hrt_ic_params *ic,
                    const hrt_matter *cot, void *noise_bar);

/* Launch-shape variants. Some kernels can map particles or rays onto workgroups in several
 * ways (Lagrangian patches of different shapes, linear order, pixel patches or rows) and
 * group workgroups per XCD or not; every variant computes bit-identical results and they
 * differ only in speed (matter_kd also has shapes with two particles per lane, paint_tiles
 * shapes that paint two or four tiles per workgroup or spread the FP32 sums over two to
 * eight LDS copies). Tunable kernel ids: bin_count, bin_scatter
 * (8 variants each), ray_step (6), matter_kd (16), paint_tiles (14), kd_tiles (8: the particle order of hrt_run, see
 * there, 3 and 4 being the paint-bin order with a persistent pipelined kick-drift and with
 * x-pairs of tiles per workgroup; not chosen by hrt_autotune). hrt_num_variants(id) gives the count (1 = not
 * tunable, 0 = no such id); hrt_set_variant forces a choice (HRT_EINVAL out of range);
 * hrt_get_variant reads it. A new context starts with variant 0 everywhere. */
int hrt_num_variants(int kernel_id);
int hrt_set_variant(hrt_ctx *ctx, int kernel_id, int variant);
int hrt_get_variant(const hrt_ctx *ctx, int kernel_id, int *variant);

/* Autotuner: runs pm_force(m, step), then times every variant of each tunable kernel on
 * this context's sizes (a warm-up and 5 launches each, HIP events on the context's stream;
 * synchronises the host) and keeps the fastest. With cache_path (may be NULL) the choices
 * are kept in that JSON file under a key made of the device architecture, kernel name,
 * dtype and every realisation's sizes: keys already in the file are applied without
 * timing, new ones are added (the file is rewritten through a temporary and a rename).
 * m (all six arrays) and r (may be NULL: the ray kernel is then not tuned) are scratch:
 * the timed launches advance them, so pass copies of a representative state. Not valid
 * with HRT_STATIC. Overwrites the force mesh. */
int hrt_autotune(hrt_ctx *ctx, const hrt_matter *m, const hrt_rays *r, int step,
                 const char *cache_path);

/* Optional per-kernel timing with HIP events recorded on the context's stream around
 * every kernel launch (for measurement; off by default). hrt_profile_enable(ctx, 1)
 * clears the totals and starts recording, 0 stops. hrt_profile_read synchronises the
 * stream and writes, for kernel ids 0..n-1, the summed milliseconds and launch counts.
 * hrt_kernel_name(id) names kernel id (NULL past the last id, HRT_NUM_KERNELS). */
enum { HRT_NUM_KERNELS = 19 };
int hrt_profile_enable(hrt_ctx *ctx, int on);
int hrt_profile_read(hrt_ctx *ctx, double *total_ms, int64_t *launches, int n);
const char *hrt_kernel_name(int id);

#ifdef __cplusplus
}
#endif

#endif /* HRT_H */
