/*
 * lbm.h - C ABI of the MI355X (gfx950) implementation of the
 * interpolation-free, state-adaptive compressible lattice Boltzmann step of
 * Coreixas & Latt, "Compressible lattice Boltzmann methods with adaptive
 * velocity stencils: An interpolation-free formulation" (arXiv 2009.13426).
 *
 * One time step (Sec. IV.A.4, algorithm overview), per node x:
 *   - pull the 2 x 21 post-collision populations h*_i(x - c_i), c_i = xi_i + U(x)
 *     (eq. stream); where the source node's populations live in another
 *     lattice, rebuild them by Grad's ansatz in the receiver's lattice
 *     (eqs. GradGeneral, GradGeneral_f, GradGeneral_g);
 *   - moments rho, u, polyatomic T (eq. polyTemp);
 *   - lattice shift for the next pull from the local velocity (eq. criterion);
 *   - 8-constraint numerical equilibrium by Newton iteration on its Lagrange
 *     multipliers (eqs. feqNum_8Mom, G0_8mom-G3yaa_8mom), g_eq (eq. gEq);
 *   - optional Knudsen-number sensor on the relaxation time (eq. DeltaAvg);
 *   - BGK collision (eq. coll), tau = 1/2 + nu / T (App. E).
 *
 * Conventions
 *   Grid nx x ny, periodic in x and y, node n = y * nx + x.  Field arrays are
 *   float64 [ny][nx].  Unless stated otherwise pointers are DEVICE pointers
 *   (memory on the GPU the context runs on); the library borrows them for the
 *   duration of the call only.  Every call returns lbm_status; no C++
 *   exception crosses this boundary.  A context is not thread-safe; calls on
 *   one context are ordered on the HIP stream it was created with.
 *
 * Memory ownership
 *   The library never allocates device memory.  The caller allocates one
 *   device workspace of lbm_workspace_bytes(cfg) bytes and keeps it alive
 *   until lbm_destroy.  lbm_create/lbm_destroy allocate and free only the
 *   small host-side context.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_Q 21            /* velocities of D2Q21 (Sec. I, Fig. 1) */
#define LBM_HIST_BINS 32    /* Newton-iteration histogram bins */

typedef struct lbm_ctx lbm_ctx;

typedef enum {
  LBM_OK = 0,
  LBM_ERR_ARG = -1,          /* invalid argument or configuration */
  LBM_ERR_WORKSPACE = -2,    /* workspace missing, too small or misaligned; or, from a
                                step, the queue of links to rebuild (4 nx ny pairs of
                                source and lattice; 21 nx ny below 65536 nodes, which
                                cannot fill) overflowed */
  LBM_ERR_HIP = -3,          /* a HIP runtime call failed */
  LBM_ERR_STATE = -4,        /* call out of order (e.g. step before init) */
  LBM_ERR_NEWTON = -5,       /* an equilibrium solve did not converge */
  LBM_ERR_NONPHYSICAL = -6   /* rho <= 0, T <= 0, non-finite, or |U| > max_abs_shift */
} lbm_status;

typedef enum {
  LBM_FP64 = 0,              /* populations stored, streamed and collided in FP64 */
  LBM_FP32_STORE = 1         /* FP32 populations and collision; FP64 moments and Newton */
} lbm_precision;

typedef enum {
  LBM_SHIFT_ADAPTIVE = 0,    /* eq. (criterion), optional hysteresis half-width */
  LBM_SHIFT_FIXED = 1,       /* one lattice (fixed_ux, fixed_uy) everywhere */
  LBM_SHIFT_STATIC = 2,      /* per-node map given to lbm_init_fields_static */
  LBM_SHIFT_NEIGHBOURHOOD = 3 /* overlapping ranges of half-width shift_halfwidth (< 1);
                                 among the admissible shifts, the one most of the four
                                 nearest neighbours use (Sec. III.A.2), ties to the
                                 node's own, then to eq. (criterion).  8 constraints,
                                 default schedule, not in lbm_step_batched */
} lbm_shift_mode;

typedef struct {
  int32_t nx, ny;            /* grid; both >= 1, nx * ny * (8 or 4 bytes) < 2^32 */
  int32_t precision;         /* lbm_precision */
  double gamma;              /* heat capacity ratio; Cv = 1/(gamma-1), Cp = gamma Cv */
  double nu;                 /* kinematic viscosity >= 0 (lattice units) */
  int32_t shift_mode;        /* lbm_shift_mode */
  int32_t fixed_ux, fixed_uy;
  double shift_halfwidth;    /* >= 0.5; 0.5 reproduces eq. (criterion) exactly */
  double newton_tol;         /* max |G_a| per unit density; the paper uses 1e-12 */
  int32_t newton_max_iter;   /* iterations before LBM_ERR_NEWTON */
  int32_t max_abs_shift;     /* admissible |U_alpha|, 0..12 */
  int32_t sensor;            /* 1: tau scaled by alpha(eps_Kn), eq. (DeltaAvg) */
  int32_t collect_stats;     /* 1: keep Newton/mismatch counters (small cost) */
  int32_t constraints;       /* moment constraints of the numerical equilibrium:
                                8 = eq. (8moments) (default); 4 = mass, momentum and
                                energy only, eq. (feqNum_4Mom), Sec. "Reduced models"
                                (4 x 4 solve; runs the default schedule only);
                                13 = the paper's reference model (App. C, eqs.
                                (G0)-(G4yyaa)): the D2Q49 lattice {-3..3}^2 with all
                                moments up to third order and the contracted
                                fourth-order ones, 13 x 13 solve from the lattice
                                Maxwellian.  FP64 only, shift modes 0-2, default
                                schedule, not in lbm_step_batched */
  double prandtl;            /* Prandtl number nu / (thermal diffusivity): 1 (or 0) =
                                the BGK collision, eq. (coll); otherwise in [0.01, 1000)
                                the flexible-Prandtl collision of eq. (Shakhov), App. E:
                                BGK plus (1/tau - 1/tau_Pr) h_eq phi_S with q the heat
                                flux of the collided populations, tau_Pr = 1/2 +
                                (tau - 1/2)/Pr, phi_S the monatomic heat-flux shape
                                made free of mass, momentum and energy on the lattice
                                (the printed polyatomic shape carries momentum), and
                                kappa = rho Cp nu / Pr in the Grad rebuild.  8 or 13
                                constraints, no neighbourhood choice, default schedule,
                                not in lbm_step_batched */
  int32_t fallback;          /* 0 (default): a state whose 8-moment equilibrium has no
                                solution stops the run with LBM_ERR_NEWTON; 1: that
                                collision or rebuilt link takes the four-constraint
                                equilibrium of the same state instead, eq.
                                (feqNum_4Mom), solved from the lattice Maxwellian with
                                backtracking (the paper leaves the case open; it
                                arises at rebuilt links whose source moves at |u'| ~
                                1.6 in the receiver's lattice).  Counted in
                                lbm_diag.fallback_solves.  BGK only (prandtl 1);
                                without effect for 4 or 13 constraints */
} lbm_config;

typedef struct {
  int64_t steps_done;        /* steps completed since init */
  int32_t status;            /* first error seen on the device (lbm_status) */
  int32_t fail_step;         /* step index of that error, -1 if none */
  int64_t fail_node;         /* lowest failing node index of that step, -1 if none */
  int64_t newton_calls;      /* equilibrium solves (nodes + rebuilt links) */
  int64_t newton_iters;      /* Newton iterations over those solves */
  int64_t mismatched_links;  /* links rebuilt by Grad's ansatz */
  int64_t iter_hist[LBM_HIST_BINS];
  double conserved[4];       /* mass, x/y momentum, total energy of the current state */
  int64_t fallback_solves;   /* collisions and rebuilt links (each link counted) that
                                took the four-constraint equilibrium
                                (lbm_config.fallback), initial condition included */
} lbm_diag;

/* Launch schedule of a context's step loop.  Changing it changes how the
 * nodes are spread over workgroups, never what a node computes: results
 * are bitwise the same under every valid schedule. */
typedef struct {
  int32_t step_block;      /* lanes per workgroup of the step kernel: 64 or 128,
                            * or 256 in FP32 storage (default 64) */
  int32_t tiles_per_block; /* consecutive tiles of step_block nodes one workgroup
                            * runs one after the other, 1..64 (default 1) */
  int32_t xcd_remap;       /* 1: each XCD runs one contiguous range of tiles
                            * (default); 0: tiles in dispatch order */
  int32_t rebuild_blocks;  /* 256-lane workgroups of the link-rebuild launch,
                            * 1..65535; 0: one per 256 nodes, at most 4096 (default) */
} lbm_schedule;

/* Fills cfg with the defaults used by the paper's tests: gamma 1.4, nu 0,
 * adaptive shifts with half-width 0.5, Newton tolerance 1e-12 and 30
 * iterations, |U| <= 6, FP64, no sensor, no counters, 8 constraints,
 * Prandtl number 1, no fallback equilibrium. */
void lbm_default_config(lbm_config* cfg, int32_t nx, int32_t ny);

/* Device bytes the context needs for cfg (two population buffers, lattice
 * tags, the moments and rebuild queue carried between steps, diagnostics,
 * initial-guess table).  0 if cfg is invalid. */
size_t lbm_workspace_bytes(const lbm_config* cfg);

/* Creates a context on the current HIP device.  dev_workspace: device
 * pointer, 256-byte aligned, at least lbm_workspace_bytes(cfg) bytes, owned
 * by the caller and borrowed until lbm_destroy.  hip_stream: a hipStream_t
 * (NULL = default stream) on which every later call enqueues its work.
 * Builds the Newton initial-guess table on the device (synchronous). */
lbm_status lbm_create(const lbm_config* cfg, void* dev_workspace, size_t bytes,
                      void* hip_stream, lbm_ctx** out);

/* As lbm_create, but the initial-guess table is copied (device to device, on
 * the stream) from the existing context `like` on the same device instead of
 * being built (for callers that create many contexts, e.g. a job server);
 * built as by lbm_create if `like` has another constraint count.
 * `like` stays valid and unchanged; the copy is ordered on hip_stream. */
lbm_status lbm_create_like(const lbm_ctx* like, const lbm_config* cfg, void* dev_workspace,
                           size_t bytes, void* hip_stream, lbm_ctx** out);

/* Grad initial condition (Sec. IV.A.1, eq. GradGeneral): per node the lattice
 * is selected from u (or fixed), h(0) = h_eq (1 + phi_h) with central
 * differences of the input fields, then one collision gives the stored
 * post-collision state.  rho, ux, uy, T: device float64 [ny][nx].
 * Synchronous; returns the first error met. */
lbm_status lbm_init_fields(lbm_ctx* ctx, const double* rho, const double* ux,
                           const double* uy, const double* T);

/* As lbm_init_fields for shift_mode LBM_SHIFT_STATIC: Ux, Uy (device int8
 * [ny][nx]) give every node's lattice for the whole run (the paper's
 * 'static' Sod configuration, Sec. IV.C.1). */
lbm_status lbm_init_fields_static(lbm_ctx* ctx, const double* rho, const double* ux,
                                  const double* uy, const double* T,
                                  const int8_t* Ux, const int8_t* Uy);

/* Advances nsteps >= 0 steps, waits for them and checks the device error
 * flag.  On LBM_ERR_NEWTON / LBM_ERR_NONPHYSICAL, lbm_get_diag tells the
 * step and node; the state is then undefined until the next init. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Enqueues nsteps steps on the context's stream and returns without waiting
 * or checking; lbm_sync (or any synchronous call) reports errors later. */
lbm_status lbm_step_async(lbm_ctx* ctx, int32_t nsteps);

/* As lbm_step for nsteps >= 1, with HIP events recorded on the context's
 * stream around every launch.  ms_rebuild, ms_step (host pointers): summed
 * durations in milliseconds of the link-rebuild launches (0 when the
 * lattice is fixed) and of the step launches.  Synchronous; for measurement. */
lbm_status lbm_step_profiled(lbm_ctx* ctx, int32_t nsteps, double* ms_rebuild, double* ms_step);

/* Copies the whole state of src into dst (populations of the current
 * time level, lattice tags, the moments and rebuild lists carried to the
 * next step, steps done, diagnostics), device to device: a checkpoint or a
 * restore.  Both contexts must have the same configuration (every field of
 * lbm_config) and device, and src must be initialised; else LBM_ERR_ARG or
 * LBM_ERR_STATE.  Waits for src's stream, then copies on dst's stream and
 * waits for it.  The initial-guess table is not copied (each context has
 * its own, built or copied at creation).  dst's step graphs stay valid. */
lbm_status lbm_copy_state(lbm_ctx* dst, const lbm_ctx* src);

/* Sets the context's launch schedule (host struct, copied).  LBM_ERR_ARG
 * for a field out of range; the previous schedule then stays.  Drops the
 * context's step graphs (lbm_step_graph_async builds them again). */
lbm_status lbm_set_schedule(lbm_ctx* ctx, const lbm_schedule* sched);

/* The context's current schedule, with defaults resolved (rebuild_blocks is
 * never 0 in the result).  sched: host pointer. */
lbm_status lbm_get_schedule(const lbm_ctx* ctx, lbm_schedule* sched);

/* As lbm_step_async, but full chunks of `chunk` steps (even, 2..1024) run as
 * replays of a HIP graph holding the chunk's launches; the graph is built on
 * first use for the context's buffer parity and kept until the schedule
 * changes or the context is destroyed, and the remaining nsteps % chunk
 * steps are plain launches.  Same results, bitwise, as lbm_step_async; a
 * failure is reported with its true step.  The graph holds kernel nodes
 * only (no memset or copy nodes). */
lbm_status lbm_step_graph_async(lbm_ctx* ctx, int32_t nsteps, int32_t chunk);

/* Waits for the context's stream and returns the device error status. */
lbm_status lbm_sync(lbm_ctx* ctx);

/* Macroscopic fields of the current state (moments of the stored
 * populations in their lattice): device float64 rho, ux, uy, T [ny][nx] and
 * optionally (nullable) the lattice shift of every node, device int8.
 * Synchronous. */
lbm_status lbm_get_macros(lbm_ctx* ctx, double* rho, double* ux, double* uy,
                          double* T, int8_t* Ux, int8_t* Uy);

/* Post-collision populations as device float64 [Q][ny][nx] each, Q = 21
 * (or 49 with 13 constraints; FP32 storage is widened), in the velocity
 * order of lbm_lattice_velocities.  Synchronous. */
lbm_status lbm_get_populations(lbm_ctx* ctx, double* f, double* g);

/* Host arrays of 21 ints: the velocity set in storage order. */
void lbm_velocities(int32_t* cx, int32_t* cy);

/* The storage-order velocity set of a constraint count's lattice (Sec. I;
 * App. C for D2Q49: velocity k = (k mod 7 - 3, k div 7 - 3)) into host
 * arrays of up to 49 ints (nullable); returns the number of velocities, 21
 * or 49, or 0 for a constraint count the library does not build. */
int32_t lbm_lattice_velocities(int32_t constraints, int32_t* cx, int32_t* cy);

/* Counters, error record and conserved sums (computed on the device in a
 * fixed summation order).  out: host pointer.  Synchronous. */
lbm_status lbm_get_diag(lbm_ctx* ctx, lbm_diag* out);

/* Advances n <= 1024 distinct contexts that share one HIP stream, device,
 * precision and constraint count: ctxs[k] by nsteps[k] steps.  Per step one rebuild launch and
 * one step launch cover all contexts still running (the job table lives in
 * ctxs[0]'s workspace).  The step launch takes step_block and xcd_remap
 * from ctxs[0]'s schedule and runs one tile per workgroup; the rebuild
 * launch spreads every context's list over at most 4096 workgroups.
 * ctxs, nsteps: host arrays of n entries.
 * Synchronous; returns the first error (lbm_sync on each context tells
 * which). */
lbm_status lbm_step_batched(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n);

/* As lbm_step_batched (same arguments, results bit for bit, errors), with
 * the quantum's launches (per step the rebuild and the step launch) recorded
 * as a HIP graph of kernel nodes and replayed: form (2)'s step loop in a
 * graph.  The graph is kept by ctxs[0] and rebuilt only when the launch
 * shape changes (number of contexts, the largest nsteps, the contexts'
 * grid sizes or ctxs[0]'s schedule); the kernels read the job table at a
 * fixed address in ctxs[0]'s workspace, which is refreshed before every
 * replay.  graph_built (host pointer, nullable): 1 if this call recorded
 * the graph, 0 if it replayed the kept one. */
lbm_status lbm_step_batched_graph(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n,
                                  int32_t* graph_built);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): lbm_step_batched with
 * the same arguments, results and errors, except that the job table and the
 * failure words live in a library-owned device array of fixed size (up to
 * 1024 contexts, about 260 KB; every device the library runs on holds its
 * own copy until the process ends) instead of ctxs[0]'s workspace.  Calls
 * no hipMalloc, hipFree or other allocating routine.  The current device
 * must be the contexts' device (else LBM_ERR_ARG); n > 1024 gives
 * LBM_ERR_ARG.  All calls on one device share that array, so calls that
 * overlap on one device (other streams or threads) race; the host-side
 * staging is shared by the process, and calls are serialised on it. */
lbm_status lbm_step_batched_noalloc(lbm_ctx* const* ctxs, const int32_t* nsteps, int32_t n);

/* Copies `bytes` bytes from device buffer src to device buffer dst (16-byte
 * aligned, not overlapping) on hip_stream with the library's streaming copy
 * kernel (16-byte nontemporal loads and stores, several in flight per lane):
 * the practical HBM bandwidth that the step kernels' traffic is measured
 * against, beside the device's nominal peak.  Asynchronous; LBM_ERR_ARG for
 * null or misaligned pointers. */
lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

/* Frees the host context; the workspace stays the caller's. */
void lbm_destroy(lbm_ctx* ctx);

const char* lbm_status_str(lbm_status s);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
