/*
 * mprk.h -- C ABI of the MI355X (gfx950) multirate partitioned Runge-Kutta
 * (MPRK) library for two vertically stacked compressible Navier-Stokes
 * domains coupled through a rigid lid.
 *
 * Paper: Kang et al., "Multirate partitioned Runge-Kutta methods for coupled
 * Navier-Stokes equations" (arXiv 2202.11890).
 *
 * What it computes
 *   The coupled semi-discrete system of Section 3, eq.
 *   (semi-discretized-coupled-model): dq^F/dt = R^F(q^F, q^B),
 *   dq^B/dt = R^B(q^B, q^F, q^S), dq^S/dt = R^S(q^S, q^B), where F is the
 *   fast domain, B the n_buffer slow rows next to the interface Gamma and S
 *   the remaining slow rows.  R is the cell-centred second-order finite-volume
 *   RHS of Section 2.1 and Appendix B (local Lax-Friedrichs inviscid flux with
 *   a Roe-average wave speed, common-value viscous flux, bulk-coefficient
 *   coupling at Gamma, eq. bulk-flux), in the x-z plane (dim 2) or in three
 *   dimensions (dim 3, Appendix B as printed: x and y periodic).
 *   Time integration is the MPRK method of eq. (MRK2) with the stage
 *   schedule of Algorithm 1: the fast domain takes m substeps of dt/m, the
 *   buffer restarts from q^B_n at each substep with the full step and is
 *   averaged, the slow region takes one base step whose s stage values are
 *   reused at every substep.
 *
 * Data layout (device memory, caller-owned)
 *   dim 2: q_lower, q_upper are float64 [4][nz][nx], x fastest, row 0 at the
 *   bottom, components (rho, rho u, rho w, rho E).
 *   dim 3: float64 [5][nz][ny][nx], components (rho, rho u, rho v, rho w,
 *   rho E), x fastest, then y, then z (plane 0 at the bottom).
 *   Nondimensional (Appendix A).  Gamma lies between the top row (plane) of
 *   q_lower and the bottom one of q_upper.  x (and y) are periodic; the bottom
 *   of the lower domain and the top of the upper domain are slip adiabatic
 *   walls.
 *
 * Ownership and threading
 *   State, workspace and stream belong to the caller; the library never calls
 *   hipMalloc or hipFree.  Its device footprint is exactly the two state
 *   arrays plus mprk_workspace_bytes().  mprk_step and mprk_run update the
 *   state in place, asynchronously on the context's stream.  A context is not
 *   thread-safe; calls on one context must not overlap.
 *
 * Errors
 *   Every function returns MPRK_OK (0) or a negative mprk_status; nothing
 *   throws across the ABI.  Kernel launches are asynchronous: a state that
 *   becomes non-finite or non-physical is reported at the next check
 *   (mprk_run's check points, mprk_diagnostics) as MPRK_ENONFINITE.
 */
#ifndef MPRK_H
#define MPRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPRK_ABI_VERSION 2

enum mprk_status {
    MPRK_OK = 0,
    MPRK_EINVAL = -1,       /* invalid configuration or argument                    */
    MPRK_EBUFFER = -2,      /* n_buffer < 2s-1 while strict_buffer is set           */
    MPRK_EWORKSPACE = -3,   /* workspace missing, too small or not 256-B aligned     */
    MPRK_EHIP = -4,         /* a HIP runtime call or kernel launch failed            */
    MPRK_ENONFINITE = -5,   /* non-finite value, rho <= 0 or p <= 0 detected         */
    MPRK_EUNSUPPORTED = -6, /* valid request the library or device does not support  */
    MPRK_ETIMEOUT = -7      /* persistent execution: a tile waited over its time limit
                               for a neighbour (the run was aborted; the state is not
                               a completed step)                                      */
};

/* How mprk_step / mprk_run (and mprk_batch_run) execute a slow step. */
enum mprk_exec {
    MPRK_EXEC_LAUNCH = 0,     /* one kernel launch per stage (m*s per slow step)        */
    MPRK_EXEC_PERSISTENT = 1, /* one cooperative launch per run segment: workgroups stay
                                 resident and start a tile's next stage as soon as the
                                 tiles it reads have finished the previous one           */
    MPRK_EXEC_GRAPH = 2       /* the stage launches of one slow step recorded once as a
                                 HIP graph and replayed per step (rebuilt when dt or the
                                 tile shape changes)                                     */
};

/* Tile shapes of the stage kernel (columns x rows of cells per workgroup).
 * Results do not depend on the shape: every face is evaluated by the same
 * operations whichever tile holds it. */
enum mprk_tile {
    MPRK_TILE_32X16 = 0,      /* default (2D with either flux precision, and 3D) */
    MPRK_TILE_16X32 = 1,
    MPRK_TILE_64X8 = 2,
    MPRK_TILE_32X8 = 3,
    MPRK_TILE_SHAPES = 4
};

/* Regions of eq. (semi-discretized-coupled-model), as bits. */
enum mprk_region {
    MPRK_REGION_F = 1,
    MPRK_REGION_B = 2,
    MPRK_REGION_S = 4,
    MPRK_REGION_ALL = 7
};

typedef struct mprk_config {
    int32_t abi_version;    /* must be MPRK_ABI_VERSION                              */
    int32_t dim;            /* 2 (x-z plane) or 3 (x-y-z)                            */
    int32_t nx, ny;         /* cells in x and y (periodic); nx >= 4; ny must be 1 when
                               dim == 2, >= 4 when dim == 3                           */
    int32_t nz_lower;       /* rows of the lower domain (>= 3)                       */
    int32_t nz_upper;       /* rows of the upper domain (>= 3); a domain holds at most
                               2^28 cells (nx * ny * nz)                              */
    double dx, dy;          /* cell sizes in x (and y); dy is ignored in 2D          */
    double dz_lower;        /* cell height of the lower domain                       */
    double dz_upper;        /* cell height of the upper domain                       */
    int32_t fast_is_lower;  /* 1: the lower domain is F; 0: the upper domain is F    */
    int32_t n_buffer;       /* slow rows next to Gamma forming B, 1..nz_slow-2       */
    int32_t base_rk;        /* 2: two-stage RK2 of Table 1; 3: three-stage SSP-RK3   */
    int32_t m;              /* rate ratio 1..64; m == 1 is the single-rate base method */
    double gamma;           /* ratio of specific heats (> 1)                         */
    double prandtl;         /* Prandtl number (> 0)                                  */
    double mu_lower;        /* nondimensional viscosity of the lower domain (> 0)    */
    double mu_upper;        /* nondimensional viscosity of the upper domain (> 0)    */
    double gravity;         /* signed vertical gravity; source (0, 0, rho g, rho w g) */
    int32_t flux_bits;      /* 64: FP64 throughout; 32: face fluxes in FP32 (state,
                               stage sums, flux differences and the interface flux
                               stay FP64, so conservation is unchanged)              */
    int32_t strict_buffer;  /* 1: reject n_buffer < 2s-1 with MPRK_EBUFFER           */
} mprk_config;

typedef struct mprk_stats {
    double totals_lower[5]; /* sum of q |K| per component, lower domain (Sec. 5.1);
                               2D: (rho, rho u, rho w, rho E, 0)                      */
    double totals_upper[5]; /* same, upper domain                                     */
    double lambda_lower;    /* max over cells of sum_d (|u_d| + a) / d_d              */
    double lambda_upper;
    double courant_lower;   /* max over cells and directions of (|u_d| + a) / d_d     */
    double courant_upper;   /* (dt times this is the paper's Courant number)          */
    double visc_lower;      /* max over cells of max(4/3, gamma/Pr) mu/rho sum 1/d_d^2 */
    double visc_upper;
    int64_t steps_done;     /* slow steps taken by this context                        */
    int32_t status;         /* 0: state physical; 1: non-finite / rho<=0 / p<=0 seen   */
    int32_t reserved;
} mprk_stats;

typedef struct mprk_ctx mprk_ctx;

/* Check a configuration on the host; no GPU needed.  Writes a NUL-terminated
 * reason into msg (if msg != NULL and len > 0).  Returns MPRK_OK, MPRK_EINVAL,
 * MPRK_EBUFFER (only with strict_buffer) or MPRK_EUNSUPPORTED.  A buffer
 * shorter than 2s-1 rows is accepted without strict_buffer: the method then
 * runs, but is not exactly conservative (Section 3, Remark 1). */
int mprk_validate(const mprk_config* cfg, char* msg, size_t len);

/* Device workspace bytes a context needs for cfg (0 if cfg is invalid).
 * Host-only.  The workspace holds what one slow step of eq. (MRK2) keeps
 * besides the state (Algorithm 1): the stage values of the base method
 * (s-1 per domain, low-storage), the slow stage values that Algorithm 1
 * copies to later stages (only the rows the buffer's stencil reads), the
 * buffer's accumulated increments, and the reduction partials. */
size_t mprk_workspace_bytes(const mprk_config* cfg);

/* Create a context bound to caller-owned device memory: one instance of the
 * coupled problem of Section 3, eq. (semi-discretized-coupled-model), with
 * its partition into F, B and S (the index sets of the regions, Section 4)
 * fixed by cfg (fast_is_lower, n_buffer) and the MPRK tableaux of eq. (MRK2)
 * built from (base_rk, m) (Table 1 for base_rk = 2, m = 2).
 *   q_lower, q_upper : device state arrays (layout above), updated in place
 *                      by mprk_step / mprk_run.
 *   workspace        : device memory of at least mprk_workspace_bytes(cfg)
 *                      bytes, 256-byte aligned, owned by the caller and not
 *                      touched by anyone else while the context lives.
 *   hip_stream       : hipStream_t to launch on (NULL: the null stream).
 * On success *out receives the context (host memory owned by the library,
 * released by mprk_destroy). */
int mprk_create(const mprk_config* cfg, double* q_lower, double* q_upper, void* workspace,
                size_t workspace_bytes, void* hip_stream, mprk_ctx** out);

/* Change the stream later launches go to. */
int mprk_set_stream(mprk_ctx* ctx, void* hip_stream);

/* One evaluation of the coupled RHS f(q) of eq. (semi-discretized-coupled-
 * model) at the given device state (which need not be the context's state),
 * written to r_lower / r_upper (same layout) on the rows of the regions in
 * region_mask; other rows of r are not written.  Asynchronous. */
int mprk_rhs(mprk_ctx* ctx, const double* q_lower, const double* q_upper, double* r_lower,
             double* r_upper, int region_mask);

/* One slow step of size dt (eq. MRK2, Algorithm 1): m*s stage launches on the
 * context's stream; the state is updated in place.  Asynchronous. */
int mprk_step(mprk_ctx* ctx, double dt);

/* nsteps slow steps of size dt (eq. MRK2 with the stage schedule of
 * Algorithm 1, repeated).  Every check_every steps (and after the last
 * one) runs the device reductions (the totals of Section 5.1, which are
 * conserved when the buffer is long enough, Remark 1) and synchronises the
 * stream; returns
 * MPRK_ENONFINITE at the first check that sees a bad state.  check_every <= 0
 * checks only after the last step.  nsteps == 0 leaves the state alone and
 * only runs the reductions; nsteps < 0, or nsteps > 0 with a dt that is not
 * positive and finite, returns MPRK_EINVAL without touching the state.  If
 * out != NULL it receives the stats of the last check. */
int mprk_run(mprk_ctx* ctx, double dt, int64_t nsteps, int64_t check_every, mprk_stats* out);

/* Device reductions on the context's current state (totals, stability
 * measures, status); synchronises the stream.  Returns MPRK_ENONFINITE if the
 * state is bad (out is still filled). */
int mprk_diagnostics(mprk_ctx* ctx, mprk_stats* out);

/* Allocation-free variant of mprk_diagnostics, for callers that cannot
 * allocate device memory or create a context (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  Runs the same
 * device reductions (the same kernels, so the same bits as mprk_diagnostics)
 * on the given device states q_lower / q_upper (layout as above, dim 2 or 3)
 * for the configuration cfg (checked as by mprk_validate), on hip_stream
 * (NULL: the null stream), and synchronises that stream.  out (optional)
 * receives the stats; steps_done is 0.  Returns MPRK_ENONFINITE for a bad
 * state (out is still filled), MPRK_EINVAL / MPRK_EBUFFER /
 * MPRK_EUNSUPPORTED for a configuration mprk_validate rejects, MPRK_EHIP on
 * a HIP error.
 * Scratch: the reduction partials live in a file-scope device array of the
 * library, 57,568 bytes per device (2 domains x 256 partial blocks x 14
 * fields, then 2 x 14 final fields, FP64), held by every device the library
 * runs on until the process ends.  The need does not depend on the problem
 * size: any size mprk_validate accepts fits.  The call allocates nothing
 * (no hipMalloc, no workspace, no context).  Every call on one device shares
 * that device's array: calls that overlap on one device (two host threads,
 * or two streams without ordering between them) race and give wrong stats;
 * callers must serialise them. */
int mprk_diagnostics_static(const mprk_config* cfg, const double* q_lower, const double* q_upper,
                            void* hip_stream, mprk_stats* out);

/* Stable slow step from stats (host-only).  Per domain the step limit is
 * 1 / (lambda/cr + visc/dn) (advective and diffusive limits combined); the
 * slow step is min(m * fast-domain limit, slow-domain limit).  Returns
 * MPRK_ENONFINITE if st->status is set, MPRK_EINVAL for non-positive cr, dn
 * or wave speeds. */
int mprk_stable_dt(const mprk_config* cfg, const mprk_stats* st, double cr, double dn,
                   double* dt_out);

/* Select the execution of later mprk_step / mprk_run calls (default
 * MPRK_EXEC_LAUNCH).  Both give bit-identical results: every cell is
 * computed by the same code from the same inputs.  The persistent mode needs
 * cooperative launch support (else mprk_run returns MPRK_EUNSUPPORTED).  Each
 * persistent launch (one run segment between check points) is bounded in
 * time: a tile that is still waiting for a neighbour once the launch has run
 * longer than the limit of mprk_set_wait_limit aborts it, every workgroup
 * then exits, and the run returns MPRK_ETIMEOUT.  Kernel timing (mprk_profile_*) covers the launch mode only.  3D
 * contexts support MPRK_EXEC_LAUNCH and MPRK_EXEC_GRAPH (MPRK_EXEC_PERSISTENT:
 * MPRK_EUNSUPPORTED). */
int mprk_set_exec(mprk_ctx* ctx, int mode);

/* Longest time (seconds, default 10) one persistent launch may run, counted
 * from its start: a tile still waiting for a neighbour after that aborts the
 * run with MPRK_ETIMEOUT (the state is then not a completed step).  The bound
 * is on the launch, not on each wait, so a launch ends within the limit plus
 * one tile's work.  0 aborts at the first wait that is not already met. */
int mprk_set_wait_limit(mprk_ctx* ctx, double seconds);

/* Tile shape of later launches (an mprk_tile value; default MPRK_TILE_32X16).
 * Results are bit-identical for every shape.  3D contexts have one tile shape
 * per flux precision, selected by MPRK_TILE_32X16 (other values:
 * MPRK_EUNSUPPORTED). */
int mprk_set_tile(mprk_ctx* ctx, int shape);

/* Kernel timing aid.  While enabled, every stage launch is bracketed by a
 * pair of HIP events recorded on the context's stream (host-side event
 * objects only; no device allocation).  mprk_profile_take waits for the
 * recorded events and returns the summed stage-kernel time in milliseconds
 * and the number of launches since the previous take (or since enabling).
 * Disabling drops unread timings. */
int mprk_profile_enable(mprk_ctx* ctx, int on);
int mprk_profile_take(mprk_ctx* ctx, double* kernel_ms, int64_t* launches);

/* Release the context created by mprk_create (host memory only; not the
 * caller's state, workspace or stream).  Synchronises its stream first, so
 * the state holds the last completed step of eq. (MRK2).  NULL:
 * MPRK_EINVAL. */
int mprk_destroy(mprk_ctx* ctx);

/* Static description of a status code. */
const char* mprk_strerror(int code);

/* ---- Batches of independent problems ----------------------------------------
 * Many coupled two-domain problems ("members": ensembles, served requests),
 * each with its own sizes, parameters, rate ratio m, base method and step,
 * advanced together: every launch covers the tiles of all members that have
 * a stage in it.  A slow step is a fixed number of launches L (the largest
 * m*s of the batch); member i's stage p (0-based within its slow step) runs
 * in launch floor(p * L / (m_i s_i)), so every member's stages are spread
 * evenly over the step and members with small m do not leave launches
 * empty.  A member's arithmetic is exactly that of a single context with the
 * same configuration and step: results are bit-identical whatever else is in
 * the batch, and in every execution mode and tile shape.
 * Members are 2D problems (dim 3: MPRK_EUNSUPPORTED) and must share
 * flux_bits.  States are caller-owned device arrays
 * (layout as above) that must not overlap. */
typedef struct mprk_member {
    mprk_config cfg;
    double* q_lower;        /* device state, updated in place                     */
    double* q_upper;
    double dt;              /* slow step of this member (> 0)                      */
} mprk_member;

typedef struct mprk_batch mprk_batch;

/* Host-only check of every member (as mprk_validate) and of the batch rules
 * (1..4096 members, one flux_bits, dt > 0).  msg as in mprk_validate. */
int mprk_batch_validate(const mprk_member* members, int32_t n, char* msg, size_t len);

/* Device workspace bytes of a batch (0 if invalid): the members' scratch
 * plus the launch tables.  Host-only. */
size_t mprk_batch_workspace_bytes(const mprk_member* members, int32_t n);

/* Create a batch over caller-owned states and workspace (256-byte aligned,
 * at least mprk_batch_workspace_bytes).  The member array is copied; the
 * states must stay valid while the batch lives.  MPRK_EINVAL if states
 * overlap. */
int mprk_batch_create(const mprk_member* members, int32_t n, void* workspace, size_t workspace_bytes,
                      void* hip_stream, mprk_batch** out);

/* Execution mode (mprk_exec) and tile shape (mprk_tile; default as for a
 * context of the members' flux precision) of later runs. */
int mprk_batch_set_exec(mprk_batch* batch, int mode);
int mprk_batch_set_tile(mprk_batch* batch, int shape);
int mprk_batch_set_wait_limit(mprk_batch* batch, double seconds);

/* Change member's slow step (e.g. after mprk_batch_diagnostics and
 * mprk_stable_dt); takes effect at the next run. */
int mprk_batch_set_dt(mprk_batch* batch, int32_t member, double dt);

/* Tile-shape autotuner.  For each shape, times reps repetitions (after one
 * warm-up) of a slow step's launches with every stage replaced by an RHS
 * evaluation of the same tiles into the stage scratch (the states are not
 * modified), with HIP events on the batch's stream; selects the fastest
 * shape for later runs.  ms_out (optional, MPRK_TILE_SHAPES entries) receives
 * milliseconds per slow step, *best (optional) the chosen shape.
 * Synchronises the stream. */
int mprk_batch_tune(mprk_batch* batch, int32_t reps, double* ms_out, int32_t* best);

/* nsteps slow steps of every member, in place.  Every check_every steps (and
 * after the last) runs each member's reductions and synchronises; out (n
 * entries, optional) receives per-member stats of the last check.  Returns
 * MPRK_ENONFINITE if any member's state is bad (the others still advance
 * to the check point). */
int mprk_batch_run(mprk_batch* batch, int64_t nsteps, int64_t check_every, mprk_stats* out);

/* Adaptive steps: when cr > 0, at every check point of mprk_batch_run each
 * member's slow step is reset to mprk_stable_dt(cfg, its stats, cr, dn) of
 * its current state (the rule of the initial step, tracking states that
 * change, e.g. slow cells heated through the interface).  cr = 0 (the
 * default) keeps the steps fixed.  A member's step sequence depends only on
 * its own state. */
int mprk_batch_set_adaptive(mprk_batch* batch, double cr, double dn);

/* Current slow step of a member. */
int mprk_batch_get_dt(mprk_batch* batch, int32_t member, double* dt);

/* Per-member reductions on the current states (n entries); synchronises. */
int mprk_batch_diagnostics(mprk_batch* batch, mprk_stats* out);

/* Release the batch (not the caller's memory).  Synchronises its stream. */
int mprk_batch_destroy(mprk_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* MPRK_H */
