/*
 * rrmhd.h -- C ABI of the MI355X (gfx950) library for one IMEX step of
 * relativistic radiation magnetohydrodynamics under the gray M1 closure with
 * the Jacobian-free PVM-int Riemann solver (Lopez-Miralles, Marti & Perucho,
 * "On the application of Jacobian-free Riemann solvers for relativistic
 * radiation magnetohydrodynamics under M1 closure", CPC, arXiv 2212.00370).
 *
 * Conventions for every entry point:
 *   - Array pointers marked "device" are HIP device pointers owned by the
 *     caller; the library never allocates, frees or retains device memory
 *     beyond the caller-provided workspace (see rrmhd_init).
 *   - State arrays are structure-of-arrays float64: variable q of cell c is at
 *     U[q * var_stride + c], cells numbered i + n0 * (j + n1 * k) (x fastest).
 *     Conserved order (Section 2.1, vector U):
 *       0 D, 1..3 S^j, 4 tau_e, 5..7 B^j, 8 E_r, 9..11 F_r^j
 *     Primitive order (Section 2.1, vector V):
 *       0 rho, 1..3 v^j, 4 p, 5..7 B^j, 8 E_r, 9..11 F_r^j
 *     Units: c = 1, 1/sqrt(4 pi) absorbed in B.
 *   - Work is enqueued on the stream given to rrmhd_init and the call returns
 *     without waiting, except where a call says it synchronizes. Argument and
 *     launch errors are returned directly; numerical failures (primitive
 *     recovery, implicit solve, non-finite values) are counted on the device
 *     and read with rrmhd_report_sync.
 *   - A context is used by one host thread at a time. Error strings are
 *     static.
 */
#ifndef RRMHD_H
#define RRMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { RRMHD_NVAR = 12 };

typedef enum {
  RRMHD_OK = 0,
  RRMHD_E_INVALID = -1,    /* bad argument (null pointer, size mismatch, bad option) */
  RRMHD_E_C2P = -2,        /* primitive recovery failed in at least one cell (report) */
  RRMHD_E_IMPLICIT = -3,   /* implicit source solve failed in at least one cell     */
  RRMHD_E_NONFINITE = -4,  /* a non-finite value was produced                       */
  RRMHD_E_DEVICE = -5,     /* a HIP call or kernel launch failed                    */
  RRMHD_E_WORKSPACE = -6   /* workspace null, too small or misaligned               */
} rrmhd_status;

typedef enum { RRMHD_BC_PERIODIC = 0, RRMHD_BC_OUTFLOW = 1, RRMHD_BC_INFLOW = 2 } rrmhd_bc;
/* Reconstruction (Section 3.2): piecewise constant, or PLM with the MinMod, MC
 * or VanLeer slope limiter. */
enum { RRMHD_RECON_GODUNOV = 0, RRMHD_RECON_MINMOD = 1, RRMHD_RECON_MC = 2, RRMHD_RECON_VANLEER = 3 };
enum { RRMHD_BETA_ALL = 0, RRMHD_BETA_RAD_ONLY = 1, RRMHD_BETA_OFF = 2 };
enum { RRMHD_IMP_PICARD_NEWTON = 0, RRMHD_IMP_NEWTON = 1, RRMHD_IMP_PICARD = 2 };
/* Face flux (Section 3.2). RRMHD_SOLVER_PVM: the Jacobian-free PVM-int flux
 * with the opacity factor beta (nested finite differences with step pvm_eps).
 * RRMHD_SOLVER_HLL: Rad-HLL, the HLL flux with separate signal speeds for the
 * magnetofluid rows (extreme roots of the RMHD quartic) and the radiation rows
 * (eqs. lam1-lam3, limited by eq. limits). RRMHD_SOLVER_PVM_JVP: the same
 * PVM-int polynomial with every Jacobian-vector product exact (forward-mode
 * derivative through the primitive recovery) instead of a difference; pvm_eps
 * and pvm_eps_mixed are unused (with RRMHD_MIXED the flux products are binary32
 * and the recovery of U_m and its derivative binary64). With RRMHD_MIXED,
 * Rad-HLL runs entirely in binary32. Every solver and precision can be mixed
 * in one batch of rrmhd_step_batch. */
enum { RRMHD_SOLVER_PVM = 0, RRMHD_SOLVER_HLL = 1, RRMHD_SOLVER_PVM_JVP = 2 };
/* Precision of the explicit step. RRMHD_FP64: everything in binary64.
 * RRMHD_MIXED: reconstruction, fluxes and the PVM Horner / finite-difference
 * arithmetic in binary32, each difference taken with a step normalised to
 * its direction (U_m + s w with s = pvm_eps_mixed max|U_m| / max|w| over the
 * chain's rows, divided by s); all primitive recoveries, the flux divergence
 * and the implicit solve in binary64. */
enum { RRMHD_FP64 = 0, RRMHD_MIXED = 1 };

/* Cartesian grid of interior cells (Section 3.1: finite volumes, cell
 * averages). Cells outside the domain are not stored: periodic boundaries
 * wrap, outflow copies the nearest interior cell (zero gradient), inflow
 * (allowed only on the lo side of the last axis) takes inflow_U where
 * inflow_mask is set and copies elsewhere. */
typedef struct {
  int ndim;                         /* 1, 2 or 3                                          */
  int n[3];                         /* interior cells per axis; unused axes must be 1;
                                       n0*n1*n2 < 2^31                                    */
  double dx[3];                     /* cell sizes                                         */
  int bc_lo[3], bc_hi[3];           /* rrmhd_bc per axis side                             */
  long long var_stride;             /* elements between variable planes, >= n0*n1*n2     */
  const double* inflow_U;           /* device [12][transverse cells], conserved; or NULL  */
  const unsigned char* inflow_mask; /* device [transverse cells]; or NULL                 */
} rrmhd_grid;

/* Method parameters. rrmhd_default_params fills the values used by the
 * paper's scheme (PVM-int-8, eps = 1e-8, PLM MinMod, IMEX RK2 analogue). */
typedef struct {
  double gamma;     /* ideal-gas index (eq. eos)                                       */
  double a_rad;     /* radiation constant a_R; 4 pi B = a_R T^4                        */
  double t_coeff;   /* T = t_coeff * p / rho                                           */
  double pvm_eps;   /* finite-difference step of the Jacobian-free chain (1e-8)        */
  double c2p_tol;   /* relative Newton tolerance of primitive recovery                 */
  double imp_tol;   /* relative tolerance of the implicit radiation solve              */
  double rho_floor; /* state substituted (and counted) where recovery fails            */
  double p_floor;
  int pvm_k;        /* internal polynomial p_k, degree 2^k, k = 0..4 (3: PVM-int-8)     */
  int beta_mode;    /* RRMHD_BETA_*: which rows the opacity factor beta scales          */
  int recon;        /* RRMHD_RECON_*                                                    */
  int rk_order;     /* 2: SSP-RK2 analogue of the paper's scheme; 3: the paper's RK3    */
  int c2p_maxit;
  int imp_maxit;
  int imp_picard_it;/* Picard iterations before Newton (eq. C^(m) iteration)            */
  int imp_method;   /* RRMHD_IMP_*                                                      */
  int precision;    /* RRMHD_FP64 | RRMHD_MIXED                                         */
  double pvm_eps_mixed; /* size of the FP32 chain's difference step relative to max|U_m|
                           (2^-12; see RRMHD_MIXED)                                  */
  double e_floor;   /* 0 (default): a non-positive E_r entering the implicit solve fails
                       the cell; > 0: it is raised to e_floor keeping tau + E_r and
                       S + F_r (the gas pays), and counted in e_floor_hits           */
  int solver;       /* RRMHD_SOLVER_*: face flux of the explicit step                 */
  int ct;           /* 0: cell-centred B; 1: constrained transport (Section 4: div B
                       kept by CT with CT-contact averaged edge EMFs). With ct = 1
                       the state carries, after its 12 planes, one plane per grid
                       dimension: plane 12 + a holds the normal field b_a of the
                       face on the lower side of each cell along a, and the
                       cell-centred B_a (a < ndim) is kept equal to the mean of
                       its cell's two face values. Periodic grids with ndim >= 2
                       only; not available in rrmhd_step_batch                */
} rrmhd_params;

/* Gray comoving opacities per unit mass (eqs. g0, gi): device arrays [ncell]
 * (x fastest, plain cell count stride) or NULL to use the uniform value. */
typedef struct {
  const double* kappa;
  const double* sigma;
  double kappa0, sigma0;
} rrmhd_opacities;

/* Failure counters accumulated on the device since init or the last
 * rrmhd_report_sync. first_bad_cell is the smallest failing cell index or
 * -1. max_*_it are the largest iteration counts seen. */
typedef struct {
  long long c2p_fail, pvm_fallback, imp_fail, nonfinite, e_floor_hits;
  long long first_bad_cell;
  int max_c2p_it, max_imp_it;
} rrmhd_report;

typedef struct rrmhd_ctx rrmhd_ctx;

/* Fill *p with the default parameters. */
void rrmhd_default_params(rrmhd_params* p);

/* Bytes of device workspace rrmhd_init needs for this grid and these
 * parameters (stage state, primitives, face fluxes, reduction scratch,
 * counters). Returns 0 for an invalid grid. */
size_t rrmhd_workspace_bytes(const rrmhd_grid* g, const rrmhd_params* p);

/* Create a context. `workspace` is caller-owned device memory of at least
 * rrmhd_workspace_bytes(g, p) bytes, 256-byte aligned, used exclusively by
 * this context until rrmhd_destroy. `hip_stream` is a hipStream_t (NULL: the
 * default stream). Allocates a small pinned host buffer; zeroes the counters
 * (enqueued). Errors: RRMHD_E_INVALID, RRMHD_E_WORKSPACE, RRMHD_E_DEVICE. */
rrmhd_status rrmhd_init(rrmhd_ctx** ctx, const rrmhd_grid* g, const rrmhd_params* p,
                        void* workspace, size_t ws_bytes, void* hip_stream);

/* Primitive -> conserved map of eq. eqU on every cell of the context's grid.
 * V, U: device, [12][var_stride] (with ct = 1 only U's first 12 planes are
 * written; the face planes are the caller's). Enqueued. */
rrmhd_status rrmhd_prim_to_cons(rrmhd_ctx* ctx, const double* V, double* U);

/* Conserved -> primitive recovery (the inversion used in the PVM algorithm and
 * the implicit step) on every cell. Failing cells get the floor state and are
 * counted. U, V: device, [12][var_stride]. Enqueued. */
rrmhd_status rrmhd_cons_to_prim(rrmhd_ctx* ctx, const double* U, double* V);

/* One IMEX step of size dt (Section 3.1: explicit stage with the PVM-int
 * face fluxes of Section 3.2, eq. explicit, then the implicit solve of
 * Section 3.3, eq. impliciteq; stages of the SSP RK pattern). U: device
 * [12][var_stride] ([12 + ndim][var_stride] with ct = 1: the face fields
 * advance by the curl of the CT-contact edge EMFs), updated in place. g must
 * describe the context's grid (same ndim and n; dx and boundaries are taken
 * from g). Enqueued; on a
 * numerical failure the failing cells keep their explicit state and the
 * counters say which. */
rrmhd_status rrmhd_step(rrmhd_ctx* ctx, double* U, const rrmhd_grid* g, double dt,
                        const rrmhd_opacities* opac);

/* Largest signal speed over all cells and directions (fluid fast-speed bound
 * and the M1 eigenvalues of eqs. lam1-lam3), capped at 1. Synchronizes the
 * stream and writes the value to *smax_host. */
rrmhd_status rrmhd_max_speed(rrmhd_ctx* ctx, const double* U, const rrmhd_grid* g,
                             double* smax_host);

/* nsteps IMEX steps (as rrmhd_step), each with its time step taken on the
 * device from the state at the start of the step: dt = (cfl * min_d dx_d) /
 * s_max, s_max as rrmhd_max_speed computes it (CFL condition, Section 3.2;
 * signal speeds of eqs. lam1-lam3). The result is bitwise that of calling
 * rrmhd_max_speed and then rrmhd_step with that dt on the host, nsteps times,
 * but nothing waits on the host: the work is enqueued on the context's stream.
 * (Capturing it in a HIP graph is untested and not supported.) The first stage's
 * primitive recovery and the signal speeds share one pass, so a recovery
 * failure in the step's initial state is counted once in the report (the
 * separate calls count it in both). A step whose s_max is 0 or not a number
 * runs with dt = 0 and adds one to the report's nonfinite count.
 * cfl: > 0. dt_out: optional caller-owned DEVICE array of nsteps doubles that
 * receives each step's dt (NULL: not written). U as in rrmhd_step.
 * Errors: RRMHD_E_INVALID for a grid of another shape, cfl not > 0 and finite
 * or nsteps < 0 (nothing enqueued); RRMHD_E_DEVICE on a launch failure. */
rrmhd_status rrmhd_advance(rrmhd_ctx* ctx, double* U, const rrmhd_grid* g, double cfl, int nsteps,
                           const rrmhd_opacities* opac, double* dt_out);

/* Allocation-free variant of rrmhd_advance, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc): the
 * same nsteps IMEX steps with dt formed on the device, bitwise equal to
 * rrmhd_advance on a context with the same grid and parameters, but with no
 * context, no caller workspace and no allocation of any kind (device or
 * host). Its workspace is a per-device array inside the library of 64 MiB
 * (67108864 bytes), loaded with the library's code object and held by each
 * GPU until the process ends; a grid whose rrmhd_workspace_bytes exceeds it
 * (above about 140 000 cells, e.g. 2D grids beyond 360^2) returns
 * RRMHD_E_WORKSPACE with nothing enqueued.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: the call clears what must start at zero (counters,
 * iteration maxima) itself, but calls that overlap on one GPU (on different
 * streams, or from host threads without ordering) race and give undefined
 * results. Work runs on the current device, enqueued on hip_stream (NULL:
 * the default stream), which must belong to that device.
 * g, p: as for rrmhd_init; U, cfl, nsteps, opac, dt_out: as for
 * rrmhd_advance. report_dev: optional caller-owned DEVICE pointer to one
 * rrmhd_report, which receives this call's failure counters once its work
 * has run (enqueued after it; NULL: not written).
 * Errors: RRMHD_E_INVALID (bad grid, parameters, cfl or nsteps; nothing
 * enqueued), RRMHD_E_WORKSPACE (grid too large for the scratch array),
 * RRMHD_E_DEVICE (no current device, symbol lookup or launch failure). */
rrmhd_status rrmhd_advance_noalloc(const rrmhd_grid* g, const rrmhd_params* p, double* U, double cfl, int nsteps,
                                   const rrmhd_opacities* opac, double* dt_out, rrmhd_report* report_dev,
                                   void* hip_stream);

/* Diagnostic: the face fluxes of the first stage for state U (recovery,
 * reconstruction and PVM-int flux, Section 3.2). Fh: device, the directions
 * one after another, each [12][faces_d] with faces_d = prod(n) with n_d + 1
 * along d, face i along d between cells i-1 and i, x fastest. Enqueued. */
rrmhd_status rrmhd_face_fluxes(rrmhd_ctx* ctx, const double* U, const rrmhd_opacities* opac,
                               double* Fh);

/* Diagnostic kernel timing. Each launch of a selected kernel class is
 * bracketed by HIP events recorded on the context's stream (up to 8192
 * launches; further launches are not timed). Kernel classes:
 * RRMHD_K_PRIMS (cell recovery), RRMHD_K_FACES (reconstruction + PVM-int face
 * flux), RRMHD_K_UPDATE (flux divergence + Picard phase of the implicit
 * solve), RRMHD_K_NEWTON (Newton phase for the cells Picard left), and
 * RRMHD_K_SPEED (signal speeds). `enable` is a bit mask, bit k selecting
 * class k (RRMHD_PROFILE_ALL: every class; 0: timing off); other values are
 * RRMHD_E_INVALID. Each event pair serializes the stream around the launch it
 * brackets, so select only what is needed. Enabling clears earlier records.
 * Allocates host-side event objects only. */
enum { RRMHD_K_PRIMS = 0, RRMHD_K_FACES = 1, RRMHD_K_UPDATE = 2, RRMHD_K_SPEED = 3, RRMHD_K_NEWTON = 4,
       RRMHD_K_COUNT = 5 };
enum { RRMHD_PROFILE_ALL = (1 << RRMHD_K_COUNT) - 1 };
rrmhd_status rrmhd_profile_enable(rrmhd_ctx* ctx, int enable);

/* Time only every stride-th launch of each selected class (counted from the
 * last rrmhd_profile_enable; default 1). stride < 1: RRMHD_E_INVALID. */
rrmhd_status rrmhd_profile_stride(rrmhd_ctx* ctx, int stride);

/* Totals of the timed launches of kernel class k since enabling: summed
 * event time in ms, number of launches and work units (cells or faces)
 * those launches processed. Synchronizes on the last recorded event. */
rrmhd_status rrmhd_profile_read(rrmhd_ctx* ctx, int k, double* total_ms, long long* launches,
                                long long* units);

/* Read the failure counters (synchronizes the stream) and reset them. */
rrmhd_status rrmhd_report_sync(rrmhd_ctx* ctx, rrmhd_report* out);

/* ---- Batched stepping of independent simulations (serving) ----------------
 * A batch advances several contexts (each with its own grid, parameters,
 * state and workspace) with one launch per kernel class and stage: every
 * block looks its simulation up in a device descriptor table. Each
 * simulation's arithmetic is exactly that of rrmhd_step / rrmhd_max_speed,
 * so results do not depend on the batch composition. Work is enqueued on the
 * batch's stream; the contexts must not be used on other streams meanwhile.
 * All contexts of one call must use the same rk_order, and a context may
 * appear only once per call. */
typedef struct rrmhd_batch rrmhd_batch;

/* Device workspace for a batch of up to max_sims simulations (descriptor
 * table, block offsets, per-simulation maxima); 0 if max_sims is invalid. */
size_t rrmhd_batch_workspace_bytes(int max_sims);

/* Create a batch handle. workspace: caller-owned device memory, 256-byte
 * aligned, >= rrmhd_batch_workspace_bytes(max_sims). Allocates pinned host
 * staging buffers and two events. */
rrmhd_status rrmhd_batch_init(rrmhd_batch** b, int max_sims, void* workspace, size_t ws_bytes,
                              void* hip_stream);

/* Signal speed of each simulation (as rrmhd_max_speed), all in one pass;
 * one stream synchronization for the whole batch. smax_host: [nsim]. */
rrmhd_status rrmhd_max_speed_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx,
                                   const double* const* U, double* smax_host);

/* One IMEX step of each simulation s with its own dt_host[s] (as
 * rrmhd_step with the context's grid). opac: [nsim] (entries may be NULL for
 * zero opacity). Enqueued. */
rrmhd_status rrmhd_step_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, double* const* U,
                              const double* dt_host, const rrmhd_opacities* const* opac);

/* Up to nsteps steps of each simulation's own CFL loop, run on the device
 * with no host synchronization (Sec. 3.1 time stepping with the CFL rule of
 * rrmhd_max_speed): per step, the signal speeds; then, for each simulation s
 * not at its end, dt = min(cfl_dx[s] / s_max, t_end[s] - t), t += dt, n += 1,
 * and the IMEX step with that dt. Simulation s is at its end once
 * n >= max_steps[s] when max_steps[s] >= 0, else once
 * t >= t_end[s] (1 - 1e-14); from then on it is not stepped (its blocks of
 * every launch return at once). Each simulation's time steps and states are
 * those of the host loop rrmhd_max_speed_batch + rrmhd_step_batch with the
 * same rule, bit for bit, whatever else is in the batch. After the first
 * step of a call, the last stage of each step also recovers the next step's
 * primitives and signal speeds (no separate passes for them).
 *   cfl_dx:    [nsim] host, CFL number times the smallest cell width, > 0.
 *   t_end:     [nsim] host, end time (>= 0; may be +inf for a step-count
 *              request).
 *   max_steps: [nsim] host, steps to take, or < 0 for an end-time request.
 *   t, n:      [nsim] host, the time and steps reached so far (uploaded).
 * A time step that is not finite and >= 0 is counted as non-finite in that
 * simulation's report and its time set to +inf (it takes no further step).
 * Enqueued on the batch's stream; rrmhd_batch_clock returns the clock after
 * it. RRMHD_E_INVALID for bad sizes or values (nothing enqueued). */
rrmhd_status rrmhd_advance_batch(rrmhd_batch* b, int nsim, rrmhd_ctx* const* ctx, double* const* U,
                                 const rrmhd_opacities* const* opac, const double* cfl_dx, const double* t_end,
                                 const long long* max_steps, const double* t, const long long* n, int nsteps);

/* Wait for the last rrmhd_advance_batch of this batch and copy its
 * simulations' clock to t[nsim], n[nsim] (host). nsim must be that call's.
 * Synchronizes with that call only (an event), not with later work. */
rrmhd_status rrmhd_batch_clock(rrmhd_batch* b, int nsim, double* t, long long* n);

void rrmhd_batch_destroy(rrmhd_batch* b);

/* Release the context (not the workspace, which the caller owns). */
void rrmhd_destroy(rrmhd_ctx* ctx);

/* Static description of a status code. */
const char* rrmhd_strerror(rrmhd_status s);

#ifdef __cplusplus
}
#endif

#endif /* RRMHD_H */
