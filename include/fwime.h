/*
 * fwime.h -- C ABI of the MI355X (gfx950) FWIME hot-path library.
 *
 * Operations follow Section 2 of Barnier, Biondi, Clapp and Biondi, "Full
 * waveform inversion by model extension: practical applications" (arXiv
 * 2206.02362): nonlinear modeling f(m) with an acoustic isotropic
 * constant-density two-way wave equation, the Born operator extended with
 * horizontal subsurface offsets B~(m), its adjoint (the extended imaging
 * condition), and the FWIME objective of eq. fwime.obj with its gradients
 * (eqs. fwime.gradient.split, fwime.gradient.born, fwime.gradient.tomo),
 * evaluated at a given extended perturbation p~.
 *
 * Discretization (the paper prints none; the choices are stated once here):
 *   - padded grid: the model grid (nz, nx) plus an absorbing strip of nb cells
 *     on every side (NZ = nz + 2 nb, NX = nx + 2 nb); the velocity is copied
 *     from the nearest model cell into the strip;
 *   - equation n = 0 .. nt-2:  u^{n+1} = g (2 u^n - g u^{n-1} + V (L u^n + f^n)),
 *     u^{-1} = u^0 = 0, V = v^2 dt^2, L the radius-4 (8th-order) Laplacian with
 *     zero values outside the padded grid, g(iz, ix) = g_z(iz) g_x(ix) the
 *     Cerjan taper with g_1D(k) = exp(-(sponge_alpha * k / nb)^2) for the cell
 *     k = 1..nb cells into the strip (Cerjan et al. 1985, cited in Section 3);
 *   - point source f^n = w^n / (dx dz) at the source cell; receivers record
 *     d^k = u^k at their cell for k = 0 .. nt-1 (d^0 = 0);
 *   - extended Born with offset h = ih dx, ih in [-(nh-1)/2, (nh-1)/2]: in
 *     equation n the scattered field receives
 *       s_n(z, y + h) += 2 p~(z, y, h) / (v(z, y)^3 dt^2) * T2u_n(z, y - h),
 *     T2u_n = u^{n+1}/g - 2 u^n + g u^{n-1}; terms whose y -/+ h leave the
 *     padded grid are dropped; nh = 1 is ordinary Born;
 *   - p~ is an extended VELOCITY perturbation (m/s) on the model grid.
 *
 * Conventions for every entry point:
 *   - Layout: z is the fastest axis.  vel[nx][nz], ptilde[nh][nx][nz],
 *     data[nshots][nrec][nt], wavelet[nshots][nt].
 *   - Memory: arrays of floating-point values are DEVICE pointers on the
 *     context's device, owned by the caller.  The geometry index arrays
 *     (src_iz, src_ix, rec_iz, rec_ix) and the DSO weights are HOST pointers.
 *     Outputs are overwritten, never accumulated into.
 *   - Execution: work is enqueued on `stream` (a hipStream_t, passed as void*)
 *     and the call returns once it is enqueued.  Before enqueuing, each call
 *     validates its inputs, which includes one small device reduction and a
 *     stream synchronization (velocity range for the CFL test, finiteness).
 *   - Errors: on any nonzero return nothing has been written to the outputs.
 *   - Threads: a context is used by one host thread and one stream at a time.
 */
#ifndef FWIME_H
#define FWIME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define FWIME_OK          0
#define FWIME_EINVAL      1  /* bad dims, nh even or too large, geometry outside the model grid,
                                CFL violated, non-positive velocity, null pointer */
#define FWIME_ENOMEM      2  /* device memory or the context's HBM budget exhausted */
#define FWIME_EHIP        3  /* HIP runtime error (text via fwime_last_error) */
#define FWIME_ENONFINITE  4  /* NaN or Inf in an input array */

/* Model grid (unpadded), absorbing strip width and time axis. */
typedef struct {
  int32_t nz, nx;      /* model grid, cells                              */
  int32_t nb;          /* absorbing strip, cells on each side (>= 0)     */
  int32_t nt;          /* time samples (>= 2)                            */
  double dz, dx, dt;   /* m, m, s                                        */
  double sponge_alpha; /* taper strength (0 disables the taper)          */
  int32_t free_surface; /* nonzero: free surface on the model's first row */
} fwime_grid_t;
/* Free surface (the free-surface-multiples variant of the Marmousi2 test in
 * Section 3 models with a free surface at the water surface and absorbing
 * boundaries elsewhere, after Robertsson's image method): the pressure is
 * zero on the model's first row (padded row nb) and above it, and the
 * Laplacian of the rows below reads the field mirrored with opposite sign,
 * u(nb - k) = -u(nb + k).  The top strip is then unused; it needs nb >= 4
 * (FWIME_EINVAL otherwise).  Every operator honours it: all of them step the
 * same stencil, and the mirrored operator stays symmetric, so adjoints and
 * gradients carry over unchanged. */

/* Acquisition: nshots shots sharing the grid and velocity model. */
typedef struct {
  int32_t nshots, nrec;
  const int32_t *src_iz, *src_ix;  /* HOST [nshots], model-grid indices      */
  const int32_t *rec_iz, *rec_ix;  /* HOST [nshots][nrec], model-grid indices */
  const float *wavelet;            /* DEVICE [nshots][nt]                     */
} fwime_geom_t;

typedef struct fwime_ctx fwime_ctx_t;

/* Create a context on `device`.  It owns all scratch memory (wavefield
 * buffers, checkpoints, geometry tables) and never allocates beyond
 * `hbm_budget_bytes` (0 = no limit besides the device).  Returns FWIME_OK and
 * sets *out, or an error code. */
int fwime_ctx_create(int device, size_t hbm_budget_bytes, fwime_ctx_t **out);

/* Release every allocation of the context (synchronizes the device). */
void fwime_ctx_destroy(fwime_ctx_t *ctx);

/* Nonlinear modeling f(m), the first term of eq. fwime.obj:
 * data[s][r][k] = u^k at receiver r of shot s.  vel: DEVICE [nx][nz] m/s. */
int fwime_model(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                const fwime_geom_t *geom, float *data, void *stream);

/* Allocation-free modeling, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and same results, bit for bit, as fwime_model,
 * but every piece of device scratch (validation partials, padded velocity,
 * tapers, geometry tables, wavefields) is carved from one static device array
 * of FWIME_STATIC_SCRATCH_BYTES that the library holds on each device until
 * the process ends; the call allocates no device or pinned host memory (its
 * host-side table construction uses ordinary heap memory).  Shots run in as
 * many batches as the array needs; if one shot's scratch does not fit,
 * the call returns FWIME_ENOMEM and writes nothing.  Every call on a device
 * shares that device's array, which keeps the last call's contents (the call
 * clears what must start at zero): calls that overlap on one device, from any
 * context or stream, race and must be serialized by the caller.  Like every
 * entry point it validates its inputs with one stream synchronization. */
#define FWIME_STATIC_SCRATCH_BYTES (64u << 20)
int fwime_model_static(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, float *data, void *stream);

/* Extended Born modeling B~(m) p~ (the data-correcting term of eq. fwime.obj).
 * ptilde: DEVICE [nh][nx][nz]; nh odd, 1 <= nh <= 2 nx - 1; data as above. */
int fwime_born_ext_fwd(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, int32_t nh, const float *ptilde,
                       float *data, void *stream);

/* Adjoint of fwime_born_ext_fwd (extended migration, the imaging condition of
 * the variable-projection step, eqs. vp.obj and vp.pseudo.inv):
 * ptilde_out(z,y,h) = 2/(v(z,y)^3 dt^2) sum_shots sum_n T2u_n(z,y-h) lambda_n(z,y+h),
 * with lambda the adjoint field driven by `data` at the receivers. */
int fwime_born_ext_adj(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, int32_t nh, const float *data,
                       float *ptilde_out, void *stream);

/* Extended Born modeling with time lags B~_tau p~ (Section 2: B~ is extended
 * with either time lags or horizontal subsurface offsets).  Lags
 * tau_k = k lag dt, k = -K .. K, ntau = 2K+1 (odd, <= 1023), lag >= 1 time
 * steps with lag (ntau - 1) <= 4 nt.  The scattering source of equation n is
 * sum_k 2 p~(z,y,k) / (v(z,y)^3 dt^2) T2u_{n-2k lag}(z,y) on the model grid,
 * terms whose background step falls outside 0 .. nt-2 dropped.  ptau: DEVICE
 * [ntau][nx][nz]; data as above (overwritten).  The background's T2 history of
 * a shot batch is held whole: about (2 nt + 10) padded fields per shot of
 * device memory, which sets the batch size; FWIME_ENOMEM if one shot does
 * not fit. */
int fwime_born_ext_tau_fwd(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                           const fwime_geom_t *geom, int32_t ntau, int32_t lag,
                           const float *ptau, float *data, void *stream);

/* Adjoint of fwime_born_ext_tau_fwd:
 * ptau_out(z,y,k) = 2/(v(z,y)^3 dt^2) sum_shots sum_n T2u_{n-2k lag}(z,y) lambda_n(z,y),
 * with lambda the adjoint field driven by `data` at the receivers.  ptau_out:
 * DEVICE [ntau][nx][nz] (overwritten); about 2 nt + 8 padded fields per shot. */
int fwime_born_ext_tau_adj(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                           const fwime_geom_t *geom, int32_t ntau, int32_t lag,
                           const float *data, float *ptau_out, void *stream);

/* FWIME objective of eq. fwime.obj at the given p~ and its gradients:
 *   r = f(m) + B~(m) p~ - dobs,
 *   obj = 1/2 ||r||^2 + eps^2/2 sum_h dso[h]^2 ||p~_h||^2,
 *   grad_vel = (B^* + T^*) r  (eqs. fwime.gradient.born and .tomo, no spline),
 *   grad_ptilde = B~^* r + eps^2 dso[h]^2 p~.
 * dobs: DEVICE [nshots][nrec][nt]; dso: HOST double [nh]; obj: DEVICE double[1];
 * grad_vel: DEVICE [nx][nz]; grad_ptilde: DEVICE [nh][nx][nz]. */
int fwime_gradient(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                   const fwime_geom_t *geom, int32_t nh, const float *ptilde,
                   const float *dobs, double eps, const double *dso,
                   double *obj, float *grad_vel, float *grad_ptilde, void *stream);

/* The same objective and gradients with B~ extended by time lags (Section 2
 * names both extensions; the paper's Marmousi2 test uses 101 lags of 16 ms):
 * ntau lags of `lag` steps as in fwime_born_ext_tau_fwd.  The tomographic
 * part spreads the adjoint field over the lags, e_m = sum_k c_k lambda_{m+2k lag}
 * with c_k = 2 ptau_k / (v^3 dt^2), and g_3 takes the lag image in place of
 * the offset image.  dso: HOST double [ntau]; ptau, grad_ptau: DEVICE
 * [ntau][nx][nz]; others as for fwime_gradient.  Every history of a shot
 * batch is kept whole: about 4 (nt + 1) + 80 padded fields per shot. */
int fwime_gradient_tau(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, int32_t ntau, int32_t lag, const float *ptau,
                       const float *dobs, double eps, const double *dso,
                       double *obj, float *grad_vel, float *grad_ptau, void *stream);

/* Variable-projection step of FWIME (Section 2, eqs. vp.obj, pert.opt and
 * vp.pseudo.inv): niter iterations of linear conjugate gradient on the normal
 * equation (B~* B~ + eps^2 D* D) p~ = B~* (dobs - f(m)), starting from p~ = 0,
 * where D is the diagonal DSO operator with weight dso[h] on offset plane h.
 * Each iteration applies B~ and B~* once (four propagations per shot).
 * dobs: DEVICE [nshots][nrec][nt]; dso: HOST double [nh];
 * ptilde_out: DEVICE [nh][nx][nz], the last iterate;
 * phi_out: HOST double [niter + 1], the objective of eq. vp.obj at p~_0 = 0
 * and after each iteration (tracked from the CG residual, no extra
 * propagations).  If a search direction has no positive curvature the
 * iteration stops and the remaining phi_out entries repeat the last value.
 * The call synchronizes `stream` once per inner product.  The solver's
 * vectors (4 model-size and 2 data-size arrays) stay in the context until
 * fwime_ctx_trim or fwime_ctx_destroy, and count against its HBM budget.
 * When they fit in half of the free memory (and of the budget), the
 * background checkpoints of every shot (6 bytes x 2 ceil((nt-1)/K) padded
 * fields per shot, K = ceil(sqrt(nt))) are kept for the whole call, so each
 * B~* after the first skips its background forward pass; the results are the
 * same bit for bit either way (FWIME_VP_NOCACHE=1 in the environment turns
 * the cache off).
 * Argument errors (FWIME_EINVAL) are reported before anything is written; a
 * failure during the iteration leaves ptilde_out and phi_out unspecified. */
int fwime_vp_solve(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                   const fwime_geom_t *geom, int32_t nh, const float *dobs, double eps,
                   const double *dso, int32_t niter, float *ptilde_out, double *phi_out,
                   void *stream);

/* The same variable-projection step with B~ extended by time lags (the
 * paper's choice in four of its five examples): CG on
 * (B~_tau* B~_tau + eps^2 D* D) p~ = B~_tau* (dobs - f(m)) with the operators
 * of fwime_born_ext_tau_fwd / _adj (ntau lags of `lag` steps, same limits).
 * dso: HOST double [ntau]; ptau_out: DEVICE [ntau][nx][nz]; phi_out as above.
 * Device memory per shot as for fwime_born_ext_tau_fwd; no checkpoint cache. */
int fwime_vp_solve_tau(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, int32_t ntau, int32_t lag, const float *dobs,
                       double eps, const double *dso, int32_t niter, float *ptau_out,
                       double *phi_out, void *stream);

/* ---- Batched modeling of jobs with different grids ----------------------
 * One job = one call's worth of fwime_model (grid, velocity, shots).  All
 * jobs advance together: every time step is one launch over the tiles of all
 * jobs (a job whose time axis is shorter idles once it is done), the time loop
 * is replayed from a captured graph, and the tile width is chosen by timing
 * the candidates on the first call for a given set of grid shapes (cached in
 * the context).  Results equal fwime_model's for each job. */
typedef struct {
  fwime_grid_t grid;
  const float *vel;        /* DEVICE [nx][nz] */
  fwime_geom_t geom;
  float *data;             /* DEVICE [nshots][nrec][nt], overwritten */
} fwime_job_t;

int fwime_model_batch(fwime_ctx_t *ctx, int32_t njobs, const fwime_job_t *jobs, void *stream);

/* ---- Continuous batching of modeling jobs (request loops) ---------------
 * An engine runs modeling jobs in shared launches while jobs come and go:
 * a submitted job joins at the next round, every round advances all joined
 * jobs by steps_per_round time steps with one two-step launch per two steps
 * over the tiles of all of them (each job at its own time index), and a job
 * leaves once its last sample is recorded.  Each job computes exactly what
 * fwime_model computes for it, bit for bit.  Per-job device memory (about
 * four padded fields per shot plus tables) is allocated stream-ordered on the
 * engine's stream at submission and released the same way after the job's
 * last round.  The job's vel, wavelet and data stay owned by the caller and
 * must stay valid until fwime_engine_poll reports the job done.
 * All engine calls come from one host thread. */
typedef struct fwime_engine fwime_engine_t;
typedef struct {
  int32_t pending;     /* submitted, not yet joined              */
  int32_t active;      /* in the time loop                       */
  int32_t finishing;   /* last round enqueued, not yet completed */
  int64_t step;        /* global step counter                    */
  int64_t rounds, launches;
} fwime_engine_info_t;

/* steps_per_round: even, >= 2; max_jobs: jobs held at once (pending +
 * active); stream: the engine's stream, used by every later engine call. */
int fwime_engine_create(fwime_ctx_t *ctx, int32_t steps_per_round, int32_t max_jobs, void *stream,
                        fwime_engine_t **out);
/* Validates the job (one device reduction and a synchronization of
 * check_stream, the stream on which its inputs were written: not the engine's
 * stream, whose rounds keep running), prepares it on the engine's stream and
 * queues it for the next round.  *ticket identifies it in fwime_engine_poll. */
int fwime_engine_submit(fwime_engine_t *e, const fwime_job_t *job, void *check_stream, int64_t *ticket);
/* Enqueues one round on the engine's stream (nothing when no job is joined). */
int fwime_engine_run(fwime_engine_t *e);
/* Reports up to cap jobs whose data is complete (*ndone of them, in tickets)
 * and releases them; does not block. */
int fwime_engine_poll(fwime_engine_t *e, int64_t *tickets, int32_t cap, int32_t *ndone);
int fwime_engine_info(const fwime_engine_t *e, fwime_engine_info_t *out);
/* Waits for the engine's stream and releases everything it holds. */
void fwime_engine_destroy(fwime_engine_t *e);

/* Context state, for schedulers and tests. */
typedef struct {
  size_t arena_bytes;        /* scratch arena currently held            */
  size_t tape_bytes;         /* device memory held by live tapes         */
  int32_t tile_x;            /* default stencil tile width               */
  int32_t last_batch_tile_x; /* width used by the last fwime_model_batch */
  int32_t tuned_signatures;  /* batch shapes with a tuned width          */
  int64_t last_stencil_launches; /* stencil launches of the last timed call, -1 if none */
  double last_stencil_ms;    /* event time of those launches, ms         */
} fwime_info_t;

/* With timing on, the last fwime_model / fwime_model_batch call's stencil
 * launch loop is bracketed by two HIP events recorded on the call's stream;
 * this call then waits for the second event and reports the elapsed time
 * and the number of stencil launches (a launch advances every active shot
 * by one or two time steps).  Without timing, last_stencil_launches is -1. */
int fwime_ctx_info(const fwime_ctx_t *ctx, fwime_info_t *out);

/* Turn the event timing above on (on != 0) or off.  It adds two event
 * records per modeling call and nothing to the kernels. */
int fwime_ctx_set_timing(fwime_ctx_t *ctx, int32_t on);

/* Release the context's scratch arena after `stream` (its stream) is idle.
 * The next call allocates again.  For schedulers that share one HBM budget
 * among several contexts. */
int fwime_ctx_trim(fwime_ctx_t *ctx, void *stream);

/* Device bytes one call of operator `op` needs to run all nshots shots in a
 * single batch (the scratch the context arena must hold).  Calls with less
 * budget run their shots in several batches. */
#define FWIME_OP_MODEL     0
#define FWIME_OP_BORN_FWD  1
#define FWIME_OP_BORN_ADJ  2
#define FWIME_OP_GRADIENT  3
int fwime_footprint(const fwime_grid_t *grid, int32_t nshots, int32_t nrec, int32_t nh, int32_t op,
                    size_t *bytes);

/* ---- Forward / backward split for automatic differentiation ------------
 * The pair below evaluates d = f(m) + B~(m) p~ (the predicted data of
 * eq. fwime.obj) and, later, the adjoint-state backward of that map: given
 * an adjoint source a = dL/dd, grad_vel = (B^* + T^*) a (the Born and
 * tomographic parts of eqs. fwime.gradient.born and .tomo) and
 * grad_ptilde = B~^* a.  The forward keeps sqrt(nt)-spaced checkpoints of the
 * background and scattered wavefields of every shot in a tape (device memory
 * owned by the tape, counted against the context's HBM budget), plus copies of
 * vel, ptilde and the wavelets; the backward recomputes one segment at a time
 * from them.  A tape serves exactly one backward (its checkpoints are
 * consumed); free it with fwime_tape_free in every case. */
typedef struct fwime_tape fwime_tape_t;

/* data: DEVICE [nshots][nrec][nt] receives f(m) + B~(m) p~; *tape is set on success. */
int fwime_forward_tape(fwime_ctx_t *ctx, const fwime_grid_t *grid, const float *vel,
                       const fwime_geom_t *geom, int32_t nh, const float *ptilde, float *data,
                       fwime_tape_t **tape, void *stream);

/* adjsrc: DEVICE [nshots][nrec][nt]; grad_vel: DEVICE [nx][nz]; grad_ptilde: DEVICE [nh][nx][nz]. */
int fwime_backward_tape(fwime_ctx_t *ctx, fwime_tape_t *tape, const float *adjsrc,
                        float *grad_vel, float *grad_ptilde, void *stream);

/* Release a tape (synchronizes the device); null is ignored. */
void fwime_tape_free(fwime_tape_t *tape);

/* Linear spline operator S of Section 2: the model lives on a spline grid of
 * node coordinates zn[nzn] (depth) and xn[nxn] (lateral), in the units of dz
 * and dx, and S maps node values onto the finite-difference grid by linear
 * interpolation along z and along x (the tensor product of the two 1D hat
 * interpolations; grids refined by halving end on the finite-difference grid,
 * where S is the identity).  Fine point (ix, iz) sits at (ix dx, iz dz).
 * zn, xn: HOST double, strictly increasing, 2 to 2^24 nodes each, covering
 * [0, (nz-1) dz] and [0, (nx-1) dx] (to 1e-9 of the node span); read during
 * the call only.  mc: DEVICE [nxn][nzn]; out: DEVICE [nx][nz], z fastest.
 * The call synchronizes `stream` twice (before taking the context's arena and
 * after the node upload); the interpolation tables
 * (about 12 bytes per fine point and node) live in the context's arena.
 * Argument errors (FWIME_EINVAL) are reported before anything is written;
 * non-finite node values propagate. */
int fwime_spline_apply(fwime_ctx_t *ctx, int32_t nz, int32_t nx, double dz, double dx,
                       int32_t nzn, const double *zn, int32_t nxn, const double *xn,
                       const float *mc, float *out, void *stream);

/* Adjoint S* of fwime_spline_apply (Section 2: the gradient with respect to
 * the node values is S* applied to the model-grid gradient, eq.
 * fwime.gradient.split): f: DEVICE [nx][nz] onto mc_out: DEVICE [nxn][nzn].
 * Each node gathers the fine points of its two neighbouring cells with their
 * weights in a fixed order, so results do not depend on scheduling.  Same
 * node arguments, synchronization and errors as fwime_spline_apply; the
 * arena also holds an [nx][nzn] FP32 intermediate. */
int fwime_spline_adjoint(fwime_ctx_t *ctx, int32_t nz, int32_t nx, double dz, double dx,
                         int32_t nzn, const double *zn, int32_t nxn, const double *xn,
                         const float *f, float *mc_out, void *stream);

/* Model on the next, finer spline grid (Section 2: the inversion moves along
 * a sequence of spline grids of decreasing spacing): the node values mc on
 * (zn, xn) evaluated by the same linear interpolation at the new nodes
 * (zf, xf).  zn, xn: HOST double as for fwime_spline_apply (starting at the
 * grid's origin); zf[nzf], xf[nxf]: HOST double, strictly increasing, within
 * the old nodes' span (to 1e-9 of it), 1 to 2^24 each; read during the call
 * only.  mc: DEVICE [nxn][nzn]; mf_out: DEVICE [nxf][nzf].  Synchronizes
 * `stream` twice; argument errors (FWIME_EINVAL) before anything is written. */
int fwime_spline_refine(fwime_ctx_t *ctx, int32_t nzn, const double *zn, int32_t nxn, const double *xn,
                        const float *mc, int32_t nzf, const double *zf, int32_t nxf, const double *xf,
                        float *mf_out, void *stream);

/* L-BFGS search direction (Section 3 minimizes the FWIME objective over the
 * spline nodes with L-BFGS): d_out = -H g, where H is the limited-memory
 * inverse-Hessian approximation built from npairs pairs (s_i, y_i), oldest
 * first, with initial matrix (s.y / y.y of the newest pair) I, or I when
 * npairs = 0; the two-loop recursion, never forming H.  Inner products in FP64
 * with a fixed reduction order, vector updates in FP32.
 * s, y: DEVICE [npairs][n]; g, d_out: DEVICE [n] (d_out may be g, must not
 * overlap s or y).  0 <= npairs <= 256, n >= 1.  Every pair must have
 * s_i.y_i > 0 (callers drop the others); otherwise FWIME_EINVAL before
 * anything is written.  The call synchronizes `stream` once before it starts
 * and once per inner product (3 npairs + 1 of them). */
int fwime_lbfgs_direction(fwime_ctx_t *ctx, int64_t n, int32_t npairs, const float *s, const float *y,
                          const float *g, float *d_out, void *stream);

/* Objective callback of fwime_lbfgs_minimize: evaluate f at the DEVICE
 * vector x[n], write the gradient to the DEVICE vector g[n] and f to *f;
 * return 0, or nonzero to stop the minimization.  Device work must be queued
 * on the minimization's stream or be complete when the callback returns. */
typedef int (*fwime_objective_fn)(void *user, const float *x, float *g, double *f);

/* L-BFGS minimization (Section 3: the FWIME objective is minimized over the
 * spline nodes with L-BFGS and a More-Thuente line search).  From x, each
 * iteration takes d = -H g from the last `memory` pairs (as
 * fwime_lbfgs_direction), searches a step along d for the strong Wolfe
 * conditions (ftol 1e-4, gtol 0.9, first trial step 1, at most 100 trials),
 * and keeps the new pair if s.y > 1e-12 |s| |y|.  It stops after maxiter
 * iterations, when |g| <= gtol |g_0|, when d is not a descent direction, or
 * when the line search ends without an acceptable step.
 * x: DEVICE [n], the start on entry and the last accepted iterate on return.
 * work: DEVICE float [work_floats], at least 4096 + (2 memory + 6) n floats,
 * 8-byte aligned, caller-owned (nothing is allocated, so the callback may use
 * the same context freely); a smaller or misaligned buffer is FWIME_EINVAL.
 * f_hist: HOST double [maxiter + 1], f at x_0 and after each iteration, the
 * last value repeated past the stop; iters: HOST, iterations taken.
 * 1 <= memory <= 256.  A callback error stops with FWIME_EINVAL and a
 * non-finite objective with FWIME_ENONFINITE; x then holds the last accepted
 * iterate.  The call synchronizes `stream` once per inner product. */
int fwime_lbfgs_minimize(fwime_ctx_t *ctx, int64_t n, int32_t memory, int32_t maxiter, double gtol,
                         fwime_objective_fn fg, void *user, float *x, float *work, int64_t work_floats,
                         double *f_hist, int32_t *iters, void *stream);

/* Static description of a return code. */
const char *fwime_strerror(int code);

/* Detail of the last error raised on this context (empty if none). */
const char *fwime_last_error(const fwime_ctx_t *ctx);

#ifdef __cplusplus
}
#endif
#endif /* FWIME_H */
