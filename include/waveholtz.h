/*
 * waveholtz.h -- C ABI of libwaveholtz, a gfx950 (MI355X) implementation of the
 * WaveHoltz filter operator and its deflated Krylov acceleration.
 *
 * The operations follow "Numerical Study of Eigenvector Deflation to Accelerate
 * the WaveHoltz Method" (Appelo, Henshaw, Peng):
 *   - the Helmholtz problem  L u + omega^2 u = f,  L = div(c^2 grad), homogeneous
 *     Dirichlet data on the unit box (Section 2.1, eq. helmholtzBVP, eq. L);
 *   - the filter  Pi v = (2/Tbar) int_0^Tbar (cos(omega t) - 1/4) w(t; v) dt
 *     (eq. waveHoltzFilter) evaluated by the explicit scheme eq. discreteWaveExplicit
 *     and the trapezoid rule eq. quadrature, with the time-discretisation error
 *     removed by an adjusted frequency (Section 2.2);
 *   - the linear system A u = (I - S_h) u = b, b = Pi_h 0 (eq. WaveHoltzMatrixEquation),
 *     solved by the fixed-point iteration (Algorithm 1), CG / deflated CG
 *     (Algorithm 3) or restarted GMRES (Algorithm 4, augmented by the deflation set when
 *     one is given), or with direct eigenvector deflation around them (Algorithm 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Grid.    Unit box [0,1]^dim, dim in {2,3}, n cells per side, h = 1/n, nodes
 *          x_j = j h, j = 0..n (eq. discreteHelmholtz).  order == 2:
 *          (L_h W)_p = h^-2 sum_faces c2_f (W_q - W_p), c2_f = (c2_p + c2_q)/2.
 *          order == 4 (c == 1 only; the paper's spatial order): per axis
 *          h^-2 (-W_{i-2} + 16 W_{i-1} - 30 W_i + 16 W_{i+1} - W_{i+2}) / 12, the
 *          boundary closed by odd reflection (W_{-1} = -W_1, W_{n+1} = -W_{n-1});
 *          single-step kernels only, stability c dt / h < sqrt(3 / (4 dim)), no
 *          batched or adjoint solves.
 * Layout.  Every grid function is a nodal array of (n+1)^dim doubles, C order with
 *          x fastest (index (k*(n+1) + j)*(n+1) + i).  Boundary entries of inputs
 *          v, f, u are ignored (read as 0); boundary entries of outputs are written 0.
 *          c2 is nodal including the boundary (boundary faces use it).
 * Memory.  Arrays marked "device" are device pointers on the context's GPU;
 *          "host" are host pointers.  The caller owns every buffer, including the
 *          workspace; the library allocates no device memory (it keeps a small
 *          pinned host block per context for scalar read-backs).
 * Stream.  All device work is enqueued on the context stream.  wh_apply_filter is
 *          asynchronous when params->c_max > 0; solvers block until they return.
 * Errors.  Nothing aborts or throws across the ABI: every entry point that can
 *          allocate host memory catches any C++ exception and returns WH_EHOST.
 *          Negative status: outputs are not valid; WH_ENOCONV: the best iterate is
 *          returned with its residual in wh_info.  wh_last_error() gives a message for
 *          the last failure (with ctx == NULL: the calling thread's last failure of a
 *          call that has no context).
 */
#ifndef WAVEHOLTZ_H
#define WAVEHOLTZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WH_OK = 0,
  WH_ENOCONV = 1,        /* tolerance not met within max_iters / max_outer; result valid */
  WH_EINVAL = -1,        /* bad argument (null pointer, size, range, c2 <= 0)            */
  WH_EUNSUPPORTED = -2,  /* dim not in {2,3}, order != 2, unsupported combination        */
  WH_EHIP = -3,          /* a HIP runtime call failed                                    */
  WH_EWORKSPACE = -4,    /* workspace missing, too small or misaligned (256 B)           */
  WH_EUNSTABLE = -5,     /* wave solve blew up (non-finite), e.g. CFL violated           */
  WH_EBREAKDOWN = -6,    /* Krylov breakdown: p^T A p = 0, zero Arnoldi vector norm      */
  WH_EHOST = -7          /* host-side failure inside the library (memory allocation or an
                            internal exception); caught at the entry point, message in
                            wh_last_error                                                */
} wh_status;

typedef enum { WH_F64 = 0, WH_MIXED = 1 } wh_precision;
typedef enum { WH_FPI = 0, WH_CG = 1, WH_DCG = 2, WH_GMRES = 3, WH_BICGSTAB = 4 } wh_solver;

/* Deflation sets (Section 2.1 "deflation set", Algorithm 3 matrix W). */
typedef enum {
  WH_DEFL_NONE = 0,
  WH_DEFL_SINE = 1,        /* analytic Dirichlet modes (2/n)^{dim/2} prod sin(k pi x) (c == 1 only);
                              the eigenvalues of A on them are known in closed form      */
  WH_DEFL_DENSE_EXACT = 2, /* dense columns that are eigenvectors of L_h with given lambda2 */
  WH_DEFL_DENSE = 3,       /* any dense l2-orthonormal columns (DCG); A W costs n_d wave solves */
  WH_DEFL_FACTORED = 4     /* 2D eigenvectors of L_h with given lambda2, each a sum of separable
                              terms fy_t(y) fx_t(x) (e.g. a truncated SVD of the mode as an
                              (n+1) x (n+1) array, the compression of Section 4.3); projected
                              and combined from the factors without forming the vectors   */
} wh_defl_kind;

typedef struct wh_ctx wh_ctx;

typedef struct {
  int32_t dim;    /* 2 or 3 */
  int32_t n;      /* cells per side, n >= 4 */
  int32_t order;  /* spatial order: 2, or 4 (c == 1) */
} wh_grid;

typedef struct {
  double omega;             /* Helmholtz frequency, > 0                                    */
  int32_t n_periods;        /* N_p >= 1: filter window Tbar = N_p periods (eq. waveHoltzFilter) */
  double cfl;               /* c_max dt / h, 0 < cfl < 1/sqrt(dim); default 0.5             */
  int32_t steps_per_period; /* m; 0: smallest m >= 3 with dt <= cfl h / c_max               */
  int32_t freq_correction;  /* 1 (default): dt = 2 sin(pi/m)/omega, wave solve at
                               omega_tilde = (2 pi/m)/dt, fixed point solves L_h + omega^2;
                               0: dt = 2 pi/(m omega), wave solve at omega                  */
  double c_max;             /* max_x c(x); 0: computed from c2 on the device (one read-back) */
  int32_t precision;        /* wh_precision: WH_MIXED steps the wave equation in FP32 and
                               keeps the filter sum, Krylov and deflation in FP64.  CG/DCG
                               replace their residual by the true FP64 residual each time
                               it has dropped tenfold; GMRES refines FP32 inner solves with
                               FP64 outer residuals.  A problem whose FP32 operator error
                               stalls the true residual continues in FP64.                 */
  int32_t solver;           /* wh_solver                                                    */
  int32_t restart;          /* GMRES restart length (default 40)                            */
  double tol;               /* stop when ||b - A u||_2 / ||b||_2 <= tol                      */
  int32_t max_iters;        /* solver iterations                                            */
  double inner_tol;         /* WH_MIXED, FP32 progress between FP64 residuals: GMRES, the
                               relative tolerance of each FP32 inner restart cycle (0: 1e-3);
                               CG/DCG, the residual reduction after which the recursive
                               residual is replaced by the true one (0: 0.1 for CG, 1e-3
                               for DCG, 1e-4 for deflated batch problems)                   */
  int32_t max_outer;        /* WH_MIXED GMRES: FP64 refinement sweeps (default 30)           */
  int32_t k_fuse;           /* time steps per stencil launch; 0: library choice.  Blocked
                               2D launches take 2, 3, 4, 6, 8 (FP32 also 9), 3D 2 or 3;
                               fourth order in 2D 2 or 4 (0 and values above 4: 4, 3: 2);
                               any other value, fourth order in 3D, or too few steps: one
                               per launch                                                  */
  int32_t reproject;        /* DCG A-orthogonalisation against W each iteration (Algorithm 3,
                               optional for exact eigenvectors): -1 auto (= off, every
                               deflation kind here is exact), 0 off, 1 on                  */
  int32_t check_every;      /* read the residual back every this many iterations (1)        */
  int32_t mixed_form;       /* WH_MIXED A-apply: 0 steps the defect W^n - cos(omega_w t^n) v
                               in FP32, using A v = Pi_h(0; H v) with H = L_h + omega^2
                               (exact under the corrected frequency); 1 steps W^n from
                               W^0 = v in FP32; -1 (default): 0 for CG/GMRES and batched
                               solves, 1 for DCG                                           */
  int32_t devd;             /* with a deflation set: 0 uses it in DCG (Algorithm 3); 1 runs
                               Algorithm 2 (direct eigenvector deflation) around solver FPI,
                               CG or GMRES: f_d = f - W W^T f, solve for f_d, then
                               u += sum_k (phi_k^T f) / (omega^2 - lambda_k^2) phi_k; 2: as 1
                               with every FPI iterate deflated (FPI only).  Exact
                               eigenvectors only (WH_DEFL_SINE, WH_DEFL_DENSE_EXACT,
                               WH_DEFL_FACTORED).  The
                               reported residuals are those of the deflated system.        */
  int32_t k_shape;          /* block shape of the temporally blocked kernel (2D: register rows
                               per thread and waves per block; 3D: also planes per block),
                               0..2; -1 (default): chosen with K by the autotuner           */
} wh_params;

typedef struct {
  int32_t kind;          /* wh_defl_kind                                                   */
  int32_t n_d;           /* number of vectors N_D >= 0 (<= 256)                             */
  const int32_t* modes;  /* host, WH_DEFL_SINE: n_d*dim mode numbers, x first, each 1..n-1   */
  const double* V;       /* device, dense kinds: column-major nodal columns, zero boundary  */
  int64_t ldv;           /* leading dimension of V, >= (n+1)^dim                           */
  const double* lambda2; /* host, WH_DEFL_DENSE_EXACT / FACTORED: lambda_h^2, L_h v = -lambda2 v */
  int32_t n_terms;       /* WH_DEFL_FACTORED: separable terms T, n_d <= T <= 4096           */
  const int32_t* term_mode; /* host, WH_DEFL_FACTORED: T mode indices, nondecreasing, every
                              mode 0..n_d-1 present                                          */
  const double* fx;      /* device, WH_DEFL_FACTORED: T x (n+1) x-factors, row t = term t    */
  const double* fy;      /* device, WH_DEFL_FACTORED: T x (n+1) y-factors (singular values
                              folded in); term t contributes fy_t(y_j) fx_t(x_i) at node (i, j) */
} wh_deflation;

typedef struct {
  int32_t status;          /* wh_status of the call                                         */
  int32_t iters;           /* Krylov / FPI iterations (all inner iterations for WH_MIXED)  */
  int32_t wave_solves;     /* applications of Pi_h in FP64                                  */
  int32_t wave_solves_f32; /* applications of Pi_h with FP32 stepping                       */
  int32_t outer;           /* WH_MIXED: FP64 true-residual evaluations (CG/DCG) or
                               refinement sweeps (GMRES)                                     */
  int32_t nt;              /* time steps per wave solve N_t = N_p m                         */
  int32_t m;               /* steps per period                                              */
  int32_t k_fuse;          /* time steps per stencil launch that was used                   */
  double rel_res;          /* last residual the solver tracked, relative to ||b||           */
  double true_rel_res;     /* ||b - A u|| / ||b|| recomputed with FP64 wave solves at exit   */
  double omega_tilde;      /* frequency used inside the wave solve                          */
  double dt;               /* time step                                                     */
  double c_max;            /* wave speed bound used for the time step                       */
  double ms;               /* wall time of the call in milliseconds                         */
  int32_t k_rows;          /* 2D blocked kernel: register rows per thread (0: streaming);
                              batched solver: rows per tile of its row-marching kernel      */
  int32_t k_waves;         /* 2D blocked kernel: wavefronts per block (0: streaming)        */
} wh_info;

typedef struct {
  wh_grid grid;
  const double* c2;   /* device, nodal; NULL means c == 1                                   */
  const double* f;    /* device, nodal source                                               */
  double omega;       /* overrides common->omega                                            */
  double* u;          /* device, nodal; in: initial guess, out: solution                    */
  int32_t n_defl;     /* wh_solve_batched with WH_DCG: deflate the n_defl analytic sine modes
                         whose eigenvalues lie nearest omega^2 (c == 1 only); 0: none       */
} wh_problem;

/* ------------------------------------------------------------------ context */
void wh_params_default(wh_params* p);
/* Create a context bound to HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the default stream).  The stream must outlive the context. */
wh_status wh_create(wh_ctx** ctx, int device, void* hip_stream);
wh_status wh_destroy(wh_ctx* ctx);
wh_status wh_set_stream(wh_ctx* ctx, void* hip_stream);
/* Message of the last failure on ctx; with ctx == NULL, of the calling thread's last failed
 * wh_create. */
const char* wh_last_error(const wh_ctx* ctx);
const char* wh_status_string(wh_status s);

/* The wave speed bound c_max = sqrt(max c2) of a nodal coefficient array (device, float64,
 * (n+1)^dim nodes, the layout of wh_apply_filter's c2) that fixes the CFL time step of
 * Section 2.2; every node must hold a finite c2 > 0 (WH_EINVAL otherwise).  Two reductions
 * on the context's stream into the context's own device buffer, then a synchronous
 * read-back into *c_max (host).  c2 == NULL means c == 1 and returns 1. */
wh_status wh_coeff_bound(wh_ctx* ctx, const wh_grid* grid, const double* c2, double* c_max);

/* ------------------------------------------------------------------ host helpers */
/* Time step, steps per period, N_t and adjusted frequency for given c_max (Section 2.2). */
wh_status wh_time_params(const wh_grid* grid, const wh_params* params, double c_max,
                         int32_t* m, int32_t* nt, double* dt, double* omega_tilde);
/* beta_h(lambda2) = sum_n w_n T_n(1 - lambda2 dt^2/2): the eigenvalue of S_h on an
 * eigenvector of L_h with L_h v = -lambda2 v (Section 2.3, eq. beta_fun, discrete form).
 * lambda2 and beta are host arrays of length count. */
wh_status wh_transfer(const wh_grid* grid, const wh_params* params, double c_max,
                      int32_t count, const double* lambda2, double* beta);
/* The n_d analytic Dirichlet modes whose discrete eigenvalue lambda2 (of the operator
 * of this order, 2 or 4) is nearest to omega^2 (Section 2.3: deflate the eigenvectors
 * with eigenvalues closest to omega), ties broken lexicographically by the mode
 * numbers.  modes: host n_d*dim ints, lambda2: host n_d doubles (may be NULL). */
wh_status wh_select_sine_modes(int32_t dim, int32_t n, int32_t order, double omega, int32_t n_d,
                               int32_t* modes, double* lambda2);

/* ------------------------------------------------------------------ workspace */
/* Bytes of device workspace (256-byte aligned base) needed by wh_apply_filter and
 * wh_solve with these arguments (defl may be NULL). */
size_t wh_workspace_bytes(const wh_grid* grid, const wh_params* params, const wh_deflation* defl);

/* ------------------------------------------------------------------ operations */
/* v_out = Pi_h(v_in; f): one wave solve over N_p periods with the trapezoid filter
 * (eq. WaveHoltzDiscreteFPI).  f == NULL gives S_h v_in; c2 == NULL means c == 1.
 * v_in, v_out, f, c2: device nodal; v_in and v_out must not overlap. */
wh_status wh_apply_filter(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                          const double* v_in, double* v_out, const wh_params* params,
                          void* ws, size_t ws_bytes, wh_info* info);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): wh_apply_filter without a workspace argument.  The
 * state pairs, scaled coefficients, partial sums and scalars live in a fixed device array
 * inside the library (64 MiB, one copy per GPU, held until the process ends; its address is
 * looked up once per device by wh_create).  Grids whose buffers exceed it are rejected with
 * WH_EWORKSPACE and the size they need (2D: up to about 1024^2 cells; 3D: about 100^3).  No
 * device or pinned memory is allocated and no timing runs: the steps per launch are
 * params->k_fuse / k_shape, else the autotuner's cached choice for this grid from an earlier
 * call of another entry point, else 8 (2D) or 3 (3D) with the default block shape (fourth
 * order: the choice wh_params.k_fuse describes).  With
 * params->c_max > 0 the call is asynchronous on the context stream and host-synchronisation
 * free; c_max = 0 reads the computed maximum of c back.  Every call on one GPU shares that
 * GPU's array and the array keeps the last call's contents: calls that overlap on one GPU
 * (two streams, two threads, two contexts) race.  v_in, v_out, f, c2 as in wh_apply_filter. */
wh_status wh_apply_filter_noalloc(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                                  const double* v_in, double* v_out, const wh_params* params,
                                  wh_info* info);

/* Solve A u = b, b = Pi_h(0; f), by params->solver; the fixed point is the discrete
 * Helmholtz solution (L_h + omega^2) u = f (Sections 2.1-2.2).  u: device nodal, in:
 * initial guess, out: solution.  defl is required for WH_DCG (Algorithm 3): exact
 * eigenvectors (sine, dense-exact, factored) or, with WH_DEFL_DENSE, any l2-orthonormal
 * columns, for which A W is formed by n_d FP64 wave solves before the iteration, (W^T A W)^{-1}
 * is formed on the host from the symmetrised projections, and every iteration re-projects
 * (eta = (A W)^T r, mu = (W^T A W)^{-1} eta, p = beta p + r - W mu).  Exact eigenvectors also
 * augment WH_GMRES (Algorithm 4: W heads the Arnoldi basis, A W =
 * W diag(mu)) and WH_BICGSTAB (Algorithm 5: the thin QR of A W is W diag(mu), every
 * A-product is projected off W and the W part of the solution is recovered at the
 * end), or with params->devd wraps FPI / CG / GMRES / BiCGStab in Algorithm 2; else
 * NULL.  WH_BICGSTAB without defl is plain BiCGStab; in mixed precision it runs FP32
 * inner solves inside FP64 residual refinement, like WH_GMRES. */
wh_status wh_solve(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                   const wh_deflation* defl, const wh_params* params, double* u,
                   void* ws, size_t ws_bytes, wh_info* info);

/* Relative discrete Helmholtz residual ||f - (L_h + omega^2) u|| / ||f|| over the
 * interior (eq. discreteHelmholtz); result written to *rel (host). */
wh_status wh_helmholtz_residual(wh_ctx* ctx, const wh_grid* grid, const double* c2,
                                const double* f, double omega, const double* u,
                                void* ws, size_t ws_bytes, double* rel);

/* Bytes of device workspace needed by wh_solve_batched for these problems. */
size_t wh_workspace_bytes_batched(int32_t nb, const wh_problem* probs, const wh_params* params);

/* Solve nb independent 2D problems (1 <= nb <= 4096; grids of any size 4 <= n <= 16000, own
 * omega, source and optional c2) with CG on the WaveHoltz system, in one device-driven batch: every
 * problem's wave solves and Krylov updates are advanced by shared launches captured
 * in a hipGraph (the paper's motivation of many right-hand sides and frequencies,
 * Section 1).  params->solver WH_CG: Algorithm 3 without deflation.  WH_DCG:
 * Algorithm 3 with each problem's n_defl sine modes nearest omega^2 as the
 * deflation set (exact eigenvectors for c == 1, so the start x_0 = W (W^T A W)^{-1}
 * W^T b is computed from the projections of f, and the iteration needs no
 * re-projection); problems with n_defl == 0 run plain CG.  probs: host array; each
 * problem's omega overrides params->omega; u is output only (batched solves start
 * from zero, or from x_0).  All problems must have c2 or none; with c2,
 * params->c_max must bound c and n_defl must be 0.  params->k_fuse in {2, 4, 8}
 * sets the time steps per launch (0: 4).  Every problem's grid must have the same order: 2,
 * or 4 (fourth-order differences, c == 1 only; a launch then advances k_fuse / 2 steps, whose
 * halo of 2 points per step keeps the tiles of k_fuse second-order steps; the sine modes and
 * their eigenvalues are those of the fourth-order operator).  infos: host array of nb (may be
 * NULL).  Returns the worst status over problems. */
wh_status wh_solve_batched(wh_ctx* ctx, int32_t nb, const wh_problem* probs,
                           const wh_params* params, void* ws, size_t ws_bytes, wh_info* infos);

/* Measurement helper of the batched solver: the average duration in microseconds of one launch
 * of its FP32 work kernel (the K-step register-tiled leapfrog + filter sweep over every tile of
 * every problem) with every problem of the batch in the FP32 time-stepping phase of an A-apply,
 * over `reps` back-to-back launches on the context stream between two HIP events.  *points
 * (may be NULL) receives the interior points one launch advances by K steps, sum (n-1)^2.
 * Arguments and workspace as for wh_solve_batched with params->precision = WH_MIXED (the
 * workspace contents are overwritten; every problem needs N_t >= K + 2; second-order grids
 * only, else WH_EUNSUPPORTED).  The launches carry a
 * kernel tag of their own, so that profiles list them apart from the solver's launches. */
wh_status wh_time_batch_kernel(wh_ctx* ctx, int32_t nb, const wh_problem* probs, const wh_params* params,
                               int32_t reps, void* ws, size_t ws_bytes, double* us_per_launch, int64_t* points);

/* ------------------------------------------------------------------ gradient (2D) */
/* Workspace for wh_solve_vjp / wh_adjoint_grad (params->c_max > 0 required). */
size_t wh_workspace_bytes_adjoint(const wh_grid* grid, const wh_params* params, int32_t ckpt_every);

/* grad_c2 += (d Pi_h / d c2)^T A^{-1} grad_u at the fixed point u = Pi_h(u; f, c2): the
 * vector-Jacobian product of the map c2 -> u (Sections 2.1-2.2: u solves A u = b, so
 * du/dc2 = A^{-1} dPi_h/dc2).  A^{-1} grad_u is one CG solve (A is symmetric); the
 * product with (dPi_h/dc2)^T runs the time-reversed, transposed leapfrog recurrence
 * with the trapezoid weights as its source, recomputing the forward trajectory from
 * checkpoints kept every ckpt_every steps (0: 16).  2D only; c2 required (device,
 * nodal); params->c_max must bound c; u, grad_u, f device nodal; grad_c2 device nodal
 * (all nodes, accumulated).  The time step is held fixed: the fixed point does not
 * depend on it under the corrected frequency. */
wh_status wh_solve_vjp(wh_ctx* ctx, const wh_grid* grid, const double* c2, const double* f,
                       const double* u, const double* grad_u, const wh_params* params,
                       int32_t ckpt_every, double* grad_c2, void* ws, size_t ws_bytes,
                       wh_info* info);

/* Receiver misfit J = 1/2 sum_s ||R u_s - d_s||^2 over n_src sources and its gradient
 * dJ/dc2 (overwrites grad_c2).  f: host array of n_src device source pointers;
 * rec_idx: device array of n_rec nodal linear indices (interior nodes, checked);
 * d: device n_src x n_rec data; J: host.  Each source costs two CG solves and one
 * checkpointed reverse sweep.  grad_c2 == NULL evaluates J alone (one CG solve per
 * source), as a finite-difference check of the gradient needs. */
wh_status wh_adjoint_grad(wh_ctx* ctx, const wh_grid* grid, const double* c2, int32_t n_src,
                          const double* const* f, int32_t n_rec, const int64_t* rec_idx,
                          const double* d, const wh_params* params, int32_t ckpt_every,
                          double* grad_c2, double* J, void* ws, size_t ws_bytes, wh_info* info);

/* Measurement helper: the average duration in microseconds of one launch of the
 * time-stepping kernel that wh_apply_filter / wh_solve would use for these
 * arguments (the K-step temporally blocked kernel, or the single-step kernel when
 * K = 1), with no forcing.  `reps` launches run back to back on the context stream
 * between two HIP events; *k_used receives K, and (each pointer may be NULL)
 * *rows / *waves the register rows per thread and wavefronts per block of the
 * blocked kernel (0 for the single-step kernel).  The state arrays in the workspace
 * are zeroed first and overwritten; nothing else is touched. */
wh_status wh_time_step_kernel(wh_ctx* ctx, const wh_grid* grid, const double* c2,
                              const wh_params* params, int32_t reps, void* ws, size_t ws_bytes,
                              double* us_per_launch, int32_t* k_used, int32_t* rows,
                              int32_t* waves);

#ifdef __cplusplus
}
#endif
#endif /* WAVEHOLTZ_H */
