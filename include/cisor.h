/*
 * cisor.h -- C ABI of the MI355X (gfx950) CISOR hot-path library.
 *
 * CISOR (arXiv 1708.01663) reconstructs a real permittivity contrast f from
 * scattered-field measurements y by minimising F(f) = D(f) + R(f), with
 *   D(f) = 1/2 sum_t ||y_t - H diag(u_t) f||^2,   u_t = A^{-1} u_in,t,
 *   A    = I - G diag(f)                          (eqs. D_def, Z_def, A_def)
 *   R(f) = tau TV_iso(f) + indicator of a box     (eq. R_def)
 * using relaxed FISTA (eqs. algo1-algo3) and the adjoint gradient of Prop. 1.
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Pointers documented as "device" point to GPU memory owned by the caller;
 *    "host" pointers to CPU memory owned by the caller.  The library never
 *    frees caller memory.  The context owns its own device buffers (Green's
 *    kernel spectrum, receiver matrix H, incident fields, solver workspaces).
 *  - Element types follow the context precision chosen at creation:
 *      precision 0: real = float,  complex = interleaved float  {re, im}
 *      precision 1: real = double, complex = interleaved double {re, im}
 *    Norms, inner products, the misfit D and the solver stop test are always
 *    accumulated in FP64.
 *  - 2D grids: pixel q = i*n + j sits at ((i-(n-1)/2) h, (j-(n-1)/2) h),
 *    N = n*n.  3D grids: voxel q = (i*n + j)*n + l sits at
 *    ((i-(n-1)/2) h, (j-(n-1)/2) h, (l-(n-1)/2) h), N = n*n*n.
 *    Fields are transmitter-major [T][N]; data are [T][M].
 *  - All calls enqueue on the context's HIP stream.  Calls that return host
 *    values (iteration counts, D) synchronise that stream before returning.
 *  - Return codes: CISOR_OK, or CISOR_NOT_CONVERGED (soft: every output is
 *    written, some solve hit maxit), or a negative error.  Invalid arguments
 *    are rejected with CISOR_E_ARG before anything is launched.
 *  - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef CISOR_H
#define CISOR_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cisor_ctx cisor_ctx;

enum {
  CISOR_OK = 0,
  CISOR_NOT_CONVERGED = 1,   /* soft: outputs written, a solve reached maxit */
  CISOR_E_ARG = -1,          /* invalid size, null pointer, bad option */
  CISOR_E_NOMEM = -2,        /* device allocation failed */
  CISOR_E_DEVICE = -3,       /* HIP runtime error */
  CISOR_E_NONFINITE = -4,    /* NaN/Inf met in an FP64 reduction */
  CISOR_E_UNSUPPORTED = -6,  /* no compiled FFT length for the grid, or a configuration
                                the call does not implement (stated per call) */
  CISOR_E_SIZE = -7          /* the problem exceeds the fixed static work area of a
                                non-allocating call (cisor_tv_prox_noalloc) */
};

/* Scattering geometry ("Problem Formulation"; discrete system of eqs.
 * discrete2D_measurement / discrete2D_constraint).  Lengths share one unit
 * (e.g. wavelengths).  The library builds, in FP64 on the host:
 *  - incident fields: plane waves u_in,t(r) = exp(i k_b dir_t . r), k_b = k sqrt(eps_b)
 *    (tx_kind 0), or unit point sources at pos_t (tx_kind 1), the background
 *    Green's function u_in,t(r) = (i/4) H0(k_b |r - pos_t|) in 2D and
 *    exp(i k_b d)/(4 pi d), d = |r - pos_t|, in 3D, sampled at the cell centres;
 *  - G: the Green's convolution on the grid, each pixel replaced by the
 *    equal-area disk, so G[p,q] = K(|r_p - r_q|) with
 *      K(0)   = ((i pi/2) k_b a H1(k_b a) - 1) / eps_b,
 *      K(rho) = (i pi/2) k_b a J1(k_b a) H0(k_b rho) / eps_b,  a = h/sqrt(pi)
 *    (outgoing Hankel functions of the first kind; H0 is (i/4)H0 times k^2
 *    integrated over the cell).  In 3D each voxel is replaced by the
 *    equal-volume ball, a = h (3/(4 pi))^(1/3), and the scalar Green's
 *    function exp(i k_b d)/(4 pi d) of the 3D form of eq. green gives
 *      K(0) = ((1 - i k_b a) exp(i k_b a) - 1) / eps_b,
 *      K(d) = (4 pi / k_b) (sin k_b a - k_b a cos k_b a) exp(i k_b d)/(4 pi d) / eps_b.
 *    G is stored as the spectrum of its embedding on the P^dim circulant
 *    grid (P >= 2n, below);
 *  - H[m,q] = K(|r_m - r_q|), the same cell integral evaluated at receiver m. */
typedef struct {
  int dim;                 /* 2 or 3 */
  int n;                   /* grid side, 2 <= n <= 512; the FFT length P is the smallest of
                              64, 128, 192, 256, 384, 512, 768, 1024 that is >= 2n.  A 3D
                              context holds P^3 spectrum values and T*n*P^2 intermediates,
                              so device memory bounds n there (n = 64: P = 128) */
  double h;                /* pixel size */
  double wavelength;       /* vacuum wavelength (k = 2 pi / wavelength) */
  double eps_b;            /* background permittivity (> 0) */
  int T;                   /* transmitters, >= 1 */
  int M;                   /* receivers, >= 1 */
  const double *tx_dir;    /* host, [T][dim] propagation directions (normalised by the library);
                              tx_kind 0 only (may be NULL otherwise) */
  const double *rx_pos;    /* host, [M][dim] receiver positions, outside every grid cell */
  int precision;           /* 0 = complex64 fields, 1 = complex128 fields */
  int tx_kind;             /* 0 = plane waves (tx_dir), 1 = point sources (tx_pos) */
  const double *tx_pos;    /* host, [T][dim] source positions, strictly outside the grid's
                              square/cube [-n h/2, n h/2]^dim; tx_kind 1 only */
} cisor_geometry;

/* Options of the Lippmann-Schwinger solves A u = b and A^H v = b (eq.
 * u_and_v).  The solver is BiCGSTAB batched over transmitters; a system is
 * converged when its true relative residual ||b - A x|| / ||b||, evaluated
 * with an FP64 operator, is <= tol. */
typedef struct {
  double tol;              /* target true relative residual, > 0 */
  int maxit;               /* iteration cap per system, >= 1 */
  int start;               /* 0: x0 = 0, 1: x0 = b (first-Born start), 2: x0 given in the output buffer,
                              3: per system, the given x0 or the first-Born x0 = b, whichever has the
                              smaller FP64 true residual (cisor_get_start_choice reports which),
                              4: cisor_fista_step only (CISOR_E_ARG elsewhere): the previous fields
                              extrapolated along the FISTA path (see cisor_fista_step),
                              5: not for cisor_fista_step: per system, the given x0, or x0 = 0 where the
                              starting residual of x0 (in the field precision) is larger than ||b||,
                              the zero start's residual (so the check costs no operator application;
                              cisor_get_start_choice reports 1 where the zero start was taken) */
  int replace_every;       /* FP64 residual replacement period in iterations (0: 50); a running
                              system's residual is also replaced at the next poll once its
                              recurrence residual has fallen ~31.6x below its largest value since
                              the last replacement */
  int check_every;         /* host convergence poll period in iterations (0: 10); the first poll
                              of a solve comes one iteration after the most any system needed in
                              the context's last solve of the same kind (forward / adjoint), if
                              that is sooner, and the polls after it come 2, 4, 8 iterations
                              apart before the period applies */
} cisor_ls_opts;

/* Relaxed-FISTA state (eqs. algo1-algo3).  f, f_prev, s: device real [N].
 * t: the scalar t_k (start at 1); k: completed iterations (start at 0). */
typedef struct {
  void *f;
  void *f_prev;
  void *s;
  double t;
  int k;
} cisor_fista_state;

/* Host-side report of one relaxed-FISTA iteration. */
typedef struct {
  double D;                /* misfit D(s_k) in FP64 */
  int fwd_iters_max, adj_iters_max;
  long long fwd_iters_sum, adj_iters_sum;
  double max_true_relres;  /* largest final true relative residual of the solves */
  int status;              /* worst status of the solves */
} cisor_step_info;

/* Create a context for a geometry; stream is a hipStream_t (NULL = default
 * stream).  Builds u_in, G's spectrum and H.  On success *out owns them. */
int cisor_create(const cisor_geometry *geom, void *stream, cisor_ctx **out);
int cisor_destroy(cisor_ctx *ctx);
int cisor_set_stream(cisor_ctx *ctx, void *stream);
/* Sizes: N, T, M, padded FFT length P, precision. Any pointer may be NULL. */
int cisor_get_sizes(const cisor_ctx *ctx, int *N, int *T, int *M, int *P, int *precision);

/* Copy the incident fields u_in (device complex [T][N]) into a caller buffer. */
int cisor_get_uin(cisor_ctx *ctx, void *u_in);
/* Copy the receiver matrix H (device complex [M][N], row-major). */
int cisor_get_H(cisor_ctx *ctx, void *H);

/* Forward model (eqs. discrete2D_constraint, Z_def): solve A u_t = u_in,t for
 * every t and, if y != NULL, project y_t = H diag(u_t) f.
 *   f: device real [N]; u: device complex [T][N] (x0 on entry if start == 2);
 *   y: device complex [T][M] or NULL; iters: host int [T] or NULL. */
int cisor_forward(cisor_ctx *ctx, const void *f, void *u, void *y,
                  const cisor_ls_opts *opts, int *iters);

/* Gradient of D at f by Prop. 1 (eqs. gradient, u_and_v):
 *   u_t = A^{-1} u_in,t;  w_t = H diag(u_t) f - y_t;  q_t = H^H w_t;
 *   v_t = A^{-H} diag(f) q_t;  grad = sum_t Re{conj(u_t) (q_t + G^H v_t)}.
 *   f: device real [N]; y_meas: device complex [T][M]; grad: device real [N];
 *   D: host double or NULL (receives 1/2 sum ||w_t||^2 in FP64);
 *   u_ws, v_ws: device complex [T][N] holding u and v on return (and the
 *   starting guesses on entry when opts->start == 2);
 *   iters: host int [2T] (forward then adjoint) or NULL. */
int cisor_grad(cisor_ctx *ctx, const void *f, const void *y_meas, void *grad, double *D,
               void *u_ws, void *v_ws, const cisor_ls_opts *opts, int *iters);

/* Vector-Jacobian product of the data map f -> y (y_t = H diag(u_t) f with
 * u_t = A^{-1} u_in,t): given the total fields u of a forward solve at f and a
 * data-space cotangent w (for a real loss L(y), w = dL/dRe y + i dL/dIm y),
 * returns grad = Re{J^H w} = sum_t Re{conj(u_t) (H^H w_t + G^H v_t)} with
 * A^H v_t = diag(f) H^H w_t.  This is the computation in the proof of Prop. 1
 * with w in place of the residual; with w = Z(f) - y it is grad D.
 *   f: device real [N]; u: device complex [T][N] (the forward fields at f);
 *   w: device complex [T][M]; grad: device real [N]; v_ws: device complex
 *   [T][N] holding v on return (the starting guess if opts->start == 2);
 *   iters: host int [T] or NULL (adjoint iterations). */
int cisor_vjp(cisor_ctx *ctx, const void *f, const void *u, const void *w, void *grad, void *v_ws,
              const cisor_ls_opts *opts, int *iters);

/* First-Born scattered fields (the right-hand side's first Neumann term of
 * eq. discrete2D_constraint): u_b,t = G diag(f) u_in,t = u_in,t - A u_in,t for
 * every transmitter, one convolution launch sequence.  f: device real [N];
 * u_b: device complex [T][N].  2D and 3D contexts. */
int cisor_born_field(cisor_ctx *ctx, const void *f, void *u_b);

/* Proximal map of lam * TV_iso + box (eq. R_def, used in eq. algo1 with
 * lam = gamma * tau): x = argmin_{lo <= x <= hi} 1/2 ||x - z||^2 + lam TV(x),
 * computed by the fast gradient projection method on the dual (Beck and
 * Teboulle 2009) with inner_iters iterations from a zero dual.  Forward
 * differences with a zero last difference (Neumann boundary).
 *   z, x: device real [N] (may alias).  lam >= 0, lo <= hi, inner_iters >= 0.
 * 2D and 3D contexts (in 3D the dual lives on the three axes of the volume and
 * the dual step is 1 / (12 lam) instead of 1 / (8 lam)). */
int cisor_tv_prox(cisor_ctx *ctx, const void *z, void *x, double lam, double lo, double hi,
                  int inner_iters);

/* The same proximal map without a context and without any device allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).  Same
 * kernels, same arithmetic and so the same result as cisor_tv_prox on a
 * context of that grid and precision.  Its work area (9 N reals: a copy of z
 * and the FGP duals) is a fixed static device array of
 * CISOR_TV_NOALLOC_SCRATCH_BYTES held by each GPU the library runs on until
 * the process ends; the library looks up its device address on the first call
 * on each device (with that device current) and zeroes what must start at zero
 * on every call.  All calls on one GPU share that array, so calls that overlap
 * in time on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.
 *   dim: 2 or 3; n: grid side (N = n^2 or n^3 <= CISOR_TV_NOALLOC_MAX_N, i.e.
 *   up to 512^2 or 64^3, else CISOR_E_SIZE before anything is launched);
 *   precision: 0 float, 1 double; z, x: device real [N] (may alias);
 *   lam >= 0, lo <= hi, inner_iters >= 0 as for cisor_tv_prox;
 *   stream: hipStream_t of the current device (NULL = default stream).
 * Asynchronous on the stream; invalid arguments give CISOR_E_ARG. */
#define CISOR_TV_NOALLOC_MAX_N 262144
#define CISOR_TV_NOALLOC_SCRATCH_BYTES (9ull * CISOR_TV_NOALLOC_MAX_N * 8ull)
int cisor_tv_prox_noalloc(int dim, int n, int precision, const void *z, void *x, double lam, double lo,
                          double hi, int inner_iters, void *stream);

/* Receivers used by each transmitter's data (the paper's experiments switch
 * off the receivers near the active transmitter): mask host [T][M], nonzero =
 * active; NULL makes every receiver active again.  With a mask, the misfit
 * D = 1/2 sum_t ||mask_t (Z_t(f) - y_t)||^2 and everything built on w = Z(f) -
 * y (the gradient's adjoint right-hand sides, the FISTA step, the projection
 * with measured data) use the active receivers only; predicted data y = Z(f)
 * are still written for every receiver.  Kept until changed; 2D and 3D. */
int cisor_set_rx_mask(cisor_ctx *ctx, const unsigned char *mask);

/* Isotropic total variation of eq. R_def, TV(x) = sum_q ||(grad x)_q||_2 with
 * forward differences and a zero last difference (the discretisation the prox
 * uses), summed in FP64; used for the objective F = D + tau TV of eq.
 * objective_func.  x: device real [N]; tv: host double.  Synchronises the
 * context stream.  2D and 3D contexts. */
int cisor_tv_value(cisor_ctx *ctx, const void *x, double *tv);

/* One relaxed-FISTA iteration (eqs. algo1-algo3):
 *   f_k = prox_{gamma R}(s_k - gamma grad D(s_k)); t_{k+1} = (sqrt(4 t_k^2 + 1) + 1)/2;
 *   s_{k+1} = f_k + alpha (t_k - 1)/t_{k+1} (f_k - f_{k-1}).
 * state is updated in place (f_prev <- f_k-1, f <- f_k, s <- s_k+1, t, k).
 * The context keeps the last total and adjoint fields and uses them as
 * starting guesses of the next iteration's solves when opts->start == 2.
 * With opts->start == 4 it also keeps the fields and evaluation point of the
 * iteration before, and starts the solves at s_k from the secant
 *   x0 = x(s_{k-1}) + theta (x(s_{k-1}) - x(s_{k-2})),
 *   theta = <s_k - s_{k-1}, s_{k-1} - s_{k-2}> / ||s_{k-1} - s_{k-2}||^2 in [0, 2]
 * (FP64 sums, computed on the device), for the total and the adjoint fields;
 * the first iteration (state->k == 0) starts from the first-Born guess and the
 * second from the previous fields.  Two more field arrays [T][N] are
 * allocated on the first such call.  The solutions do not depend on the start
 * (the stop test is on the FP64 true residual); only the iteration counts do.
 * 2D and 3D contexts (the prox takes the context's dimension). */
int cisor_fista_step(cisor_ctx *ctx, cisor_fista_state *state, const void *y_meas,
                     double gamma, double tau, double alpha, double lo, double hi,
                     int inner_iters, const cisor_ls_opts *opts, cisor_step_info *info);

/* ---- monotone APG (Li and Lin), the comparison method of "Proposed Method" ----
 * The paper contrasts relaxed FISTA with this method, which keeps the better
 * of an accelerated and a plain proximal-gradient estimate at every iteration
 * and so evaluates the gradient at two points and the objective at two more.
 * One iteration (t_0 = 0, t_1 = 1, x_0 = x_1 = z_1 on the first call):
 *   y_k     = x_k + (t_{k-1}/t_k)(z_k - x_k) + ((t_{k-1} - 1)/t_k)(x_k - x_{k-1})
 *   z_{k+1} = prox_{gamma_y R}(y_k - gamma_y grad D(y_k))
 *   v_{k+1} = prox_{gamma_x R}(x_k - gamma_x grad D(x_k))
 *   t_{k+1} = (sqrt(4 t_k^2 + 1) + 1) / 2
 *   x_{k+1} = z_{k+1} if F(z_{k+1}) <= F(v_{k+1}) else v_{k+1}
 * with R and its prox as in cisor_fista_step and F = D + tau TV (box implied).
 * Costs per iteration: two gradient evaluations (forward and adjoint solves
 * at y_k and x_k) and two forward solves (F at z and v).  Solves after the
 * first start from the nearest fields already computed (the gradient at x_k
 * from the fields of the objective evaluation that selected x_k); opts->start
 * (0 zero, 1 first Born, 2 the context's last fields) applies to the first
 * gradient of a run.  2D and 3D contexts. */
typedef struct {
  void *x;          /* device real [N]: x_k (x_1 = x_0 on the first call) */
  void *x_prev;     /* device real [N]: x_{k-1} */
  void *z;          /* device real [N]: z_k (z_1 = x_1) */
  double t, t_prev; /* t_k and t_{k-1}: 1 and 0 on the first call */
  int k;            /* iterations done (0 on the first call) */
} cisor_apg_state;
typedef struct {
  double F;                  /* F(x_{k+1}) = min(F_z, F_v) */
  double F_z, F_v;           /* F at the accelerated and the proximal-gradient estimate */
  double D_y, D_x;           /* D at y_k and at x_k */
  int took_z;                /* 1 when x_{k+1} = z_{k+1} */
  int fwd_solves, adj_solves;  /* solve passes over all T transmitters in the step */
  long long fwd_iters_sum, adj_iters_sum;
  double max_true_relres;
  int status;                /* worst status of the solves */
} cisor_apg_info;
int cisor_apg_step(cisor_ctx *ctx, cisor_apg_state *state, const void *y_meas, double gamma_y, double gamma_x,
                   double tau, double lo, double hi, int inner, const cisor_ls_opts *opts, cisor_apg_info *info);

/* ---- lower-level entry points (used by tests and the autograd binding) ---- */

/* y = A x (adjoint = 0) or y = A^H x (adjoint = 1) for all T fields at once
 * (eq. A_def).  f: device real [N]; x, y: device complex [T][N], no aliasing. */
int cisor_apply_A(cisor_ctx *ctx, const void *f, const void *x, void *y, int adjoint);

/* One of the three launches that make up cisor_apply_A, for timing and
 * profiling: stage 1 = contrast product and forward row FFTs (reads f, x;
 * writes the context's intermediate X1), stage 2 = column FFTs, kernel
 * spectrum product and inverse column FFTs (X1 -> X2), stage 3 = inverse row
 * FFTs and y = x - (.) (reads X2, f, x; writes y).  Running stages 1, 2, 3 in
 * order equals cisor_apply_A.  Unused pointers may be NULL (stage 2 reads
 * none).  2D contexts only (CISOR_E_UNSUPPORTED in 3D). */
int cisor_apply_A_stage(cisor_ctx *ctx, const void *f, const void *x, void *y, int adjoint,
                        int stage);

/* Solve A x_t = b_t (adjoint = 0) or A^H x_t = b_t (adjoint = 1) for all t.
 * b, x: device complex [T][N]; iters: host int [T] or NULL. */
int cisor_solve(cisor_ctx *ctx, const void *f, const void *b, void *x, int adjoint,
                const cisor_ls_opts *opts, int *iters);

/* Receiver projection y_t = H diag(u_t) f (eq. Z_def).  u: device complex
 * [T][N]; y: device complex [T][M].  If y_meas != NULL, y is replaced by the
 * residual w = H diag(u) f - y_meas and *D (host, may be NULL) receives
 * 1/2 ||w||^2 in FP64. */
int cisor_project(cisor_ctx *ctx, const void *f, const void *u, const void *y_meas, void *y,
                  double *D);

/* Back-projection q_t = H^H w_t (the adjoint of the projection, used in eq.
 * u_and_v).  w: device complex [T][M]; q: device complex [T][N]. */
int cisor_backproject(cisor_ctx *ctx, const void *w, void *q);

/* Lipschitz constant of the first-Born misfit gradient,
 * lambda_max(v -> sum_t Re{conj(u_in,t) H^H H (u_in,t v)}), by power
 * iteration from a seeded start (used to choose the FISTA step). */
int cisor_born_lipschitz(cisor_ctx *ctx, int iters, double *L);

/* After a solve with start == 3 (or 5): choice (host int [T]) receives 1 for
 * the systems that fell back to the first-Born start (the zero start), 0
 * where the given guess was kept.  Synchronises the context stream. */
int cisor_get_start_choice(cisor_ctx *ctx, int *choice);

/* ---- launch tuning ----
 * The 2D column stage of the operator (the launch that moves the most data)
 * has 10 compiled variants: 0..3 spread each column transform over a block
 * (two radix factorisations of the transform length times two tile shapes),
 * 4 and 5 keep each column transform inside one wave (two factorisations),
 * 6 and 7 are the tile of 0 with scalar-offset buffer access and per-pass
 * twiddle tables (two factorisations), 8 and 9 run 6's transforms with 8
 * points per thread on 8 columns per block (tiles sharing a 128-byte line on
 * one XCD) or 16 (transform lengths with a factor 3 use 6).  All give the
 * same result up to rounding order.  FP64 contexts use variant 0 only. */
/* Time `reps` launches of each variant on the context's buffers and keep the
 * fastest.  variant: host int or NULL (chosen variant); times_ms: host float
 * [10] or NULL (mean time per launch, -1 where not timed).  Synchronises. */
int cisor_autotune(cisor_ctx *ctx, int reps, int *variant, float *times_ms);
/* Select a column variant explicitly (0..9; CISOR_E_ARG otherwise). */
int cisor_set_col_variant(cisor_ctx *ctx, int variant);

/* ---- batched reconstructions of many problems with uneven sizes ----
 * Not a separate method: relaxed FISTA (eqs. algo1-algo3) with the Prop. 1
 * gradient run on `count` independent problems that step together.  Problems
 * with the same grid (n, h, wavelength, eps_b) share one kernel spectrum and
 * are solved as one stacked set of fields, so each operator launch covers
 * every transmitter of every problem of that grid; different grids run
 * concurrently on their own streams.  The solver iterations, and the
 * projection / prox parts of a step, are replayed as captured HIP graphs.
 * The batch owns every buffer (one device arena), including each problem's
 * FISTA state f, f_prev, s and its measurements.  All geometries must be 2D
 * with the same precision. */
typedef struct cisor_batch cisor_batch;
/* geoms: host array [count] (each as for cisor_create).  Builds u_in and H
 * per problem and one spectrum per distinct grid. */
int cisor_batch_create(const cisor_geometry *geoms, int count, void *stream, cisor_batch **out);
int cisor_batch_destroy(cisor_batch *batch);
int cisor_batch_set_stream(cisor_batch *batch, void *stream);
/* Sizes of problem p (any pointer may be NULL); group: index of its grid. */
int cisor_batch_get_sizes(const cisor_batch *batch, int p, int *N, int *T, int *M, int *P, int *group);
int cisor_batch_num_groups(const cisor_batch *batch, int *groups);
/* Measurements y_meas (device complex [T][M], copied) and the step size gamma
 * > 0 and TV weight tau >= 0 of problem p; resets its state to f = f_prev =
 * s = 0, t = 1, k = 0.  Every problem must be set before a step. */
int cisor_batch_set_problem(cisor_batch *batch, int p, const void *y_meas, double gamma, double tau);
/* One relaxed-FISTA iteration of every problem (as cisor_fista_step, with
 * the previous iteration's fields as starting guesses when opts->start == 2,
 * extrapolated along each problem's own path of evaluation points when
 * opts->start == 4).  info: host [count] or NULL. */
int cisor_batch_fista_step(cisor_batch *batch, double alpha, double lo, double hi, int inner_iters,
                           const cisor_ls_opts *opts, cisor_step_info *info);
/* Copy the current iterate f_k of problem p (device real [N]). */
int cisor_batch_get_f(cisor_batch *batch, int p, void *f);
/* Forward model of every problem at once (as cisor_forward): f: host array
 * [count] of device real [N_p]; u: host array [count] of device complex
 * [T_p][N_p] (starting guesses in when opts->start == 2; start == 3 is not
 * accepted); y: host array [count] of device complex [T_p][M_p] (entries may
 * be NULL) or NULL; iters: host int [sum T_p] (problem-major) or NULL. */
int cisor_batch_forward(cisor_batch *batch, const void *const *f, void *const *u, void *const *y,
                        const cisor_ls_opts *opts, int *iters);
/* Largest eigenvalue of the Born Gauss-Newton operator of problem p (as
 * cisor_born_lipschitz); synchronises the device. */
int cisor_batch_born_lipschitz(cisor_batch *batch, int p, int iters, double *L);
/* Autotune the column stage of every grid (see cisor_autotune).  variants:
 * host int [groups] or NULL; times_ms: host float [groups][10] or NULL. */
int cisor_batch_autotune(cisor_batch *batch, int reps, int *variants, float *times_ms);

/* ---- learned warm start for the Lippmann-Schwinger solves ----
 * Not part of the paper: a convolutional encoder-decoder that predicts the
 * total field u of A u = u_in (eq. u_and_v) from (f, u_in), used as the
 * starting guess x0 of the solves (start == 3 keeps the first-Born start
 * wherever the prediction is worse).  The solve always runs to the requested
 * true residual; the network only changes where it starts.
 * Architecture (fixed): inputs f, Re u_in, Im u_in and, optionally, Re/Im of
 * the first-Born scattered field u_B = G diag(f) u_in (which the caller forms
 * with one operator application, u_B = u_in - A u_in) on the H x W grid; four
 * levels of two 3x3 convolutions + ReLU with base, 2 base, 4 base, 8 base
 * channels, 2x2 average pooling down, nearest x2 upsampling and channel
 * concatenation with the encoder features up, and a 3x3 head producing
 * Re/Im of u - u_in.  BF16 weights and activations on the matrix cores with
 * FP32 accumulation; FP32 master weights; Adam.
 * Parameter vector (FP32, device): for each of the 15 convolutions in order
 * (enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, bott_a, bott_b, dec3a, dec3b,
 * dec2a, dec2b, dec1a, dec1b, head): weights [3][3][Cout][Cin] (row-major,
 * kernel tap ky*3+kx first) then bias [Cout]; the first layer has Cin = 32
 * (inputs f, Re u_in, Im u_in, Re u_B, Im u_B in channels 0..4, the rest
 * zero) and the head Cout = 32 (outputs in channels 0..1, the rest zero). */
typedef struct cisor_net cisor_net;
/* H, W multiples of 16, base a multiple of 32, H*W*max_batch a multiple of
 * 8192; seeded He-normal initialisation.  stream: hipStream_t or NULL. */
int cisor_net_create(int height, int width, int base, int max_batch, unsigned long long seed, void *stream,
                     cisor_net **out);
int cisor_net_destroy(cisor_net *net);
int cisor_net_set_stream(cisor_net *net, void *stream);
int cisor_net_num_params(const cisor_net *net, long long *n);
/* Copy the FP32 parameter vector to / from device memory (set resets Adam). */
int cisor_net_get_params(cisor_net *net, float *params);
int cisor_net_set_params(cisor_net *net, const float *params);
/* u0 = u_in + net(f, u_in, u_B) for a batch of fields.  f: device float [B][H*W];
 * u_in, u0: device complex64 [B][H*W]; u_born: device complex64 [B][H*W] or
 * NULL (channels 3, 4 zero); 1 <= B <= max_batch. */
int cisor_net_forward(cisor_net *net, const float *f, const void *u_in, const void *u_born, void *u0, int batch);
/* Relative-L2 loss (1/B) sum_b ||net_b - (u_b - u_in,b)||^2 / ||u_b - u_in,b||^2
 * and its gradient with respect to the parameter vector.  loss: host double
 * or NULL; grad: device float [num_params] or NULL. */
int cisor_net_loss_grad(cisor_net *net, const float *f, const void *u_in, const void *u_born, const void *u,
                        int batch, double *loss, float *grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss, with the
 * gradient scaled by min(1, clip / ||grad||_2) first (clip <= 0: no clipping). */
int cisor_net_train_step(cisor_net *net, const float *f, const void *u_in, const void *u_born, const void *u,
                         int batch, double lr, double clip, double *loss);
/* Layer-level hooks: one 3x3 convolution (x: bf16 [B][H][W][Ci], w: bf16
 * [3][3][Co][Ci], bias: float [Co] or NULL, y: bf16 or float [B][H][W][Co];
 * Ci, Co multiples of 32, B*H*W a multiple of 128; tile 0 picks the block
 * tile automatically, 1..6 forces pixels x channels 256x128, 128x128, 256x64,
 * 128x64, 256x32, 128x32, CISOR_E_ARG if it does not divide) and its weight gradient
 * (dy: bf16 [B][H][W][Co]; dw: float [3][3][Co][Ci]; scratch: float
 * [max_splits][3][3][Co][Ci]). */
int cisor_nn_conv3x3(const void *x, const void *w, const float *bias, void *y, int B, int H, int W, int Ci, int Co,
                     int relu, int out_f32, int tile, void *stream);
int cisor_nn_conv3x3_wgrad(const void *x, const void *dy, float *dw, float *scratch, int B, int H, int W, int Ci,
                           int Co, int max_splits, void *stream);
/* The same convolution with two options (test hook of the network's own
 * launches): x2 != NULL reads the channel concatenation [x | up2(x2)]
 * without forming it (x: bf16 [B][H][W][C1], x2: bf16 [B][H/2][W/2][Ci - C1],
 * up2 the nearest-neighbour 2x upsampling; C1 a multiple of 32 with
 * 0 < C1 < Ci, H and W even), bit-identical to cisor_nn_conv3x3 on the formed
 * concatenation; splits > 1 spreads the K = 9 Ci loop over that many blocks
 * (larger values act as 9 Ci / 32), whose FP32 partials in workspace (device float,
 * workspace_elems >= splits B H W Co) are summed in split order.  splits = 1:
 * no split (workspace may be NULL).  CISOR_E_ARG on any violation. */
int cisor_nn_conv3x3_ex(const void *x, const void *x2, int C1, const void *w, const float *bias, void *y, int B,
                        int H, int W, int Ci, int Co, int relu, int out_f32, int tile, int splits, float *workspace,
                        size_t workspace_elems, void *stream);

/* ---- 3D vectorial (electromagnetic) model: the appendix on 3D imaging ----
 * Three-component fields E = (E_x, E_y, E_z) (the stacking of eq. u_def),
 * stored device complex128 [T][3][N] (transmitter, component, voxel; voxel
 * order as above).  With G0 the cell-integrated scalar Green's function
 * (the 3D kernel K above divided by k^2) applied to each component:
 *   B = G0 (f E),   E = E_in + (k^2 I + D) B        (eq. discrete0_constrain)
 *   A E = E - (k^2 I + D)(I_3 x G0 diag f) E        (eq. 3DA_def)
 *   y_t,m = sum_q sum_j Ht[m][j N + q] f_q E_t^(j)_q (eq. discrete0_measurement)
 * where D is the grad-div operator with the paper's second-order stencils
 * (three-point second difference along an axis; the four-corner cross
 * difference over 4 h^2 between two axes), fields taken as zero outside the
 * grid, and Ht[m][j N + q] = h^3 Gd_3j(r_m - r_q): the third row of the dyadic
 * Green's function (eq. dyadicGreen; receivers polarised along z).
 * Transmitters are plane waves along dir_t (tx_kind 0) or unit electric
 * dipoles at pos_t (tx_kind 1; strictly outside the grid's cube), with
 * E_in = Gd(r - pos_t) p_t / k^2.  The polarisation p_t is z projected
 * transverse to the direction of travel: dir_t, or the direction from pos_t
 * to the grid's centre (x when that direction is along z).
 * Requirements: dim 3, precision 1 (complex128 throughout), eps_b 1
 * (CISOR_E_UNSUPPORTED otherwise); every receiver strictly outside the grid's
 * cube (CISOR_E_ARG).  The linear systems (3N unknowns per transmitter)
 * are solved by BiCGSTAB with FP64 reductions; opts->tol is the true relative
 * residual; replace_every and check_every are ignored. */
typedef struct cisor_vec_ctx cisor_vec_ctx;
/* stream: hipStream_t or NULL. */
int cisor_vec_create(const cisor_geometry *geom, void *stream, cisor_vec_ctx **out);
int cisor_vec_destroy(cisor_vec_ctx *ctx);
int cisor_vec_set_stream(cisor_vec_ctx *ctx, void *stream);
int cisor_vec_get_sizes(const cisor_vec_ctx *ctx, int *N, int *T, int *M);
/* Copy E_in (device complex128 [T][3][N]) / Ht (device complex128 [M][3N]). */
int cisor_vec_get_uin(cisor_vec_ctx *ctx, void *E_in);
int cisor_vec_get_H(cisor_vec_ctx *ctx, void *H);
/* y = A x (adjoint 0) or A^H x = x - f G0^H (k^2 I + D) x (adjoint 1);
 * f: device double [N]; x, y: device complex128 [T][3][N], x != y. */
int cisor_vec_apply_A(cisor_vec_ctx *ctx, const double *f, const void *x, void *y, int adjoint);
/* Solve A E_t = E_in,t for every t and, if y != NULL, project y (device
 * complex128 [T][M]).  E: device complex128 [T][3][N] (the starting guess on
 * entry when opts->start == 3; start 0 zero, 1 E_in); iters: host int [T] or
 * NULL; max_rel: host double or NULL (largest final true relative residual). */
int cisor_vec_forward(cisor_vec_ctx *ctx, const double *f, const cisor_ls_opts *opts, void *E, void *y,
                      int *iters, double *max_rel);
/* Receivers used by each transmitter's data, as cisor_set_rx_mask: mask host
 * [T][M], nonzero = active, NULL = all active.  With a mask, D and the
 * gradient use w_t = mask_t (y_t - y_meas,t); predicted data are still
 * written for every receiver.  Kept until changed. */
int cisor_vec_set_rx_mask(cisor_vec_ctx *ctx, const unsigned char *mask);
/* y = Ht (I_3 x diag f) E (y: device complex128 [T][M]). */
int cisor_vec_project(cisor_vec_ctx *ctx, const double *f, const void *E, void *y);
/* Gradient of D = 1/2 sum_t ||y_t - y_meas,t||^2 (eqs. 3Du_and_v, 3Dg_def,
 * 3Dgradient): A E_t = E_in,t; w_t = y_t - y_meas,t (on the active
 * receivers, see cisor_vec_set_rx_mask); q_t = Ht^H w_t;
 * A^H V_t = (I_3 x diag f) q_t; grad = Re sum_t sum_j conj(E_t^(j))
 * (q_t + (I_3 x G0^H)(k^2 I + D) V_t)^(j).  f: device double [N]; y_meas:
 * device complex128 [T][M]; grad: device double [N]; D: host double;
 * opts->start 0 zero, 1 first Born, 2 the fields of this context's previous
 * gradient (first Born on the first call); iters: host int [2T] (forward then
 * adjoint) or NULL; max_rel: host double or NULL. */
int cisor_vec_grad(cisor_vec_ctx *ctx, const double *f, const void *y_meas, double *grad, double *D,
                   const cisor_ls_opts *opts, int *iters, double *max_rel);
/* One relaxed-FISTA iteration (eqs. algo1-algo3) of the vectorial model: the
 * gradient above at state->s, then the step, the 3D TV/box prox (as
 * cisor_tv_prox on a 3D grid) and the momentum update, as cisor_fista_step.
 * state: f, f_prev, s device double [N]; opts->start as in cisor_vec_grad
 * (2: the fields of the previous iteration); info as cisor_fista_step. */
int cisor_vec_fista_step(cisor_vec_ctx *ctx, cisor_fista_state *state, const void *y_meas, double gamma,
                         double tau, double alpha, double lo, double hi, int inner_iters,
                         const cisor_ls_opts *opts, cisor_step_info *info);

/* Human-readable text of a status code. */
const char *cisor_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* CISOR_H */
