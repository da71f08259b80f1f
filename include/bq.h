/*
 * bq -- MI355X (gfx950) hot path of the mini-batch quasi-Newton proximal
 * method for TV-constrained 3D reconstruction (Hong, Pham, Yavneh, Unser,
 * arXiv:2307.02043).
 *
 * The library evaluates the two kernels that dominate each iteration of
 * the method's Algorithm 4.1:
 *
 *   - the mini-batch data-term gradient  grad F_s(x) = (S/L) sum_{l in S_s}
 *     grad f_l(x),  f_l(x) = 1/2 ||H_l(x) - y_l||^2  (Section 1 eq.
 *     defMainPro, Section 4 eq. NewModelPro), where H_l is the optical
 *     diffraction tomography model of Section 6: the Lippmann-Schwinger
 *     equation (I - G diag(x)) u_l = u_in,l solved by BiCGSTAB, one solve
 *     for H_l and two for grad f_l; or its first-Born linearisation;
 *
 *   - the weighted proximal mapping of constrained TV (Section 3.4
 *     definition of the WPM; Section 4.1 dual formulation; Lemma 4.1;
 *     Theorem 3.1 with the metric tau I + u u^T of Algorithm 4.2).
 *
 * Conventions common to all calls
 *   - Arrays are C-order [z][y][x] with N^3 voxels (x fastest).  Complex
 *     arrays are interleaved (re, im) pairs: complex64 (2 x float) when the
 *     context precision is BQ_F32, complex128 (2 x double) for BQ_F64; real
 *     arrays are float / double accordingly.
 *   - Pointers named "device" must point to device memory of the current
 *     HIP device; "host" pointers to host memory.  All arrays are owned by
 *     the caller: the library never frees them and keeps no reference to
 *     them after the call returns.
 *   - Work is enqueued on the stream given at creation; each call
 *     synchronises that stream before returning (it reads solver status),
 *     so outputs are ready when it returns.
 *   - A context is not thread-safe; use one per host thread.
 *   - Return value: BQ_OK (0), a negative error (no output written or
 *     outputs undefined), or a positive warning (outputs written; at least
 *     one solve did not converge cleanly; per-system detail in the stats).
 *     bq_last_error() describes the last error or warning of a context.
 *
 * Physical units: lengths in micrometres; x is the scattering potential
 * k0^2 (n^2 - n_b^2) in um^-2; the discrete Green's operator includes the
 * voxel volume, so G is dimensionless.
 */
#ifndef BQ_H
#define BQ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BQ_OK = 0,
  BQ_EINVAL = -1,        /* invalid argument (null pointer, size, index)   */
  BQ_ENOMEM = -2,        /* device allocation failed                        */
  BQ_EDEVICE = -3,       /* HIP runtime error                               */
  BQ_EUNSUPPORTED = -4,  /* grid size without a kernel instantiation        */
  BQ_NOTCONV = 1,        /* a solve hit max_iter before reaching tol        */
  BQ_BREAKDOWN = 2,      /* a BiCGSTAB scalar (rho, <rhat,v>, omega) vanished */
  BQ_NONFINITE = 3       /* NaN/Inf met in a solve                          */
} bq_status;

typedef enum { BQ_F32 = 0, BQ_F64 = 1 } bq_precision;
typedef enum { BQ_MODEL_LS = 0, BQ_MODEL_BORN = 1 } bq_model;

/* flags of bq_geom */
#define BQ_FLAG_PLAIN 1u    /* solve one illumination at a time, with a host
                               round trip per BiCGSTAB iteration (baseline) */
#define BQ_FLAG_FUSED_XY 2u /* run the x/y FFTs of G as one LDS-resident plane
                               pass where it exists (N = 16..128 complex64,
                               16..64 complex128) instead of three passes   */
#define BQ_FLAG_GRAPH 4u    /* batched solves replay one captured BiCGSTAB
                               iteration as a HIP graph on a stream of the
                               library's own instead of launching its kernels
                               one by one (same results; measured no faster
                               for these kernel lengths, so not the default) */

/* Grid, optics and solver settings (Section 6.1 describes the setting). */
typedef struct {
  int N;             /* grid edge; supported: 8 12 16 24 32 48 64 96 128 256 */
  double h_um;       /* voxel edge (um)                                     */
  double lambda0_um; /* vacuum wavelength (um)                              */
  double n_b;        /* background refractive index                         */
  int precision;     /* bq_precision of fields and FFTs                     */
  int model;         /* bq_model                                            */
  double tol;        /* BiCGSTAB relative residual tolerance (>= 0)         */
  int max_iter;      /* BiCGSTAB iteration cap (>= 0)                       */
  unsigned flags;    /* BQ_FLAG_*                                           */
  double det_dist_um; /* detector plane distance beyond the exit plane z =
                         N-1 (um, >= 0).  0: the detector is the exit plane.
                         > 0: the exit-plane scattered field, periodic over
                         the N x N window, is propagated by the angular
                         spectrum exp(i k_z d) (evanescent parts decaying);
                         the adjoint uses the conjugate transfer function  */
  int cam_n;          /* camera pixels per side M (0 <= M <= 4096).  0: the
                         detector images are the N x N lateral window.  > 0:
                         an M x M camera centred on the optical axis samples
                         the detector-plane field (after the propagation
                         above) at its pixel centres (a - (M-1)/2) pitch, by
                         trigonometric interpolation of the window's samples
                         (the field taken as periodic over the window and
                         band limited to its DFT frequencies, the Nyquist bin
                         of an even N at -pi/h).  Images, measurements y and
                         residuals are then M x M; the adjoint right-hand
                         side uses the adjoint sampling.  The paper's cameras
                         (512^2, 150^2 pixels, Section 6) have their own pixel
                         count and pitch; their optics are not given      */
  double cam_pitch_um; /* camera pixel pitch in the sample plane (um, > 0 when
                          cam_n > 0)                                        */
} bq_geom;

/* Unit propagation direction of a plane-wave illumination
 * u_in(r) = exp(i k_b d . r), k_b = 2 pi n_b / lambda0 (Section 6.1). */
typedef struct {
  double dx, dy, dz;
} bq_illum;

/* Per-illumination outcome of the solves of one call. */
typedef struct {
  int iters_fwd, iters_adj;   /* BiCGSTAB iterations (0 for the Born model) */
  int status_fwd, status_adj; /* 0 converged, 1 not converged, 2 breakdown,
                                 3 non-finite                               */
  double relres_fwd, relres_adj; /* final relative recursive residuals      */
  int green_apps;             /* applications of G for this illumination in
                                 the call (solver matvecs, initial
                                 residuals, adjoint right-hand side)        */
  int pad_;
} bq_solve_stats;

typedef struct bq_ctx bq_ctx;

/* Create a context for one geometry and a set of L illuminations.
 *   g      host, geometry/solver settings (copied)
 *   dirs   host, L unit directions (copied; |d| must be 1 within 1e-6)
 *   stream hipStream_t to enqueue on (NULL = default stream)
 *   out    host, receives the context
 * Precomputes the Green's transfer function of the padded grid on the
 * device.  Errors: BQ_EINVAL, BQ_EUNSUPPORTED, BQ_ENOMEM, BQ_EDEVICE. */
bq_status bq_create(const bq_geom* g, const bq_illum* dirs, int L, void* stream, bq_ctx** out);

/* Release all device memory of a context.  NULL is accepted. */
bq_status bq_destroy(bq_ctx* ctx);

/* Text of the last error or warning of ctx (or of the last failed
 * bq_create when ctx is NULL).  Valid until the next call on ctx. */
const char* bq_last_error(const bq_ctx* ctx);

/* Forward model H_l(x) for the illuminations idx[0..B-1] (Section 6: one
 * Lippmann-Schwinger solve per illumination; first Born: S G(x u_in)).
 *   x      device, N^3 real potential
 *   idx    host, B indices in [0, L)
 *   y_out  device, B x D x D complex (D = cam_n, or N without a camera): the
 *          scattered field S(u_l - u_in,l) on the detector plane z = N-1,
 *          propagated and sampled by the camera as set in bq_geom
 *   st     host, B entries or NULL */
bq_status bq_forward(bq_ctx* ctx, const void* x, const int* idx, int B, void* y_out,
                     bq_solve_stats* st);

/* Total fields u_l = (I - G diag(x))^-1 u_in,l for idx[0..B-1].
 *   u_out  device, B x N^3 complex (Born model: u_in,l)  */
bq_status bq_fields(bq_ctx* ctx, const void* x, const int* idx, int B, void* u_out,
                    bq_solve_stats* st);

/* Mini-batch gradient and loss (Section 4 eq. NewModelPro with the scale
 * S/L passed explicitly):
 *   g_out = scale * sum_b Re(conj(u_b) . w_b),
 *   (I - G^H diag(x)) w_b = G^H S^T r_b,  r_b = S(u_b - u_in,b) - y_b,
 *   *loss = scale * sum_b 1/2 ||r_b||^2
 *   (S including the propagation and the camera when set in bq_geom).
 *   x      device, N^3 real
 *   y      device, B x D x D complex (D as for bq_forward), y[b] measured
 *          for illumination idx[b]
 *   g_out  device, N^3 real, overwritten
 *   loss   host, may be NULL
 *   st     host, B entries or NULL */
bq_status bq_grad(bq_ctx* ctx, const void* x, const void* y, const int* idx, int B, double scale,
                  void* g_out, double* loss, bq_solve_stats* st);

/* bq_grad with the fields kept and, optionally, used as starting points
 * (warm start across outer iterations; LS model only).
 *   u_io, w_io  device, B x N^3 complex each (context precision), aligned
 *               with idx.  On return they hold the forward fields u_b and the
 *               conjugated adjoint fields w_b of the batch.
 *   start       0: the solves start from their right-hand sides (as bq_grad);
 *               otherwise from u_io and w_io (BiCGSTAB with r0 = b - A e0; a
 *               system whose right-hand side is zero returns zero).
 * Other arguments, results and errors as bq_grad; BQ_EUNSUPPORTED for the
 * Born model. */
bq_status bq_grad_ws(bq_ctx* ctx, const void* x, const void* y, const int* idx, int B, double scale,
                     void* g_out, double* loss, bq_solve_stats* st, void* u_io, void* w_io, int start);

/* Mini-batch loss only: *loss = scale * sum_b 1/2 ||S(u_b - u_in,b) - y_b||^2
 * (forward solves and detector residual, no adjoint solve).  Arguments as
 * for bq_grad.  Used by differentiation wrappers whose backward pass calls
 * bq_grad, which solves the forward fields again instead of storing them. */
bq_status bq_loss(bq_ctx* ctx, const void* x, const void* y, const int* idx, int B, double scale,
                  double* loss, bq_solve_stats* st);

/* Apply the discrete Green's operator to B complex fields:
 * out_b = G v_b (adjoint != 0: G^H v_b).  v, out: device, B x N^3 complex;
 * v and out must not overlap. */
bq_status bq_green_apply(bq_ctx* ctx, const void* v, void* out, int B, int adjoint);

/* Device timing of the passes of the Green's operator (HIP events recorded
 * on the context stream around every launch of a timed pass).  enable is a
 * bit mask over bq_pass (bit p times pass p; BQ_TIMING_ALL times all); a
 * nonzero mask clears the counters and starts timing, 0 stops it.  Each
 * timed launch adds two event records to the stream, so time only the
 * passes of interest where the event overhead matters.  Events are read
 * back lazily: bq_timing (either value) synchronises the context stream and
 * brings the totals up to date.  bq_timing_get then returns the summed duration (ms)
 * and the number of launches of one pass since the last enable.
 * Errors: BQ_EINVAL (no context, mask outside [0, BQ_TIMING_ALL], pass out
 * of range). */
typedef enum {
  BQ_PASS_ZF = 0,  /* z lines, forward, with the input prologue          */
  BQ_PASS_XF = 1,  /* x rows, forward (split path)                        */
  BQ_PASS_YC = 2,  /* y columns: FFT, transfer function, inverse FFT      */
  BQ_PASS_XI = 3,  /* x rows, inverse (split path)                        */
  BQ_PASS_ZI = 4,  /* z lines, inverse, with the epilogue and partial sums */
  BQ_PASS_XY = 5,  /* fused x/y plane pass (LDS-resident planes)          */
  BQ_PASS_VEC = 6, /* BiCGSTAB vector updates                             */
  BQ_PASS_COUNT = 7
} bq_pass;
#define BQ_TIMING_ALL ((1 << BQ_PASS_COUNT) - 1)
bq_status bq_timing(bq_ctx* ctx, int enable);
bq_status bq_timing_get(const bq_ctx* ctx, int pass, double* total_ms, long long* launches);

/* Launch shapes of the Green's operator passes (implementation choices, no
 * part of the paper's method): the rows per workgroup of the x passes and
 * the threads per workgroup of the padded z-forward pass.  No value any
 * call computes depends on them (neither pass forms a partial sum).
 *
 * bq_autotune times a short forward solve of B systems (or of the launch
 * set a batch of B runs in, see bq_set_batch_limit; tolerance 0, two
 * BiCGSTAB iterations, a weak uniform potential, the first B illuminations)
 * under each candidate shape, one at a time, keeps the fastest in the
 * context for every later call, and reports it in *out (may be NULL; 0 in a
 * field = the default shape).  It allocates the batch workspace for B
 * systems (as a call with B systems would) and a temporary N^3 potential,
 * synchronises the context stream, and leaves tolerance, iteration limit,
 * per-pass timing and the convergence-check history as they were.
 * bq_set_plan sets the shapes directly (0 = default).
 * Errors: BQ_EINVAL (no context, B < 1, a shape not available for the
 * grid and precision), BQ_ENOMEM, BQ_EDEVICE. */
typedef struct {
  int x_tile_rows;    /* rows per workgroup of the x passes (0: default)     */
  int zf_threads;     /* threads of the padded z-forward pass (0: default)   */
  double ms_default;  /* the timed solve with the default shapes             */
  double ms_tuned;    /* the same with the chosen shapes                     */
} bq_tune_result;
bq_status bq_autotune(bq_ctx* ctx, int B, bq_tune_result* out);
bq_status bq_set_plan(bq_ctx* ctx, int x_tile_rows, int zf_threads);

/* Systems per launch set of bq_forward, bq_fields, bq_loss, bq_grad and
 * bq_grad_ws.  A batch larger than max_systems (0, the default: as many as
 * the free device memory holds next to the context's own workspace, about
 * 14 N^3 complex values per system) runs as consecutive sub-batches, each
 * solved for its own contribution; per-system fields, images and
 * iteration counts are the same, the gradient and loss are sums over the
 * sub-batches (equal up to the order of the additions).
 * Errors: BQ_EINVAL (no context, max_systems < 0). */
bq_status bq_set_batch_limit(bq_ctx* ctx, int max_systems);

/* Breakdown test of BiCGSTAB (van der Vorst 1992, the solver of the
 * Lippmann-Schwinger systems of Section 6): a system stops with status
 * "breakdown" (BQ_BREAKDOWN from the call) when |rho| = |<rhat, r>|,
 * |<rhat, A p>| or |omega| falls below floor; its iterate is kept as it was
 * at that point.  Default 1e-300 (only exact or near-exact vanishing).  A
 * larger floor stops solves early where these scalars become small
 * relative to the problem's scale.  Applies to later calls.
 * Errors: BQ_EINVAL (no context, floor negative or not finite). */
bq_status bq_set_breakdown_floor(bq_ctx* ctx, double floor);

/* State of a context, for callers that manage memory and graph replay.
 * Errors: BQ_EINVAL (null argument). */
typedef struct {
  int batch_capacity;       /* systems the held batch workspace covers (0: none) */
  int x_tile_rows;          /* launch shape in use (0: default)                  */
  int zf_threads;           /* launch shape in use (0: default)                  */
  int graphs_cached;        /* captured BiCGSTAB iteration graphs held (<= 4)    */
  long long graph_captures; /* iteration graphs captured since creation; a
                               graph is captured again after a change of batch
                               buffers, potential, incident table or launch
                               shapes (bq_set_plan); bq_autotune drops all     */
  double breakdown_floor;   /* see bq_set_breakdown_floor                        */
} bq_ctx_info;
bq_status bq_get_info(const bq_ctx* ctx, bq_ctx_info* out);

/* Self-check of the library's own addressing (no operation of the paper;
 * host code only, no GPU needed).  The padded-line passes of G read and
 * write through raw buffer resources, where an access past the resource's
 * size reads zero or is dropped instead of faulting.  For every grid and
 * precision those passes are built for, this enumerates every offset their
 * launch grids can form (and the y pass's workgroup-to-slice mapping for
 * batches of 1..40) and checks that each resource is under 2^31 bytes, lies
 * inside its allocation, and contains every access without 32-bit wrap.
 *   report    host, receives a message (may be NULL); report_len its size
 *   accesses  host, receives the number of accesses checked (may be NULL)
 * Returns the number of violations (0: all in range). */
int bq_audit_raw_ranges(char* report, int report_len, long long* accesses);

/* ---------------------------------------------------------------------
 * Weighted proximal mapping of constrained TV
 * --------------------------------------------------------------------- */
typedef enum { BQ_TV_ISO = 0, BQ_TV_ANISO = 1 } bq_tv;
typedef enum { BQ_SET_NONE = 0, BQ_SET_NONNEG = 1 } bq_set;

typedef struct {
  int newton_total;  /* root-finding passes over all dual iterations        */
  int newton_max;    /* most passes in one dual iteration                   */
  double beta_last;  /* root of Theorem 3.1's phi at the output (its first
                        component for a metric of rank >= 2)                */
  double phi_last;   /* max_i |phi_i(beta_last)|                            */
} bq_prox_stats;

#define BQ_PROX_MAX_RANK 8

typedef struct bq_prox bq_prox;

/* Workspace for proximal mappings of an nz x ny x nx image.
 * Errors: BQ_EINVAL, BQ_ENOMEM, BQ_EDEVICE. */
bq_status bq_prox_create(int nz, int ny, int nx, int precision, void* stream, bq_prox** out);
bq_status bq_prox_destroy(bq_prox* p);
const char* bq_prox_last_error(const bq_prox* p);

/* x = argmin_{x in C} 1/2 ||x - v||^2_{tau I + U U^T} + lambda TV(x)
 * (Section 4 eq. SecondProximal_WPMTV, lambda = a_k S lambda of the
 * outer iteration), by n_iter accelerated projected-gradient iterations on
 * the dual of Section 4.1 (step tau / (12 lambda), Lemma 4.1 with
 * omega_min = tau), the projection onto C by Theorem 3.1 with the
 * semi-smooth Newton root-find of Algorithm 4.3 (safeguarded: bracketing for
 * r = 1, backtracking on the function whose gradient is phi for r >= 2),
 * and the Woodbury inverse of the metric (Section 4.3).  Output x(P_K).
 *   v      device, image (nz*ny*nx real, precision of p)
 *   tau    > 0
 *   U      device, the r columns of the metric's low-rank factor, column c
 *          at U + c * nz*ny*nx (precision of p); may be NULL when r = 0
 *   r      0 <= r <= BQ_PROX_MAX_RANK (0: metric tau I)
 *   lambda > 0
 *   tv     bq_tv;  cset  bq_set;  n_iter >= 0
 *   x_out  device, image, overwritten
 *   P_io   device, 3 x image (component d = finite difference along array
 *          axis d: 0 = z, 1 = y, 2 = x) or NULL.  When given it is the
 *          starting dual point and receives P_K; NULL starts from zero.
 *   st     host or NULL
 * Runs on the workspace's own stream after the work pending on the stream
 * given at creation, and returns once the result is complete.
 * Root passes: a call launches the number of root-finding passes per dual
 * iteration that the workspace last needed plus one (at least 2); if some
 * dual iteration needs more, the whole call is run again from the same
 * starting point with the full pass limit, so the result never depends on
 * the workspace's history.  With P_io given and fewer than the full passes
 * launched, the starting dual point is first copied to a 3 x image buffer
 * that the workspace allocates on first use (if that allocation fails, the
 * full passes are launched instead).
 * With r = 0 the projection is pointwise and there is no root (st reports
 * zero passes); the first such call allocates a second 3 x image buffer
 * for the dual momentum, kept until bq_prox_destroy.
 * Errors: BQ_EINVAL (arguments), BQ_ENOMEM (r = 0, that buffer),
 * BQ_EDEVICE; BQ_NOTCONV if the root-find hit its pass limit in some dual
 * iteration (x is still returned). */
bq_status bq_wprox(bq_prox* p, const void* v, double tau, const void* U, int r, double lambda, int tv,
                   int cset, int n_iter, void* x_out, void* P_io, bq_prox_stats* st);

/* bq_wprox without a workspace object, for callers that cannot allocate
 * device memory (code under HIP graph capture elsewhere in the caller,
 * serving loops, harnesses that forbid hipMalloc): it calls no hipMalloc,
 * hipFree or other allocating routine and captures no graph.  Its scratch
 * memory is one static device array of BQ_WPROX_NOALLOC_SCRATCH bytes per
 * GPU, allocated when the library is loaded on that GPU and held until the
 * process ends; its device address is looked up on the first call on each
 * GPU.
 *   nz, ny, nx, precision  image shape (each >= 2) and bq_precision
 *   stream                 hipStream_t the work is enqueued on (NULL: the
 *                          default stream); the call synchronises it
 *   other arguments        as bq_wprox (the same computation and result)
 * Scratch needed, in bytes rounded up to 256 each: the image, the dual
 * momentum (3 images), the dual point unless P_io is given (3 images), a
 * second momentum at rank 0 (3 images), plus about 1 MB of partial sums and
 * state: in FP32 every rank fits at 128^3, in FP64 at 96^3.
 * Every call on a GPU uses that GPU's one array, which keeps the last
 * call's contents (each call initialises what it reads): calls that
 * overlap on one GPU (concurrent host threads, or streams whose work
 * overlaps) race and give undefined results.  Every root pass is launched
 * (as bq_wprox's full pass budget), so no call is run twice.
 * Errors: BQ_EINVAL (arguments, or an image whose scratch exceeds the
 * array: the message states the bytes needed), BQ_EDEVICE; BQ_NOTCONV as
 * bq_wprox.  bq_prox_last_error(NULL) returns the message (per thread). */
#define BQ_WPROX_NOALLOC_SCRATCH (96u << 20)
bq_status bq_wprox_noalloc(int nz, int ny, int nx, int precision, const void* v, double tau, const void* U,
                           int r, double lambda, int tv, int cset, int n_iter, void* x_out, void* P_io,
                           bq_prox_stats* st, void* stream);

/* ---------------------------------------------------------------------
 * Mini-batch quasi-Newton proximal iteration (Algorithm 4.1)
 * --------------------------------------------------------------------- */
typedef struct {
  int S;            /* number of subsets, 1 <= S <= BQ_PROX_MAX_RANK          */
  double a;         /* step size a_k (constant), > 0                          */
  double lambda;    /* TV weight lambda, > 0                                  */
  double alpha;     /* alpha_s of Algorithm 4.1 (every subset), > 0           */
  double gamma;     /* scaling of the initial SR1 metric (Algorithm 4.2), (0,1] */
  double tau_max;   /* upper bound on tau of Algorithm 4.2, > 0               */
  int tv;           /* bq_tv                                                  */
  int cset;         /* bq_set                                                 */
  int prox_iters;   /* dual iterations of each WPM, >= 0                      */
  int warm_start;   /* nonzero: keep each subset's forward and adjoint fields
                       and start its next solves from them (bq_grad_ws; LS
                       model; 2 x sum_s |subset s| device fields)            */
  int first_order;  /* nonzero: metric alpha I and weight a lambda at every
                       iteration (no SR1): the proximal-gradient baseline   */
} bq_qn_params;

typedef struct {
  int k;            /* iteration just completed (1-based)                     */
  int subset;       /* s', the subset whose gradient was computed             */
  double loss;      /* F_{s'}(x_{k-1}) = (S/L) sum_{l in s'} f_l              */
  double tau;       /* tau_{s'} of Algorithm 4.2 after this iteration         */
  int u_kept;       /* 1 if s' keeps its rank-one correction                  */
  int metric_rank;  /* columns of U passed to the WPM: the subsets that hold a
                       rank-one correction (0 for k <= S or when none does;
                       the others are zero columns of U and are left out)   */
  double tau_sum;   /* tau of the WPM metric: alpha (k <= S) or sum_s tau_s   */
  int prox_passes;  /* root-finding passes of the WPM                        */
} bq_qn_info;

typedef struct bq_qn bq_qn;

/* Outer iteration of Algorithm 4.1 on an LS/Born context and a prox
 * workspace of the same precision and an N x N x N image.  The S subsets
 * are given as consecutive runs of illumination indices:
 *   subset_idx  host, sum_s subset_len[s] indices into the context's L
 *               illuminations; subset_len host, S positive lengths.
 * F_s = (S/L) sum_{l in subset s} f_l (eq. NewModelPro).  Per subset the
 * object keeps xbar_s, gbar_s and u_s (3S device images, Section 4.4) and
 * tau_s.  ls and px are borrowed (they must outlive the object); the
 * object owns its buffers.  Errors: BQ_EINVAL, BQ_EUNSUPPORTED (precision or
 * shape mismatch), BQ_ENOMEM. */
bq_status bq_qn_create(bq_ctx* ls, bq_prox* px, const bq_qn_params* prm, const int* subset_idx,
                       const int* subset_len, bq_qn** out);
bq_status bq_qn_destroy(bq_qn* q);
const char* bq_qn_last_error(const bq_qn* q);

/* One iteration x_{k-1} -> x_k of Algorithm 4.1 with the choices of
 * Section 4.3 (x_s^k = x_{k-1}, g_s^k = grad F_{s'}(x_{k-1}) for every s).
 *   x     device image, in: x_{k-1}, out: x_k
 *   y     device, the measurements of all L illuminations, [L][N][N] complex
 *   pick  the subset s' for k > S: -1 = strategy I (s' = k - 1 mod S), or
 *         0..S-1 = the draw of strategy II (made by the caller); ignored for
 *         k <= S, where s' = k - 1
 *   info  host or NULL
 * Steps: gradient of subset s' (bq_grad); for a revisited subset the SR1
 * metric of Algorithm 4.2 from (x_{k-1} - xbar, g - gbar) (a subset seen
 * once keeps alpha I); for k <= S the WPM with metric alpha I and weight
 * a lambda of x_{k-1} - (a/alpha) g; for k > S the WPM with metric
 * Btilde = sum_s tau_s I + U U^T (the S columns u_s, zero where dropped)
 * and weight a S lambda of v = x_{k-1} - a S Btilde^-1 g (Woodbury).
 * Returns the status of the solves (BQ_NOTCONV etc.) or of the WPM. */
bq_status bq_qn_step(bq_qn* q, void* x, const void* y, int pick, bq_qn_info* info);

#ifdef __cplusplus
}
#endif

#endif /* BQ_H */
