/*
 * gkb.h -- C ABI of the MI355X (gfx950) implementation of AB-GKB and BA-GKB
 * for X-ray CT with an unmatched projector pair.
 *
 * The problem (Sec. 1, eq. (1)): A x ~= b with A in R^{m x n} a forward
 * projector and B in R^{n x m} a back projector built from a different
 * discretisation, B != A^T.  AB-GKB (Sec. 3.2, Alg. "AB-GKB") runs the
 * Golub-Kahan bidiagonalisation on M = AB from b and returns x = B Q_k u_k;
 * BA-GKB (Alg. "BA-GKB") runs it on M = BA from B b and returns x = Q_k u_k.
 * Both need the exact transposes A^T and B^T (Sec. 5, where the projector
 * library is modified to provide them), so all four operators are exported.
 *
 * Discretisation (pixel pitch 1; pixel (i, j) has centre
 * (i - (nx-1)/2, j - (ny-1)/2) and is stored at x[j*nx + i]; sinograms are
 * stored y[(v*n_det_v + r)*n_det_u + k]):
 *   A  -- Joseph's ray-driven projector: along every ray, at each crossing
 *         of a pixel row (column) along the ray's dominant axis, linear
 *         interpolation between the two nearest pixel centres of that row
 *         (column); the sum is multiplied by 1/|d_dom| (d the unit ray
 *         direction; ties step along rows).  3D: bilinear interpolation in
 *         the voxel plane crossed.
 *   B  -- pixel (voxel) driven back projection: every pixel centre is
 *         projected onto each view's detector and the sinogram interpolated
 *         linearly (bilinearly on a 2D detector) between the nearest bins.
 *   A^T, B^T -- the exact transposes of those matrices.
 * Geometries:
 *   GKB_PAR2D: view angle th, ray (v,k) = { p : p.(cos th, sin th) = s_k },
 *              s_k = (k - (n_det_u-1)/2) * det_pitch_u.
 *   GKB_FAN2D: source S = src_dist*(cos b, sin b); curved equiangular
 *              detector, bin k at fan angle g_k = (k - (n_det_u-1)/2) *
 *              det_pitch_u (radians) counter-clockwise from the central ray
 *              -S/|S|; no distance weighting.
 *   GKB_CONE3D: source S = src_dist*(cos b, sin b, 0); flat detector
 *              perpendicular to -S at src_det_dist from the source, u axis
 *              (-sin b, cos b, 0), v axis z; pitches det_pitch_u/v.
 * View angles: angles[v] if given, else v*angle_span/n_views.
 *
 * Conventions:
 *  - Every data pointer is a DEVICE pointer owned by the caller, holding
 *    float (GKB_F32) or double (GKB_F64) elements, contiguous.
 *  - Projector calls are asynchronous on the context's stream.  Solves block
 *    until the result is in x and fill *info on the host.
 *  - Errors are negative gkb_status values; gkb_last_error() gives the text
 *    (thread-local).  On GKB_EINVAL / GKB_ENONFINITE nothing is written to
 *    the outputs.
 *  - A context is not thread-safe: one context per host thread.
 */
#ifndef GKB_H
#define GKB_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gkb_ctx gkb_ctx;
typedef struct gkb_net gkb_net;

typedef enum {
  GKB_OK = 0,
  GKB_EINVAL = -1,        /* invalid argument */
  GKB_ENOMEM = -2,        /* device allocation failed */
  GKB_EDEVICE = -3,       /* HIP runtime error */
  GKB_ENONFINITE = -4,    /* NaN or Inf in the data */
  GKB_EUNSUPPORTED = -5   /* combination not implemented */
} gkb_status;

typedef enum {
  GKB_STOP_NONE = 0,
  GKB_STOP_DP = 1,              /* discrepancy principle met (eq. DP) */
  GKB_STOP_KMAX = 2,            /* k_max iterations, DP off */
  GKB_STOP_BREAKDOWN = 3,       /* t_{k+1} or alpha_{k+1} vanished: invariant subspace, x exact there */
  GKB_STOP_DP_NOT_REACHED = 4,  /* DP on but not met by k_max; x = x_{k_max} */
  GKB_STOP_FALLBACK = 5,        /* learned preconditioner rejected; plain BA-GKB result returned */
  GKB_STOP_RNS = 6              /* residual norm stagnation (eq. RNS): x = x_k at the first such k */
} gkb_stop_reason;

typedef enum { GKB_PAR2D = 0, GKB_FAN2D = 1, GKB_CONE3D = 2 } gkb_geom_kind;
typedef enum { GKB_F32 = 0, GKB_F64 = 1 } gkb_dtype;

typedef struct {
  int kind;                 /* gkb_geom_kind */
  int nx, ny, nz;           /* image size; nz = 1 in 2D */
  int n_views;
  const double *angles;     /* HOST array [n_views] (radians) or NULL */
  double angle_span;        /* used when angles == NULL */
  int n_det_u, n_det_v;     /* detector bins; n_det_v = 1 in 2D */
  double det_pitch_u;       /* PAR2D/CONE3D: length; FAN2D: radians */
  double det_pitch_v;
  double src_dist;          /* source to rotation centre (FAN2D, CONE3D) */
  double src_det_dist;      /* source to detector (CONE3D) */
} gkb_geometry;

typedef struct {
  int k_max;                /* >= 1 iterations */
  double lambda;            /* Tikhonov weight on ||u|| in the projected problem; 0 = the paper's */
  int use_dp;               /* 1: stop at the first k with ||A x_k - b|| <= tau*noise_norm (eq. DP) */
  double tau;               /* > 0 when use_dp; the paper uses 1 */
  double noise_norm;        /* ||e||, the noise norm the discrepancy principle compares against */
  int reorth;               /* 1 = one-sided reorthogonalisation of q: two classical Gram-Schmidt rounds, the
                               second's inner products taken from the Gram matrix of the stored basis
                               ((k_max+1)^2 doubles of device workspace); 0 = none */
  const gkb_net *precond;   /* BA only: learned sinogram filter F inside B (M = B F A); NULL = plain */
  double *residual_history; /* optional HOST [k_max]: ||A x_k - b||, k = 1..k_stop */
  double *alpha_history;    /* optional HOST [k_max+1]: alpha_1.. */
  double *t_history;        /* optional HOST [k_max+1]: t_1.. */
  double rns_eps;           /* > 0: also stop at the first k >= 2 with
                             * | ||A x_{k-1} - b|| - ||A x_k - b|| | < rns_eps ||A x_{k-1} - b||
                             * (residual norm stagnation, eq. RNS, Sec. 5) and return x_k;
                             * 0 = off.  Tested after the discrepancy principle. */
  const void *x_true;       /* optional DEVICE [n] (dtype of the solve): the exact image.  With
                             * rre_history it turns on RRE(x_k) = ||x_k - x_true|| / ||x_true||
                             * (eq. RE, Sec. 5) after every iteration: x_k is assembled as the
                             * returned solution is (an extra GEMV over Q, and for AB a B call,
                             * per iteration).  Single-slice solves only: gkb_batch_solve returns
                             * GKB_EUNSUPPORTED.  x_true = 0 gives non-finite values. */
  double *rre_history;      /* optional HOST [k_max]: RRE(x_k), k = 1..k_stop (needs x_true) */
} gkb_solve_opts;

typedef struct {
  int k_stop;               /* iterations whose solution is returned (0 if breakdown at start) */
  int reason;               /* gkb_stop_reason */
  double residual;          /* ||A x - b|| at k_stop */
  double proj_residual;     /* ||C_k u_k - t_1 e_1|| (the Tikhonov rows not included) */
  double t1, alpha1;        /* t_1 = ||rhs||, alpha_1 */
  double seconds;           /* wall time of the solve */
} gkb_solve_info;

/* Creates a context on `device` that launches on `hip_stream` (a hipStream_t;
 * NULL = the default stream), so that its work is ordered with the caller's
 * other work on that stream.  The context owns geometry tables, Krylov bases
 * and scratch; it frees them in gkb_destroy.  gkb_set_stream switches the
 * stream (NULL = the default stream). */
gkb_status gkb_create(gkb_ctx **ctx, int device, void *hip_stream);
void gkb_destroy(gkb_ctx *ctx);
gkb_status gkb_set_stream(gkb_ctx *ctx, void *hip_stream);
const char *gkb_last_error(void);

/* The four projectors (Sec. 1; transposes as in Sec. 5).  x has n = nx*ny*nz
 * elements, y has m = n_views*n_det_v*n_det_u. */
gkb_status gkb_forward(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *x, void *y);          /* y = A x   */
gkb_status gkb_back(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *y, void *x);             /* x = B y   */
gkb_status gkb_forward_adjoint(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *y, void *x);  /* x = A^T y */
gkb_status gkb_back_adjoint(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *x, void *y);     /* y = B^T x */

/* x = B y without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same kernels and result as gkb_back, for GKB_PAR2D and
 * GKB_FAN2D (GKB_CONE3D: GKB_EUNSUPPORTED).  y (m elements) and x (n elements)
 * are DEVICE pointers owned by the caller; asynchronous on the context's
 * stream.  The scratch (the per-view constants and the zero-padded sinogram,
 * n_views * (n_det_u + 2 * pad) elements with pad >= 4) lives in a fixed
 * 32 MiB device array that the library holds on every GPU it runs on until
 * the process ends; a geometry needing more returns GKB_EINVAL before any
 * launch.  Every call on one GPU shares that array and overwrites it (the
 * padding step writes every element it reads, so nothing carries over from
 * one call to the next): calls that overlap on one GPU, from any context or
 * stream, race.  The first call for a geometry builds its tables on the host
 * (host memory only); later calls copy the view constants (2 * n_views
 * values) into the array and launch two kernels. */
gkb_status gkb_back_noalloc(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *y, void *x);

/* AB-GKB (Alg. "AB-GKB"): GKB on M = AB from b; x = B Q_k u_k.
 * BA-GKB (Alg. "BA-GKB"): GKB on M = BA from B b; x = Q_k u_k.
 * Matched GKB (Alg. "GKB"): M = A, M^T = A^T; x = Q_k u_k (equivalent to LSQR).
 * u_k = argmin ||C_k u - t_1 e_1||^2 + lambda^2 ||u||^2 (eq. proj GKB).
 * GKB_F32 keeps projectors and Krylov vectors in float and every reduction,
 * alpha, t, the projected solve and the discrepancy test in double. */
gkb_status gkb_ab_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                        void *x, gkb_solve_info *info);
gkb_status gkb_ba_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                        void *x, gkb_solve_info *info);
gkb_status gkb_gkb_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                         void *x, gkb_solve_info *info);

/* The paper's comparison methods (Sec. 2.1), from x_0 = 0 on the same
 * projectors:
 *   AB-GMRES (Alg. "AB-GMRES"): GMRES on A B y = b with B as right
 *     preconditioner; Arnoldi basis in R^m from r_0 = b; x_k = B Q_k u_k.
 *   BA-GMRES (Alg. "BA-GMRES"): GMRES on B A x = B b with B as left
 *     preconditioner; Arnoldi basis in R^n from r_0 = B b; x_k = Q_k u_k.
 * u_k = argmin ||H_k u - ||r_0|| e_1|| (eq. proj) with the (k+1) x k upper
 * Hessenberg H_k of the Arnoldi relation M Q_k = Q_{k+1} H_k (eq. Arn iter).
 * The Arnoldi vectors are orthogonalised by two classical Gram-Schmidt rounds,
 * the second's inner products taken from the Gram matrix of the stored basis
 * (the coefficients of both rounds form H_k's column; the paper prints one
 * modified pass, equal up to rounding), and u_k comes from a Givens QR of
 * H_k updated once per iteration (the paper uses the SVD).  The stopping
 * rules are those of the GKB solves on ||A x_k - b|| (eqs. DP and RNS), which
 * is evaluated as ||Y_k u_k - b|| from the stored A-images Y (AB: A B q_i;
 * BA: A q_i: m x k_max extra values of the vector type); breakdown when
 * h_{k+1,k} vanishes (x_k is then the least-squares solution on an invariant
 * Krylov space).
 * Options as for the GKB solves, except: lambda must be 0 and precond NULL
 * (GKB_EUNSUPPORTED otherwise); k_max <= 1024 (GKB_EINVAL); reorth is
 * ignored (the Arnoldi basis is always orthogonalised).  Histories:
 * residual_history as for GKB; alpha_history[0] = ||r_0||, alpha_history[k] =
 * h_{k+1,k}; t_history is zeroed.  info->t1 = ||r_0||, info->alpha1 = h_{2,1},
 * info->proj_residual = ||H_k u_k - ||r_0|| e_1||. */
gkb_status gkb_ab_gmres_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b,
                              const gkb_solve_opts *o, void *x, gkb_solve_info *info);
gkb_status gkb_ba_gmres_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b,
                              const gkb_solve_opts *o, void *x, gkb_solve_info *info);

/* Hybrid regularisation and the enlarged-subspace TSVD on AB-/BA-GKB.  The
 * paper names both (a regularisation parameter chosen inside the Krylov
 * subspace, on the projected problem: Sec. 1, Sec. 6; an enlarged subspace
 * truncated back to rank k: Sec. 3.1) but fixes no rule; the rules here:
 *   lambda_rule GKB_LAMBDA_DP: iteration k solves min ||C_k u - t_1 e_1||^2 +
 *     lambda_k^2 ||u||^2 with lambda_k such that ||C_k u - t_1 e_1|| =
 *     tau_proj * eta_proj, eta_proj the noise norm in the projected
 *     residual's space (AB-GKB: ||e||; BA-GKB: ||B e||); lambda_k = 0 while
 *     the residual at lambda = 0 is at least that level;
 *   lambda_rule GKB_LAMBDA_GCV: lambda_k minimises ||C_k u - t_1 e_1||^2 /
 *     trace(I - C_k (C_k^T C_k + lambda^2 I)^-1 C_k^T)^2;
 *   both search [1e-10 s, 10 s], s = max_i ||C_k e_i||, and take a root or
 *   minimum outside it at the range's end.  rho_k = ||A x_k - b|| is formed
 *   from the stored A-images (m x k_max extra values of the vector type, as
 *   for GMRES) and the options' stopping rules act on it;
 *   tsvd_rank r >= 1 (lambda_rule GKB_LAMBDA_FIXED, lambda 0): the plain
 *   iteration runs to its stop (k_max, or earlier by a stopping rule or a
 *   breakdown), then x = Q_K u (B Q_K u) with u the rank-r truncated SVD
 *   solution of min ||C_K u - t_1 e_1|| (one-sided Jacobi in FP64, K x K and
 *   (K+1) x K doubles of workspace); info->residual is ||A x - b|| of that x.
 * lambda_history (HOST, k_max entries, may be NULL) receives lambda_k.
 * Errors: GKB_EINVAL for a rule outside the enum, neither a rule nor a rank,
 * both, a rank outside [1, k_max], a negative or non-finite tau_proj or
 * eta_proj, lambda != 0, or k_max > 1024; GKB_EUNSUPPORTED for a learned
 * filter (precond). */
typedef enum { GKB_LAMBDA_FIXED = 0, GKB_LAMBDA_DP = 1, GKB_LAMBDA_GCV = 2 } gkb_lambda_rule;
typedef struct {
  int lambda_rule;         /* gkb_lambda_rule */
  double tau_proj;         /* discrepancy rule: level tau_proj * eta_proj */
  double eta_proj;
  int tsvd_rank;           /* 0: off */
  double *lambda_history;  /* HOST, k_max entries, or NULL */
} gkb_hybrid_opts;
gkb_status gkb_ab_hybrid_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b,
                               const gkb_solve_opts *o, const gkb_hybrid_opts *h, void *x, gkb_solve_info *info);
gkb_status gkb_ba_hybrid_solve(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const void *b,
                               const gkb_solve_opts *o, const gkb_hybrid_opts *h, void *x, gkb_solve_info *info);

/* Batched multi-slice solve: n_slices independent problems, each with its own
 * geometry, b, options (k_max, lambda, tau, noise_norm, reorth, histories)
 * and discrepancy stop, solved by AB-GKB (method GKB_METHOD_AB) or BA-GKB
 * (GKB_METHOD_BA) exactly as gkb_ab_solve / gkb_ba_solve would solve each
 * one (same kernels and workgroup partitions per slice, hence the same
 * results bit for bit), but with every kernel launch covering all slices
 * that have not yet stopped.  geoms[s], b[s] (DEVICE, m_s elements), opts[s], x[s] (DEVICE,
 * n_s elements) and info[s] describe slice s; info may be NULL.
 * Constraints: 1 <= n_slices <= 1024; all geometries 2D and of one kind
 * (all GKB_PAR2D or all GKB_FAN2D); opts[s].precond must be NULL.
 * Errors: GKB_EINVAL for a bad argument in any slice (the message names the
 * slice); GKB_ENONFINITE if any b[s] holds NaN/Inf (no x is written).
 * info[s].seconds is the wall time of the whole batched call. */
typedef enum { GKB_METHOD_AB = 0, GKB_METHOD_BA = 1 } gkb_method;
gkb_status gkb_batch_solve(gkb_ctx *ctx, int method, int n_slices, const gkb_geometry *geoms, int dtype,
                           const void *const *b, const gkb_solve_opts *opts, void *const *x, gkb_solve_info *info);

/* Autotuning of launch shapes.  For a GKB_PAR2D geometry the parallel-beam
 * A^T is launched with 1, 2 or 4 views per step of each thread (2 and 4 read
 * every view's full candidate window so that the loads of the views are in
 * flight together) and B with 4 or 8 views per step; the terms are added in
 * the same order either way, so results do not change, only time.
 * gkb_autotune times every choice on the device (mean of five launches after
 * a warm-up, on a constant sinogram of the geometry), keeps the fastest in
 * the context's tables for (g, dtype), where every later projector call and
 * solve takes it from (a batch takes the choice of its slice with the most
 * pixel-views), and returns the measured times in microseconds (0 where not
 * run).  Other geometry kinds have no choices: the call returns the fixed
 * ones.  gkb_set_tuning sets them directly.  Untuned geometries use 4 and 8.
 * gkb_autotune is asynchronous to nothing: it synchronises on its events. */
typedef struct {
  int at_views_per_step;  /* 1, 2 or 4 */
  int b_views_per_step;   /* 4 or 8 */
  double at_us[3];        /* A^T with 1, 2, 4 views per step */
  double b_us[2];         /* B with 4, 8 views per step */
} gkb_tuning;
gkb_status gkb_autotune(gkb_ctx *ctx, const gkb_geometry *g, int dtype, gkb_tuning *t);
gkb_status gkb_set_tuning(gkb_ctx *ctx, const gkb_geometry *g, int dtype, const gkb_tuning *t);

/* How gkb_batch_solve issues its iterations on this context:
 *   GKB_BATCH_LAUNCHES (default): every step of an iteration is one kernel
 *     launch over all active slices;
 *   GKB_BATCH_GRAPH: the same launches are captured once into a hipGraph
 *     and replayed each iteration; the graph is captured again when slices
 *     stop.  Capture runs on a stream the context creates.
 * Results are bit for bit the same in both modes. */
typedef enum { GKB_BATCH_LAUNCHES = 0, GKB_BATCH_GRAPH = 1 } gkb_batch_mode;
gkb_status gkb_set_batch_mode(gkb_ctx *ctx, int mode);

/* ---- Learned sinogram filter inside B (BA-GKB only) ----
 * BA-GKB (Alg. "BA-GKB") applies B and B^T only, so a linear filter F on
 * the sinogram side of B keeps the algorithm as it is: M = B F A,
 * M^T = A^T F^T B^T, right-hand side B F b.  F is the frozen-mask
 * linearisation at the measured b of a bias-free 1D convolutional network N
 * along the detector axis of every view (every detector row in 3D):
 * 1 -> 32 -> 32 -> 32 -> 1 channels, kernel 9, zero "same" padding, ReLU
 * after layers 1-3; with the ReLU masks of b frozen, F is linear, F b = N(b),
 * and F^T is its exact transpose.  The discrepancy test stays on
 * ||A x - b||.  Set gkb_solve_opts.precond to a network to use it (GKB_F32,
 * gkb_ba_solve); if the learned solve does not reach the discrepancy level
 * (by k_max; the attempt ends earlier once its residual, falling at its mean
 * rate of the last five iterations, would still be above the level at
 * k_max), breaks down before iteration 3 or meets a non-finite value, the
 * plain BA-GKB result is returned with reason GKB_STOP_FALLBACK
 * (info->seconds then covers both solves).
 *
 * Weights: FP32 master copy of 19008 values, W1 [32][1][9], W2 [32][32][9],
 * W3 [32][32][9], W4 [1][32][9] ([out][in][tap], concatenated); every layer
 * uses them rounded to bfloat16.  The 32 -> 32 layers run on the matrix cores
 * (bfloat16 operands, FP32 accumulation); inside GKB each FP32 activation
 * enters them as three bfloat16 terms, so F is applied at FP32 accuracy.
 * Training (bfloat16 inputs of layers 2, 3 and bfloat16 gradients through
 * them): one of the objectives below, Adam (beta 0.9 / 0.999, eps 1e-8) with
 * bias correction.
 * A network belongs to the device of the context it was created with. */
gkb_status gkb_net_create(gkb_ctx *ctx, gkb_net **net, int channels, int ksize, int layers,
                          unsigned long long seed);   /* channels 32, ksize 9, layers 4; He initialisation */
void gkb_net_destroy(gkb_net *net);
gkb_status gkb_net_set_weights(gkb_net *net, const float *w, long long count);  /* HOST w[19008]; resets Adam */
gkb_status gkb_net_get_weights(const gkb_net *net, float *w, long long count);  /* HOST w[19008] */
gkb_status gkb_net_save(const gkb_net *net, const char *path);  /* "GKBNET1\0", int32 {32, 9, 4, 19008}, FP32 weights */
gkb_status gkb_net_load(gkb_net *net, const char *path);
/* out = N(y) for a sinogram y of geometry g (DEVICE, FP32, m elements each). */
gkb_status gkb_net_apply(gkb_ctx *ctx, const gkb_net *net, const gkb_geometry *g, const void *y, void *out);
/* out = F y (transpose = 0) or F^T y (transpose = 1), F frozen at b (DEVICE, FP32, m elements each). */
gkb_status gkb_net_frozen_apply(gkb_ctx *ctx, const gkb_net *net, const gkb_geometry *g, const void *b,
                                const void *y, void *out, int transpose);
/* Training objectives, per sample (b_i, x_i), averaged over the batch:
 *  GKB_NET_FBP:    ||B N(b_i) - x_i||^2 / ||x_i||^2 (learned filtered back projection);
 *  GKB_NET_FROZEN: ||B F_{b_i} (A x_i) - x_i||^2 / ||x_i||^2, the filter frozen at the measured b_i
 *                  (masks held fixed) applied to the noise-free data, i.e. the operator M = B F A
 *                  that BA-GKB iterates with. */
typedef enum { GKB_NET_FBP = 0, GKB_NET_FROZEN = 1 } gkb_net_objective;
/* Mean training loss over a batch and its gradient: b DEVICE [batch][m], x DEVICE [batch][n] (FP32, 2D
 * geometry); *loss and the HOST gradient grad[19008] (may be NULL).  Blocks until done. */
gkb_status gkb_net_grad(gkb_ctx *ctx, gkb_net *net, const gkb_geometry *g, int batch, const void *b,
                        const void *x, int objective, double *loss, float *grad);
/* gkb_net_grad followed by one Adam step with learning rate lr. */
gkb_status gkb_net_train_step(gkb_ctx *ctx, gkb_net *net, const gkb_geometry *g, int batch, const void *b,
                              const void *x, int objective, double lr, double *loss);

/* Host-side check of a geometry against the projector kernels' address
 * arithmetic; needs no GPU and touches no device memory.  Every stride-th
 * wavefront (2D ray-driven kernels, cone B^T), ray (cone A), pixel or voxel
 * of the launches that gkb_forward, gkb_back, gkb_forward_adjoint and
 * gkb_back_adjoint make for (g, dtype) is replayed on the host in the
 * kernels' arithmetic, and stats[0..3] (A, B, A^T, B^T) count:
 *   units          rays, pixels or voxels replayed;
 *   reads          element reads;
 *   out_of_bounds  reads outside their zero-padded line (2D) or the padded
 *                  volume or sinogram (cone): must be 0;
 *   uncovered      interpolation candidates (their weights found in double
 *                  from the operator's definition, the linear or bilinear
 *                  weights of Sec. 1's A and B) that lie outside the window
 *                  or line range the kernel reads, with a weight above the
 *                  rounding bound of the kernel's coordinates (GKB_F32:
 *                  8 L 2^-24, L = max(nx, ny, nz, n_det_u, n_det_v) + 16, as a
 *                  float coordinate moves a window edge by a few units in its
 *                  last place; GKB_F64: 1e-9): must be 0;
 *   max_uncovered_weight  the largest such weight (any size).
 * *orders_ok (may be NULL) is 1 when the dispatch orders of the 2D ray-driven
 * kernels are permutations of their launches' workgroups (1 for cone beam).
 * Windows of the pixel-driven fan-beam kernels, which depend on approximated
 * fan angles, are checked with the detector coordinate moved 1e-3 bins both
 * ways.  Errors: GKB_EINVAL (bad geometry, stride < 1, stats NULL) and the
 * geometries the projectors reject with GKB_EUNSUPPORTED. */
typedef struct {
  long long units, reads, out_of_bounds, uncovered;
  double max_uncovered_weight;
} gkb_check_stats;
gkb_status gkb_check_geometry(const gkb_geometry *g, int dtype, int stride, gkb_check_stats *stats, int *orders_ok);

/* Kernel timing.  While enabled, every launch of the named kernels is
 * bracketed by HIP events on the context's stream; gkb_trace_get returns the
 * launch count and summed device milliseconds since the last reset.  Each
 * event pair costs the stream a few microseconds between launches.
 * gkb_trace_only restricts the recording to one kernel name (NULL or "":
 * every kernel again).  Names: "fwd" (A), "back" (B), "fwd_adj" (A^T),
 * "back_adj" (B^T), "reorth", "small_solve", "residual", "filter",
 * "filter_t". */
gkb_status gkb_trace_enable(gkb_ctx *ctx, int on);
gkb_status gkb_trace_only(gkb_ctx *ctx, const char *kernel);
gkb_status gkb_trace_reset(gkb_ctx *ctx);
gkb_status gkb_trace_get(gkb_ctx *ctx, const char *kernel, int *count, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* GKB_H */
