// Internal declarations shared by the HIP translation units of libgkb.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gkb {

constexpr int kBlock = 256;
// Pixel-driven 2D kernels: a workgroup covers a kPixTileX x kPixTileY pixel
// tile with kViewGroups groups of threads, group g taking the views
// g, g + kViewGroups, ...; the groups' sums meet in LDS.
constexpr int kPixTileX = 32, kPixTileY = 2, kViewGroups = 4;
static_assert(kPixTileX * kPixTileY * kViewGroups == kBlock, "pixel tile must fill the workgroup");
// FP32 A from line segments: stage four lines' 64-element segments per
// 16-byte load through the wavefront's LDS (true), or load one element per
// lane and line and exchange it between lanes (false).
constexpr bool kFwdSegStage = true;
// lines per step of the staged form (a multiple of 4)
constexpr int kFwdStageLines = 8;
// Last-level cache (Infinity Cache) of the MI355X: a stored basis larger than
// this is read with nontemporal loads in the reorthogonalisation passes.
constexpr long long kLlcBytes = 256LL << 20;

// Integer fields of the device control block.
enum CtlInt : int {
  CI_K = 0,       // current iteration k (0 during the start-up step)
  CI_STOP = 1,    // 1 once the iteration has stopped
  CI_KSTOP = 2,   // iteration whose solution is returned
  CI_REASON = 3,  // gkb_stop_reason
  CI_COUNT = 8
};

// Double fields of the device control block.
enum CtlDbl : int {
  CD_TAUE = 0,     // tau * ||e||
  CD_LAMBDA = 1,   // Tikhonov weight
  CD_ETAEPS = 2,   // breakdown threshold factor: 100 * unit roundoff of the vector type
  CD_BSCALE = 3,   // max_i sqrt(alpha_i^2 + t_{i+1}^2)
  CD_RHOBAR = 4,   // Givens QR state of [C_k; lambda I]
  CD_PHIBAR = 5,
  CD_CPREV = 6,
  CD_SPREV = 7,
  CD_PSI2 = 8,
  CD_PRES = 9,     // projected residual at k
  CD_USEDP = 10,
  CD_KMAX = 11,
  CD_BNORM = 12,   // ||b||
  CD_RNS = 13,     // residual norm stagnation tolerance (0 = off)
  CD_XTNORM = 14,  // ||x_true|| for the relative reconstruction error
  CD_HRULE = 15,   // hybrid solves: rule choosing lambda_k on C_k (1 discrepancy, 2 GCV)
  CD_HTARGET = 16, // hybrid discrepancy rule: tau * eta of the projected residual
  CD_FINALRES = 17,  // ||A x - b|| of a solution formed after the iteration (TSVD)
  CD_REACH = 18,   // 1: stop once the residual cannot reach tau ||e|| by k_max at its recent rate
  CD_COUNT = 20
};

// Views into the control block (device memory).  Arrays indexed 1-based by
// iteration: alpha[1..K+1], t[1..K+1], rho[1..K], ...
struct Ctl {
  int *ip;
  double *dp;
  double *alpha;
  double *t;
  double *rho;
  double *pres;
  double *u;      // [K+1], u[1..k]
  double *Rd;     // diagonal of R
  double *Rth;    // superdiagonal of R (Rth[i] couples columns i-1, i)
  double *Rphi;   // rotated right-hand side
  double *c;      // CGS coefficients [K+1]
  double *rre;    // [K+2] RRE(x_k) at rre[k] (single-slice solves with x_true; else null)
  double *lamh;   // [K+2] lambda_k at lamh[k] (hybrid solves; else null)
  double *aw;     // [m] A-image of the last column of W = Q R^{-1}
  double *r;      // [m] r_k = A x_k - b
  int *host_stop; // host-mapped mirror of ip[CI_STOP] (may be null)
  int K;
  // GMRES: Hessenberg / triangular columns, column j (1-based) at hm + j * ldh
  // (rows 0..j); the Givens rotations in Rd (cosines) and Rth (sines), the
  // rotated right-hand side in Rphi[1..k+1].  Null for GKB.
  double *hm;
  long long ldh;
  // Gram matrix of the stored basis, G = Q^T Q ((K+1) x (K+1), FP64, row-major,
  // ld K + 1): row k-1 is completed at iteration k by the delayed second
  // Gram-Schmidt round (null where the classical two-round form runs)
  double *gram;
};

// A vector selected by the device-side iteration counter:
// address = base + (k + off) * ld (k read from ip[CI_K]); kptr == nullptr -> base.
template <typename T>
struct Col {
  T *base;
  long long ld;
  int off;
  const int *kptr;
  __host__ __device__ T *get() const {
    return kptr ? base + (long long)(*kptr + off) * ld : base;
  }
};

// Epilogue of a projector kernel:
//   out = raw * in_scale + prev_coef * prev
// in_scale: 1 or 1/t[k+1]; prev_coef: 0, -alpha[k]/t[k] or -t[k+1].
// Optionally stores raw to out_raw and reduces ||out||^2 into t[k+1].
enum EpiIn : int { IN_ONE = 0, IN_INV_TNEXT = 1 };
enum EpiPrev : int { PREV_NONE = 0, PREV_NEG_ALPHA_OVER_T = 1, PREV_NEG_TNEXT = 2 };

// A padded copy of a kernel's output, in the layout the next projector reads,
// written besides the output itself.  Only interior positions are written:
// the pads keep the zeros they were given when the solve started.
enum PadKind : int {
  PADK_IMAGE = 0,   // image [ny][nx]: row-major region (and the column-major one at offT >= 0)
  PADK_SINO = 1,    // sinogram [nv][nu]: rows of lead = nu + 2 off0
  PADK_SINO_W = 2   // sinogram as (w y, w) pairs (fan-beam A^T), w per ray
};
template <typename T>
struct PadOut {
  T *dst;              // nullptr: no padded copy
  int kind;            // PadKind
  int n1;              // image: nx; sinogram: nu
  int lead;            // image: ldR; sinogram: ldY
  int off0;            // image: pad; sinogram: padY
  int ldT;             // image: column-major line length
  long long offT;      // image: column-major region (-1: none)
  const T *w;          // PADK_SINO_W: per-ray weights
};

template <typename T>
struct Epi {
  Ctl ctl;             // valid when use_ctl
  int use_ctl;
  int in_sel;
  int prev_sel;
  int norm_to_t;       // 1: reduce ||out||^2 into t[k+1]
  Col<const T> prev;
  Col<T> out_raw;      // base == nullptr: not stored
  double *partials;    // per-block partial sums of ||out||^2 (norm_to_t)
  PadOut<T> pout;      // padded copy of the output (pout.dst == nullptr: none)
};

// Geometry tables kept in device memory (one set per geometry and dtype).
template <typename T>
struct RayTab {        // per ray, m entries: ray-driven kernels (A, B^T)
  const T *base;       // crossing coordinate (pixel index units) at the middle line
  const T *slope;      // d(crossing)/d(line)
  const T *w;          // 1/|d_dom|
  const int *meta;     // lines of A: lo | hi << 15 | rowdom << 30
  const int *meta_bt;  // lines of B^T: lo | hi << 15 | rowdom << 30
  const T *h;          // B^T candidate half-width (pixel index units)
  // fan-beam B^T
  const T *t0;         // distance from the source to the crossing at the middle line
  const T *dt;         // its change per line
  const T *dperp;      // signed perpendicular-distance change per unit offset along the line
  const T *dpar;       // along-ray distance change per unit offset along the line
  // fan-beam A^T: 1/|d_dom| per ray in padded sinogram layout (zeros in the pads)
  const T *wpad;
  // dispatch order of the workgroups of A and B^T: workgroup b of a launch
  // takes tile order[b]; tiles with the longest rays come first, so that the
  // last workgroups to start are short ones
  const int *order_fwd;
  const int *order_bt;
};

template <typename T>
struct ViewTab {       // per view (pixel-driven kernels B, A^T)
  const T *p0;         // PAR: cos/du            FAN: cos(beta)
  const T *p1;         // PAR: sin/du            FAN: sin(beta)
  const T *p2;         // PAR: 1/|d_dom|
  const T *p3;         // PAR: du/|d_dom| (A^T hat slope in bins)
  const T *p4;         // PAR: |d_dom|/du (A^T hat half-width in bins)
  const T *gcos;       // FAN: (cos(gamma_k), sin(gamma_k)) pairs, padded like a sinogram row [2 (n_det + 2 padY)]
  const T *htile;      // FAN: A^T candidate half-width bound per (32x2 pixel tile, view), [tile][view]
};

struct GeomDev {
  int kind;
  int nx, ny, nv, nu;
  long long n, m;
  double du;           // bin pitch (length or radians)
  double D;            // source distance (fan)
  double off;          // (nu-1)/2
  double inv_du;
  double hmax_fan;     // fan A^T: candidate half-width per unit asin(|d_dom|/|p-S|), in bins
  double tan_dg;       // fan B^T: tan(bin pitch)
  double dd_spread;    // fan A^T: bound on the |d_dom| change across the candidate rays
  int fast_atan;       // fan, float: every pixel's fan angle has |tan| <= 0.5
  int bt_fast;         // fan B^T, float: series forms of the candidate weights (relative error <= 1e-6)
  int at_fast;         // fan A^T, float: first-order sine of the candidate angles (relative error <= 1e-6)
  int fwd_seg;         // A, float: adjacent rays cross a line less than a pixel apart (segment loads)
  // tuned launch choices (see gkb_autotune): parallel-beam A^T views per step
  // (1, 2 or 4) and B views per step (4 or 8); results do not depend on them
  int at_vu, b_vu;
  // padded image: row-major region (ny lines of ldR = nx + 2 pad), then the
  // column-major region at offT (nx lines of ldT = ny + 2 pad)
  int pad, ldR, ldT;
  long long offT;
  long long pad_elems;
  // padded sinogram: nv lines of ldY = nu + 2 padY
  int padY, ldY;
  long long ypad_elems;
  int nc_bt;           // B^T candidates per line
  int nc_at;           // A^T candidate bins per view
  double uclamp_at;    // A^T: detector coordinates are clamped to [-uclamp_at, nu-1+uclamp_at]
  // ---- cone beam (kind 2) ----
  int nz, nw;          // volume depth, detector rows
  double dw;           // detector row pitch
  double SDD;          // source to detector
  double offw;         // (nw-1)/2
  double Su, Sw;       // SDD/du, SDD/dw
  double hk_fac;       // A^T: candidate columns within hk_fac/depth of the voxel's detector coordinate
  double dmax3;        // B^T: bound on the depth D - (x cos + y sin) of every padded voxel
  // padded volume: x-dominant copy [i][l+P][j+P] (planes of (nz+2P) x ldX),
  // then at offYD the y-dominant copy [j][l+P][i+P] (planes of (nz+2P) x ldV)
  int P3, ldX, ldV;
  long long planeX, planeY, offYD, vol_pad_elems;
  // padded sinogram for B: [v][r+PY][k+PY], rows of ldSu, views of sliceY
  int PY3, ldSu;
  long long sliceY, sino_pad_elems;
};

// Cone-beam ray tables, one entry per (view, detector column): the ray's
// dominant axis (x or y; the z axis never dominates), its crossing of the
// in-plane coordinate at the middle plane and the slope, the source-distance
// parameter lambda at the middle plane and per plane (lambda * d_z gives z),
// |d_xy|^2, and the plane ranges of A and B^T.
template <typename T>
struct ConeTab {
  const T *base1;      // in-plane index coordinate of the crossing at the middle plane
  const T *slope1;     // its change per plane
  const T *lmid;       // lambda at the middle plane (= -S_ax / d_ax)
  const T *lslope;     // lambda per plane (= 1 / d_ax)
  const T *dxy2;       // d_x^2 + d_y^2 (unnormalised direction, detector at SDD)
  const T *h1;         // B^T: in-plane candidate half-width
  const int *meta;     // planes of A: lo | hi << 15 | ydom << 30
  const int *meta_bt;  // planes of B^T
  const T *pk;         // (1/d_ax, ydom) pairs for A^T
};

// Workgroup index and count within one slice's share of a launch.
struct Blk {
  unsigned id;
  unsigned n;
};

// ---- batched multi-slice solves ----
// Vector operands of a batched launch, resolved per slice on the device
// (k = the slice's iteration counter).
enum BufSel : int {
  BS_NONE = 0,
  BS_B,       // right-hand side b
  BS_X,       // solution x
  BS_S,       // s~ (unnormalised s)
  BS_W,       // w (q~ before normalisation)
  BS_TN,      // n-vector temporary
  BS_TM,      // m-vector temporary
  BS_Q_PREV,  // Q[:, k-1] = q_k
  BS_Y_CUR    // the current A-image Y_k
};

// Everything one slice of a batch needs on the device.
template <typename T>
struct SliceDev {
  GeomDev g;
  RayTab<T> rt;
  ViewTab<T> vt;
  Ctl ctl;
  T *xpad, *ypad;
  T *Q, *yk, *s, *w, *tn, *tm;
  const T *b;
  T *x;
  long long ldq, dimq, dims;
  double *partials;
  int has_coldom;
  int reorth;
};

// Families of per-slice workgroup counts.  pre[f * (na + 1) + a] is the first
// workgroup of active slice a in a launch of family f; pre[f * (na + 1) + na]
// is the launch's total.
enum BlockFam : int {
  BF_RAY = 0,  // ray-driven projectors: ceil(m / 256)
  BF_PIX,      // pixel-driven projectors: 32x2 tiles (2D), 32x8 (cone)
  BF_VQ,       // vector kernels over Q's dimension
  BF_VM,       // vector kernels over m
  BF_PADR,     // row-major image padding
  BF_PADC,     // column-major image padding (32x32 tiles)
  BF_PADS,     // sinogram padding
  BF_VQU,      // CGS update over Q's dimension (upd_blocks)
  BF_VQD,      // inner products of the delayed CGS round over Q's dimension (dots_blocks)
  BF_RAYBT,    // B^T: bt_blocks
  BF_COUNT
};

template <typename T>
struct BatchDev {
  const SliceDev<T> *sd;  // [n_slices]
  const int *active;      // [na] slice ids
  const int *pre;         // [BF_COUNT][na + 1]
  int na;
  int ignore_stop;        // 1: run on stopped slices too
};

// Host-side summary of a batched launch configuration.
struct BatchLaunch {
  int na;
  int tot[BF_COUNT];
  int kmax;      // largest k_max over the slices
  int fan;       // all slices fan beam (else all parallel beam)
  int nc_bt, nc_at;
  int at_vu, b_vu;  // views per step of A^T and B: the tuned choices of the slice with the most pixel-views
};

// Epilogue selection of a batched projector launch (see Epi).
struct EpiCfg {
  int in_sel;
  int prev_sel;
  int prev_buf;     // BufSel of prev
  int norm_to_t;
  int out_raw_buf;  // BufSel of out_raw or BS_NONE
};

// ---- launchers (proj2d.hip) ----
template <typename T>
void launch_pad_image(const GeomDev &g, Col<const T> x, T *pad, bool cols, const int *stop, hipStream_t s);
template <typename T>
void launch_pad_sino(const GeomDev &g, Col<const T> y, T *pad, const int *stop, hipStream_t s);
// input of A^T: the padded sinogram, or for fan beam (w y, w) pairs (2x the elements)
template <typename T>
void launch_pad_sino_adj(const GeomDev &g, const RayTab<T> &rt, Col<const T> y, T *pad, const int *stop,
                         hipStream_t s);
template <typename T>
void launch_fwd(const GeomDev &g, const RayTab<T> &rt, const T *pad, Col<T> y, const Epi<T> &e, const int *stop,
                hipStream_t s);
template <typename T>
void launch_back_adj(const GeomDev &g, const RayTab<T> &rt, const T *pad, Col<T> y, const Epi<T> &e,
                     const int *stop, hipStream_t s);
template <typename T>
void launch_back(const GeomDev &g, const ViewTab<T> &vt, const T *ypad, T *x, const Epi<T> &e, const int *stop,
                 hipStream_t s);
template <typename T>
void launch_fwd_adj(const GeomDev &g, const ViewTab<T> &vt, const RayTab<T> &rt, const T *ypad, T *x,
                    const Epi<T> &e, const int *stop, hipStream_t s);
int pixel_blocks(const GeomDev &g);
int ray_blocks(const GeomDev &g);
int bt_blocks(const GeomDev &g);  // workgroups of B^T (fan: 64 bins x 2 views x 2 halves of the rays)

// ---- cone-beam launchers (cone3d.hip) ----
template <typename T>
void launch_cone_pad_volume(const GeomDev &g, Col<const T> x, T *pad, int want_x, int want_y, const int *stop,
                            hipStream_t s);
template <typename T>
void launch_cone_pad_sino(const GeomDev &g, Col<const T> y, T *pad, const int *stop, hipStream_t s);
template <typename T>
void launch_cone_weight_sino(const GeomDev &g, const ConeTab<T> &ct, Col<const T> y, T *wy, const int *stop,
                             hipStream_t s);
template <typename T>
void launch_cone_fwd(const GeomDev &g, const ConeTab<T> &ct, const T *pad, Col<T> y, const Epi<T> &e,
                     const int *stop, hipStream_t s);
template <typename T>
void launch_cone_back_adj(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt, const T *pad, Col<T> y,
                          const Epi<T> &e, const int *stop, hipStream_t s);
template <typename T>
void launch_cone_back(const GeomDev &g, const ViewTab<T> &vt, const T *ypad, T *x, const Epi<T> &e,
                      const int *stop, hipStream_t s);
template <typename T>
void launch_cone_fwd_adj(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt, const T *wy, T *x,
                         const Epi<T> &e, const int *stop, hipStream_t s);
int cone_voxel_blocks(const GeomDev &g);

// ---- Krylov vector kernels (krylov.hip) ----
int vec_blocks(long long dim);
int upd_blocks(long long dim);  // workgroups of the CGS update
int dots_blocks(long long dim);  // row blocks of the delayed CGS inner products
template <typename T>
void launch_copy(const T *src, T *dst, long long n, hipStream_t s);
template <typename T>
void launch_norm_to(Ctl ctl, const T *v, long long dim, int which, double *partials, hipStream_t s);
// delayed two-round Gram-Schmidt: one read of Q gives c1 = Q^T w and the
// Gram row of the newest column q_k; then c = c1 + (c1 - G c1) in ctl.c, for
// launch_cgs_update (partials: 2 (K+2) doubles per row block)
template <typename T>
void launch_dcgs_dots(Ctl ctl, const T *Q, long long ld, const T *w, long long dim, double *partials, hipStream_t s,
                      bool nt = false);
void launch_dcgs_coef(Ctl ctl, hipStream_t s);
template <typename T>
void launch_cgs_update(Ctl ctl, const T *Q, long long ld, T *w, long long dim, int last, double *partials,
                       hipStream_t s, int reorth = 1);
template <typename T>
void launch_normalize(Ctl ctl, const T *w, T *Q, long long ld, long long dim, hipStream_t s,
                      PadOut<T> pout = PadOut<T>{});
// w -= Q c (reorth != 0) with the partials of ||w||^2, then q_{k+1} = w / alpha_{k+1},
// alpha_{k+1} formed from those partials inside the normalisation; nt: Q's
// columns with nontemporal loads (both passes take the same choice)
template <typename T>
void launch_update_normalize(Ctl ctl, T *Q, long long ld, T *w, long long dim, double *partials, hipStream_t s,
                             int reorth, PadOut<T> pout = PadOut<T>{}, bool nt = false);
template <typename T>
void launch_resid(Ctl ctl, const T *yk, long long m, double *partials, hipStream_t s);
// rre[k_stop] = ||x - x_true|| / dp[CD_XTNORM] (eq. RE); runs after a stop too
template <typename T>
void launch_rre(Ctl ctl, const T *x, const T *x_true, long long n, double *partials, hipStream_t s);
template <typename T>
void launch_resid_init(Ctl ctl, const T *b, long long m, double *partials, hipStream_t s);
// t[k+1] (NORM_T1) or alpha[k+1] (NORM_ALPHA1) = sqrt(sum of nb partials), after
// the kernel that wrote them (a projector with norm_to_t, cgs_update, norm_to);
// skipped when stop is set
void launch_norm_finalize(Ctl ctl, const double *partials, int nb, int which, const int *stop, hipStream_t s);
void launch_small_solve(Ctl ctl, hipStream_t s);
template <typename T>
void launch_solution(Ctl ctl, const T *Q, long long ld, long long dim, T *out, hipStream_t s);
void launch_set_int(int *p, int v, hipStream_t s);

// ---- learned sinogram filter (netk.hip) ----
// Derived weight layouts (see k_net_prep): FP32 for the 1 <-> 32 channel
// layers, bfloat16 [out][tap][in] for the 32 -> 32 layers; *t: the
// transposed filter (flipped taps, channels swapped).
struct NetW {
  float *w1, *w1t, *w4, *w4t;
  __bf16 *w2b, *w3b, *w2t, *w3t;
};
constexpr int kNetC = 32, kNetK = 9;
constexpr int kNetParams = 2 * kNetC * kNetK + 2 * kNetC * kNetC * kNetK;  // 19008
int net_segments(int L, int tile);
// mode: 0 none, 1 compute (ReLU + mask bits), 2 apply frozen mask bits
void launch_net_c1(Col<const float> s, float *out, unsigned *mask, const float *w, int L, long long rows, int mode,
                   const int *stop, hipStream_t st);
void launch_net_c4(const float *a, float *out, const float *w, int L, long long rows, const int *stop,
                   hipStream_t st);
void launch_net_c32(const float *a, float *out, unsigned *mask, const __bf16 *wb, int L, long long rows, int nsplit,
                    int mode, const int *stop, hipStream_t st);
int net_wgrad_blocks();
void launch_net_wgrad32(const float *g, const float *a, float *partials, int L, long long rows, hipStream_t st);
void launch_net_wgrad_edge(const float *G, const float *S, float *partials, int L, long long rows, int sgn,
                           hipStream_t st);
void launch_net_reduce(const float *partials, int nparts, int count, float *out, double scale, hipStream_t st);
void launch_net_adam(float *w, float *m, float *v, const float *g, int n, double lr, double b1, double b2,
                     double eps, int step, hipStream_t st);
void launch_net_prep(const float *W, const NetW &nw, hipStream_t st);
// training loss of one sample: r = xhat - x; sums[0] = ||r||^2, sums[1] = ||x||^2;
// then r *= 2 / (||x||^2 * batch)
void launch_net_resid(const float *xhat, const float *x, float *r, long long n, double *partials, double *sums,
                      hipStream_t st);
void launch_net_scale(float *r, long long n, const double *sums, int batch, hipStream_t st);

// targets of the finalising reductions: t[k+1], alpha[k+1], dp[CD_BNORM] =
// ||b||, and rho[k] = ||r_k|| with the stopping decision of iteration k
enum NormTarget : int { NORM_T1 = 0, NORM_ALPHA1 = 1, NORM_BNORM = 2, NORM_RHO = 3, NORM_XTRUE = 4, NORM_RRE = 5,
                        NORM_GMRHO = 6, NORM_FINAL = 7 };

// ---- GMRES (Algs. "AB-GMRES", "BA-GMRES") on the same vectors and reductions ----
constexpr int kGmMaxK = 1024;  // k_max limit of the GMRES solves
// Hessenberg column k, rows 0..k-1, from the CGS coefficients ctl.c (first
// round: set; second round: added)
void launch_gm_hcol(Ctl ctl, hipStream_t s);
// Givens QR update of H_k with column k (h_{k+1,k} = alpha[k+1]), u_k by back
// substitution, projected residual into pres[k]
void launch_gm_solve(Ctl ctl, hipStream_t s);
// rho_k = ||Y_k u_k - b|| (Y: the A-images, ld a multiple of 4) and the
// stopping decision of iteration k
template <typename T>
void launch_gm_resid(Ctl ctl, const T *Y, long long ld, const T *b, long long m, double *partials, hipStream_t s,
                     int which = NORM_GMRHO, bool nt = false);

// hybrid regularisation (lambda_k chosen on C_k) and the enlarged-subspace
// TSVD: k_max at most kHyMaxK
constexpr int kHyMaxK = 1024;
enum HybridRule : int { HY_FIXED = 0, HY_DP = 1, HY_GCV = 2 };
void launch_hy_lambda(Ctl ctl, hipStream_t s);
void launch_hy_solve(Ctl ctl, hipStream_t s);
// rank-r truncated SVD solution of the projected problem at k_stop into u;
// W: (K+1) K doubles, V: K K doubles of workspace
void launch_tsvd(Ctl ctl, double *W, double *V, int rank, hipStream_t s);
// ||ax - b|| into CD_FINALRES
template <typename T>
void launch_final_residual(Ctl ctl, const T *ax, const T *b, long long m, double *partials, hipStream_t s);

// ---- batched launchers: one launch covers every active slice ----
template <typename T>
void launch_b_pad_image(const BatchDev<T> &bd, const BatchLaunch &bl, int in_sel, hipStream_t s);
template <typename T>
void launch_b_pad_sino(const BatchDev<T> &bd, const BatchLaunch &bl, int in_sel, int adj, hipStream_t s);
template <typename T>
void launch_b_fwd(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s);
template <typename T>
void launch_b_back_adj(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s);
template <typename T>
void launch_b_back(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s);
template <typename T>
void launch_b_fwd_adj(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s);
template <typename T>
void launch_b_copy(const BatchDev<T> &bd, const BatchLaunch &bl, int src_sel, int dst_sel, hipStream_t s);
template <typename T>
void launch_b_norm_to(const BatchDev<T> &bd, const BatchLaunch &bl, int sel, int fam, int which, hipStream_t s);
template <typename T>
void launch_b_norm_finalize(const BatchDev<T> &bd, const BatchLaunch &bl, int fam, int which, hipStream_t s);
template <typename T>
void launch_b_dcgs(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s);
template <typename T>
void launch_b_cgs_update(const BatchDev<T> &bd, const BatchLaunch &bl, int last, hipStream_t s);
template <typename T>
void launch_b_normalize(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s);
template <typename T>
void launch_b_resid(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s);
template <typename T>
void launch_b_resid_init(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s);
template <typename T>
void launch_b_small_solve(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s);
template <typename T>
void launch_b_solution(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, hipStream_t s);
template <typename T>
void launch_b_set_k(const BatchDev<T> &bd, const BatchLaunch &bl, int k, hipStream_t s);
template <typename T>
void launch_b_report(const SliceDev<T> *sd, int ns, int phase, double *out, hipStream_t s);

}  // namespace gkb
