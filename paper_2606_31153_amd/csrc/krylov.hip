// Krylov vector kernels for the AB-/BA-GKB iteration on gfx950.
//
// Precision split: vectors (Q, Y, s, w) are stored in T (float or double);
// every inner product, norm and reorthogonalisation update is formed and
// accumulated in double; alpha, t, the projected solve and the discrepancy
// test are double.  All reductions are deterministic: fixed-order wave
// butterflies, one partial per workgroup, and a fixed-order sum of the
// partials by a one-workgroup finalising kernel launched after the producer
// (no workgroup waits for or signals another).
//
// Reorthogonalisation (one-sided, on q only; Alg. "GKB" step 9 and its
// AB/BA counterparts) is classical Gram-Schmidt applied twice:
//   c1 = Q^T w;  w -= Q c1;  c2 = Q^T w;  w -= Q c2;  alpha = ||w||.
// The projected problem min ||C_k u - t_1 e_1||^2 + lambda^2 ||u||^2
// (eq. proj GKB) is solved by Givens rotations updated once per iteration
// (the factorisation Paige and Saunders use for LSQR, with the damping rows
// for lambda): R_k u_k = phi_k with R_k upper bidiagonal, whose leading
// parts (and phi's leading entries) do not change from one iteration to the
// next.  This gives the same minimiser as the SVD route of the paper in O(k)
// work per iteration.
// The discrepancy residual ||A x_k - b|| (eq. DP) follows from the A-images
// Y_i of the basis (BA, GKB: A q_i; AB: A B q_i): A x_k = Y_k u_k = W_k phi_k
// with W_k = Y_k R_k^{-1}, so with the short recurrences (in double)
//   Aw_k = (Y_k - Rth_k Aw_{k-1}) / Rd_k,   r_k = r_{k-1} + phi_k Aw_k,  r_0 = -b
// r_k = A x_k - b is carried from one iteration to the next at O(m) cost and
// rho_k = ||r_k||; only the current A-image is kept.

#include <algorithm>

#include "batch.h"
#include "epilogue.h"
#include "internal.h"
#include "reduce.h"

namespace gkb {

namespace {

constexpr int CH = 4;   // columns per workgroup in the multi-dot kernels
constexpr int UCH = 16; // columns per unrolled step of the update loops
constexpr int RPT = 4;  // rows per thread (one 4-wide vector load)
constexpr int ROWS_PER_BLOCK = kBlock * RPT;
// Rows r..r+3 of a column (zeros past dim).  Columns are stored with a
// leading dimension that is a multiple of 4, so full quads are aligned.
template <typename T>
__device__ inline void load_quad(const T *__restrict__ p, long long r, long long dim, double (&q)[RPT]) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  if (r + RPT <= dim) {
    const v4 v = *reinterpret_cast<const v4 *>(p + r);
    q[0] = (double)v.x;
    q[1] = (double)v.y;
    q[2] = (double)v.z;
    q[3] = (double)v.w;
  } else {
#pragma unroll
    for (int i = 0; i < RPT; ++i) q[i] = (r + i < dim) ? (double)p[r + i] : 0.0;
  }
}

// A column of the stored basis, read once per pass; nt: with nontemporal
// loads, for a basis larger than the last-level cache, which would otherwise
// push out what the other kernels of the iteration read from it
template <typename T>
__device__ inline void load_quad_q(const T *__restrict__ p, long long r, long long dim, double (&q)[RPT], bool nt) {
  if (nt) {
    typedef T v4 __attribute__((ext_vector_type(4)));
    if (r + RPT <= dim) {
      const v4 v = __builtin_nontemporal_load(reinterpret_cast<const v4 *>(p + r));
      q[0] = (double)v.x;
      q[1] = (double)v.y;
      q[2] = (double)v.z;
      q[3] = (double)v.w;
      return;
    }
  }
  load_quad(p, r, dim, q);
}

template <typename T>
__device__ inline void store_quad(T *__restrict__ p, long long r, long long dim, const T (&q)[RPT]) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  if (r + RPT <= dim) {
    v4 v;
    v.x = q[0];
    v.y = q[1];
    v.z = q[2];
    v.w = q[3];
    *reinterpret_cast<v4 *>(p + r) = v;
  } else {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (r + i < dim) p[r + i] = q[i];
  }
}

// ---- delayed second round of classical Gram-Schmidt ---------------------------
// The second round's coefficients are Q^T (w - Q c1) = c1 - G c1, with G = Q^T Q
// the Gram matrix of the stored (rounded) basis, so that round needs no second
// read of Q: one pass forms c1 = Q^T w together with the Gram row of the newest
// column, Q^T q_k, and one pass subtracts Q (c1 + c2).  In exact arithmetic
// G = I and c2 = 0; with rounding, c2 = (I - G) c1 removes what the stored
// basis has lost of its orthogonality, as the second classical round does.
// Partials: row block bx at bx * 2 (K+2): c1 terms at column j, Gram terms at
// K + 2 + j.
template <int N>
__device__ inline double block_sum_vec_n(double (&v)[N], double *lds /* [4][N] */) {
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] = wave_sum(v[j]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) lds[wid * N + j] = v[j];
  }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < N) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) r += lds[w * N + threadIdx.x];
  }
  return r;
}

// A workgroup takes CH2 columns over kDotsQuads x 1024 rows: the block sums,
// whose cost does not depend on the rows, are spread over four times the rows
// of the other vector kernels.
constexpr int CH2 = 4, kDotsQuads = 4;
template <typename T>
__device__ inline void dots2_body(const Ctl &ctl, const T *__restrict__ V, long long ld, const T *__restrict__ w,
                                  long long dim, double *partials, unsigned bx, unsigned by, int ncol,
                                  bool nt = false) {
  constexpr int CH = CH2;
  const int c0 = by * CH;
  if (c0 >= ncol) return;
  __shared__ double lds[(kBlock / 64) * 2 * CH];
  double acc[2 * CH];
#pragma unroll
  for (int j = 0; j < 2 * CH; ++j) acc[j] = 0.0;
  const T *__restrict__ qk = V + (long long)(ncol - 1) * ld;  // q_k, the newest column
#pragma unroll
  for (int qd = 0; qd < kDotsQuads; ++qd) {
    const long long r = (((long long)bx * kDotsQuads + qd) * kBlock + threadIdx.x) * RPT;
    if (r >= dim) break;
    double wq[RPT], nq[RPT];
    load_quad(w, r, dim, wq);
    load_quad(qk, r, dim, nq);
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      if (c0 + j < ncol) {
        double q[RPT];
        load_quad_q(V + (long long)(c0 + j) * ld, r, dim, q, nt);
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          acc[j] = fma(q[i], wq[i], acc[j]);
          acc[CH + j] = fma(q[i], nq[i], acc[CH + j]);
        }
      }
    }
  }
  const double sum = block_sum_vec_n<2 * CH>(acc, lds);
  const int t = threadIdx.x;
  const long long ldp = ctl.K + 2;
  if (t < 2 * CH) {
    const int j = t < CH ? t : t - CH;
    if (c0 + j < ncol) partials[(long long)bx * 2 * ldp + (t < CH ? 0 : ldp) + c0 + j] = sum;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_dots2(Ctl ctl, const T *__restrict__ V, long long ld,
                                                  const T *__restrict__ w, long long dim, double *partials,
                                                  int nt) {
  if (ctl.ip[CI_STOP]) return;
  dots2_body(ctl, V, ld, w, dim, partials, blockIdx.x, blockIdx.y, ctl.ip[CI_K], nt != 0);
}

// column sums of the two partial sets; workgroup col < K + 1 sums c1[col],
// col - (K + 1) the Gram entry (q_col, q_k), which fills row and column k - 1
// of G
__device__ inline void reduce_cols2_body(const Ctl &ctl, const double *__restrict__ partials, int nb, int col,
                                         int ncol) {
  __shared__ double lds[kBlock / 64];
  const int set = col > ctl.K ? 1 : 0;
  const int j = col - set * (ctl.K + 1);
  if (j >= ncol) return;
  const long long ldp = ctl.K + 2, st = 2 * ldp, off = set * ldp + j;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 3 * kBlock < nb; b += 4 * kBlock) {
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += partials[(long long)(b + u * kBlock) * st + off];
  }
  if (b < nb) acc[0] += partials[(long long)b * st + off];
  if (b + kBlock < nb) acc[1] += partials[(long long)(b + kBlock) * st + off];
  if (b + 2 * kBlock < nb) acc[2] += partials[(long long)(b + 2 * kBlock) * st + off];
  const double tot = block_sum<kBlock>((acc[0] + acc[1]) + (acc[2] + acc[3]), lds);
  if (threadIdx.x == 0) {
    if (set == 0) {
      ctl.c[j] = tot;
    } else {
      const long long ldg = ctl.K + 1, kk = ncol - 1;
      ctl.gram[kk * ldg + j] = tot;
      ctl.gram[(long long)j * ldg + kk] = tot;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_reduce_cols2(Ctl ctl, const double *__restrict__ partials, int nb) {
  if (ctl.ip[CI_STOP]) return;
  reduce_cols2_body(ctl, partials, nb, blockIdx.x, ctl.ip[CI_K]);
}

// c = c1 + (c1 - G c1) over the k columns, in one workgroup (c1 is staged in
// LDS before any c_i is written; each row's product is summed in column order
// within each of a fixed number of column slices, the slices in order)
constexpr int kCoefMaxLds = 4096, kCoefThreads = 1024, kCoefWaves = kCoefThreads / 64;
__device__ inline void dcgs_coef_body(const Ctl &ctl, int k) {
  __shared__ double s_c1[kCoefMaxLds];
  __shared__ double s_part[kCoefWaves][64];
  for (int j = threadIdx.x; j < k; j += kCoefThreads) s_c1[j] = ctl.c[j];
  __syncthreads();
  // G is symmetric: lane i walks column i, so that the lanes of a wavefront
  // read neighbouring entries of one row at each step
  const long long ldg = ctl.K + 1;
  const int nic = (k + 63) / 64;  // 64-row chunks of the result
  if (2 * nic <= kCoefWaves) {
    // nic * S wavefronts, S >= 2: S of them split the sum of each chunk, and
    // their shares are added in a fixed order
    const int S = kCoefWaves / nic, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int ic = wv / S, sl = wv - ic * S, i = ic * 64 + lane;
    const int per = (k + S - 1) / S, j0 = sl * per, j1 = min(k, j0 + per);
    double t = 0.0;
    if (ic < nic && i < k)
      for (int j = j0; j < j1; ++j) t = fma(ctl.gram[(long long)j * ldg + i], s_c1[j], t);
    s_part[wv][lane] = t;
    __syncthreads();
    if (ic < nic && sl == 0 && i < k) {
      for (int v = 1; v < S; ++v) t += s_part[wv + v][lane];
      ctl.c[i] = s_c1[i] + (s_c1[i] - t);
    }
    return;
  }
  // more than 512 rows: one thread per row, in rounds of kCoefThreads rows
  for (int i = threadIdx.x; i < k; i += kCoefThreads) {
    double t = 0.0;
    for (int j = 0; j < k; ++j) t = fma(ctl.gram[(long long)j * ldg + i], s_c1[j], t);
    ctl.c[i] = s_c1[i] + (s_c1[i] - t);
  }
}

__global__ __launch_bounds__(kCoefThreads) void k_dcgs_coef(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  dcgs_coef_body(ctl, ctl.ip[CI_K]);
}

// Wavefronts that share the rows of a CGS update workgroup (and split its
// columns): 4 for vectors of up to 2^19 entries and 2 up to 2^21, whose
// workgroups would otherwise be too few to keep HBM busy (a 737280-entry
// vector gives 720 workgroups of 1024 rows for 256 CUs), else 1.
__host__ __device__ inline int upd_split(long long dim) {
  return dim <= (1LL << 19) ? 4 : (dim <= (1LL << 21) ? 2 : 1);
}

// ---- w -= Q[:, 0..ncols-1] c (FP64 per element); last == 1: partials of
// ||w||^2 (alpha[k+1] = ||w|| by the finalising kernel).  The four wavefronts
// of a workgroup form groups of `split` that share 256 rows (4 per lane); the
// members of a group sum a share of the columns each, added in LDS in a fixed
// order. ----
template <typename T>
__device__ __attribute__((always_inline)) inline void cgs_update_split(const Ctl &ctl, const T *__restrict__ Q,
                                                                      long long ld, T *__restrict__ w, long long dim,
                                                                      int last, double *partials, Blk b, int ncols,
                                                                      bool nt) {
  constexpr int NW = kBlock / 64;
  __shared__ double part[NW - 1][64 * RPT];
  __shared__ double lds[NW];
  const double *__restrict__ cc = ctl.c;
  const int split = upd_split(dim), groups = NW / split;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int grp = wid / split, mem = wid - grp * split;
  const long long r = (((long long)b.id * groups + grp) * 64 + lane) * RPT;
  const int per = (ncols + split - 1) / split;
  const int j0 = mem * per, j1 = min(ncols, j0 + per);
  // the leading member starts from w, the others from 0
  double acc[RPT] = {0.0, 0.0, 0.0, 0.0};
  if (mem == 0) load_quad(w, r, dim, acc);
  for (int c0 = j0; c0 < j1; c0 += UCH) {
#pragma unroll
    for (int j = 0; j < UCH; ++j) {
      if (c0 + j < j1) {
        double q[RPT];
        load_quad_q(Q + (long long)(c0 + j) * ld, r, dim, q, nt);
        const double cj = cc[c0 + j];
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc[i] = fma(-cj, q[i], acc[i]);
      }
    }
  }
  if (split > 1) {
    const int slot = grp * (split - 1) + mem - 1;  // LDS slot of a non-leading member
    if (mem > 0) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) part[slot][lane * RPT + i] = acc[i];
    }
    __syncthreads();
    if (mem == 0) {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        for (int v = 1; v < split; ++v) acc[i] += part[grp * (split - 1) + v - 1][lane * RPT + i];
    }
  }
  double nrm = 0.0;
  if (mem == 0) {
    T out[RPT];
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      out[i] = (T)acc[i];
      nrm = fma((double)out[i], (double)out[i], nrm);
    }
    if (r < dim) store_quad(w, r, dim, out);
  }
  if (last) {
    const double s = block_sum<kBlock>(nrm, lds);
    if (threadIdx.x == 0) partials[b.id] = s;
  }
}

// ---- w -= Q[:, 0..ncols-1] c (FP64 per element), each lane 4 rows and
// every column; last == 1: partials of ||w||^2 ----
template <typename T>
__device__ __attribute__((always_inline)) inline void cgs_update_rows(const Ctl &ctl, const T *__restrict__ Q,
                                                                      long long ld, T *__restrict__ w, long long dim,
                                                                      int last, double *partials, Blk b, int ncols,
                                                                      bool nt) {
  __shared__ double lds[kBlock / 64];
  const double *__restrict__ cc = ctl.c;
  const long long r = ((long long)b.id * kBlock + threadIdx.x) * RPT;
  double acc[RPT];
  load_quad(w, r, dim, acc);
  for (int c0 = 0; c0 < ncols; c0 += UCH) {
#pragma unroll
    for (int j = 0; j < UCH; ++j) {
      if (c0 + j < ncols) {
        double q[RPT];
        load_quad_q(Q + (long long)(c0 + j) * ld, r, dim, q, nt);
        const double cj = cc[c0 + j];
#pragma unroll
        for (int i = 0; i < RPT; ++i) acc[i] = fma(-cj, q[i], acc[i]);
      }
    }
  }
  T out[RPT];
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    out[i] = (T)acc[i];
    nrm = fma((double)out[i], (double)out[i], nrm);
  }
  if (r < dim) store_quad(w, r, dim, out);
  if (last) {
    const double s = block_sum<kBlock>(nrm, lds);
    if (threadIdx.x == 0) partials[b.id] = s;
  }
}

template <typename T>
__device__ __attribute__((always_inline)) inline void cgs_update_body(const Ctl &ctl, const T *__restrict__ Q,
                                                                      long long ld, T *__restrict__ w, long long dim,
                                                                      int last, double *partials, Blk b, int ncols,
                                                                      bool nt = false) {
  if (upd_split(dim) > 1)
    cgs_update_split(ctl, Q, ld, w, dim, last, partials, b, ncols, nt);
  else
    cgs_update_rows(ctl, Q, ld, w, dim, last, partials, b, ncols, nt);
}

// reorth == 0: no columns, only the partials of ||w||^2 (with last == 1)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_update(Ctl ctl, const T *__restrict__ Q, long long ld,
                                                       T *__restrict__ w, long long dim, int last,
                                                       double *partials, int reorth, int nt) {
  if (ctl.ip[CI_STOP]) return;
  cgs_update_body(ctl, Q, ld, w, dim, last, partials, Blk{blockIdx.x, gridDim.x}, reorth ? ctl.ip[CI_K] : 0,
                  nt != 0);
}

// ---- finalising kernel: t[k+1] (which == NORM_T1) or alpha[k+1]
// (NORM_ALPHA1) = sqrt of the sum of nb partials ----
__device__ inline void stop_test(const Ctl &ctl, double rho);
__device__ inline void gm_stop_test(const Ctl &ctl, double rho);

__device__ inline void norm_finalize_body(const Ctl &ctl, const double *__restrict__ partials, unsigned nb,
                                          int which) {
  __shared__ double lds[kBlock / 64];
  const double tot = partial_total<kBlock>(partials, nb, 1, lds);
  if (threadIdx.x == 0) {
    const int k = ctl.ip[CI_K];
    switch (which) {
      case NORM_T1: ctl.t[k + 1] = sqrt(tot); break;
      case NORM_ALPHA1: ctl.alpha[k + 1] = sqrt(tot); break;
      case NORM_BNORM: ctl.dp[CD_BNORM] = sqrt(tot); break;
      case NORM_XTRUE: ctl.dp[CD_XTNORM] = sqrt(tot); break;
      case NORM_RRE: ctl.rre[ctl.ip[CI_KSTOP]] = sqrt(tot) / ctl.dp[CD_XTNORM]; break;
      case NORM_GMRHO: gm_stop_test(ctl, sqrt(tot)); break;
      case NORM_FINAL: ctl.dp[CD_FINALRES] = sqrt(tot); break;
      default: stop_test(ctl, sqrt(tot)); break;  // NORM_RHO
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_norm_finalize(Ctl ctl, const double *__restrict__ partials, int nb,
                                                          int which, const int *stop) {
  if (stop && *stop) return;
  norm_finalize_body(ctl, partials, (unsigned)nb, which);
}

// ---- Q[:, k] = w / alpha[k+1] ------------------------------------------------
template <typename T>
__device__ inline void normalize_body(const Ctl &ctl, const T *__restrict__ w, T *__restrict__ Q, long long ld,
                                      long long dim, unsigned blk, const PadOut<T> &pout, double alpha) {
  const int k = ctl.ip[CI_K];
  const double inv = 1.0 / alpha;
  T *q = Q + (long long)k * ld;
  const long long r = ((long long)blk * kBlock + threadIdx.x) * RPT;
  if (r >= dim) return;
  double v[RPT];
  load_quad(w, r, dim, v);
  T out[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) out[i] = (T)(v[i] * inv);
  store_quad(q, r, dim, out);
  if (pout.dst) {
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (r + i < dim) pad_store(pout, r + i, out[i]);
  }
}

// q_{k+1} = w / alpha_{k+1}, and optionally its padded copy for the next projector
template <typename T>
__global__ __launch_bounds__(kBlock) void k_normalize(Ctl ctl, const T *__restrict__ w, T *__restrict__ Q,
                                                      long long ld, long long dim, PadOut<T> pout) {
  if (ctl.ip[CI_STOP]) return;
  normalize_body(ctl, w, Q, ld, dim, blockIdx.x, pout, ctl.alpha[ctl.ip[CI_K] + 1]);
}

// The same with alpha[k+1] = sqrt of the sum of the nb partials of ||w||^2,
// which every workgroup forms in the finalising kernel's order (the same
// value); workgroup 0 stores it.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_normalize_fin(Ctl ctl, const T *__restrict__ w, T *__restrict__ Q,
                                                          long long ld, long long dim, PadOut<T> pout,
                                                          const double *__restrict__ partials, int nb) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[kBlock / 64];
  __shared__ double s_alpha;
  const double tot = partial_total<kBlock>(partials, (unsigned)nb, 1, lds);  // valid in thread 0
  if (threadIdx.x == 0) {
    s_alpha = sqrt(tot);
    if (blockIdx.x == 0) ctl.alpha[ctl.ip[CI_K] + 1] = s_alpha;
  }
  __syncthreads();
  normalize_body(ctl, w, Q, ld, dim, blockIdx.x, pout, s_alpha);
}

// ---- projected solve, discrepancy test, advance --------------------------------
// Iteration k has alpha[1..k], t[1..k+1] (and alpha[k+1] unless k == K).
// Givens rotations G = [[c, s], [-s, c]] reduce [C_k; lambda I] to upper
// bidiagonal R (diagonal Rd, superdiagonal Rth) with right-hand side Rphi;
// u_k solves R u = Rphi.  The quantities the serial steps touch are staged in
// LDS; the quadratic form of the residual is spread over the workgroup.
constexpr int kSolveThreads = 256;
constexpr int kMaxKLds = 4096;

__device__ inline void finish_solve(const Ctl &ctl, int k);

__device__ inline void small_solve_body(const Ctl &ctl) {
  const int k = ctl.ip[CI_K];
  double *dp = ctl.dp;
  if (threadIdx.x == 0) {
    const double ak = ctl.alpha[k];
    const double tk1 = ctl.t[k + 1];
    const double lam = dp[CD_LAMBDA];
    double rhobar, phibar;
    if (k == 1) {
      rhobar = ak;
      phibar = ctl.t[1];
      dp[CD_PSI2] = 0.0;
    } else {
      // finish column k: the previous rotation acts on row k, which holds alpha_k
      ctl.Rth[k] = dp[CD_SPREV] * ak;
      rhobar = dp[CD_CPREV] * ak;
      phibar = dp[CD_PHIBAR];
    }
    double rhat = rhobar;
    if (lam > 0.0) {
      rhat = sqrt(rhobar * rhobar + lam * lam);
      const double c1 = rhobar / rhat, s1 = lam / rhat;
      const double psi = s1 * phibar;
      dp[CD_PSI2] += psi * psi;
      phibar = c1 * phibar;
    }
    const double rk = sqrt(rhat * rhat + tk1 * tk1);
    const double c = rhat / rk, s = tk1 / rk;
    ctl.Rd[k] = rk;
    ctl.Rphi[k] = c * phibar;
    dp[CD_CPREV] = c;
    dp[CD_SPREV] = s;
    dp[CD_PHIBAR] = -s * phibar;
  }
  __syncthreads();
  finish_solve(ctl, k);
}

// u_k from R (Rd, Rth) and Rphi, and the projected residual ||C_k u - t_1 e_1||
__device__ inline void finish_solve(const Ctl &ctl, int k) {
  __shared__ double s_u[kMaxKLds + 2];
  __shared__ double s_rd[kMaxKLds + 2];
  __shared__ double s_rth[kMaxKLds + 2];
  __shared__ double s_rphi[kMaxKLds + 2];
  __shared__ double s_red[kSolveThreads / 64];
  double *dp = ctl.dp;
  // reciprocals of the diagonal, formed in parallel, so that the serial
  // back substitution below multiplies instead of dividing
  for (int i = 1 + threadIdx.x; i <= k; i += kSolveThreads) {
    s_rd[i] = 1.0 / ctl.Rd[i];
    s_rth[i] = ctl.Rth[i];
    s_rphi[i] = ctl.Rphi[i];
  }
  __syncthreads();
  // back substitution R u = Rphi (serial, operands in LDS)
  if (threadIdx.x == 0) {
    double un = s_rphi[k] * s_rd[k];
    s_u[k] = un;
    for (int i = k - 1; i >= 1; --i) {
      un = (s_rphi[i] - s_rth[i + 1] * un) * s_rd[i];
      s_u[i] = un;
    }
    s_u[0] = 0.0;
    s_u[k + 1] = 0.0;
  }
  __syncthreads();
  for (int i = 1 + threadIdx.x; i <= k; i += kSolveThreads) ctl.u[i] = s_u[i];
  // projected residual ||C_k u - t_1 e_1||: row i of C_k u is alpha_i u_i + t_i u_{i-1}
  double pr = 0.0;
  for (int i = 1 + threadIdx.x; i <= k + 1; i += kSolveThreads) {
    double r = (i <= k ? ctl.alpha[i] * s_u[i] : 0.0) + (i >= 2 ? ctl.t[i] * s_u[i - 1] : 0.0);
    if (i == 1) r -= ctl.t[1];
    pr = fma(r, r, pr);
  }
  pr = block_sum<kSolveThreads>(pr, s_red);
  if (threadIdx.x == 0) {
    dp[CD_PRES] = sqrt(pr);
    ctl.pres[k] = dp[CD_PRES];
  }
}

constexpr int kReachWindow = 5;

// ---- the discrepancy residual rho_k = ||r_k|| (kept by the recurrences above)
// and the stopping decision of iteration k (thread 0 of a finalising kernel) ----
__device__ inline void stop_test(const Ctl &ctl, double rho) {
  double *dp = ctl.dp;
  const int k = ctl.ip[CI_K];
  ctl.rho[k] = rho;
  // breakdown scale: max_i sqrt(alpha_i^2 + t_{i+1}^2)
  const double ak = ctl.alpha[k], tk1 = ctl.t[k + 1];
  const double sc = fmax(dp[CD_BSCALE], sqrt(ak * ak + tk1 * tk1));
  dp[CD_BSCALE] = sc;
  const double eta = dp[CD_ETAEPS] * sc;
  int reason = 0;
  if (dp[CD_USEDP] != 0.0 && rho <= dp[CD_TAUE])
    reason = 1;  // GKB_STOP_DP
  else if (dp[CD_RNS] > 0.0 && k >= 2 && fabs(ctl.rho[k - 1] - rho) < dp[CD_RNS] * ctl.rho[k - 1])
    reason = 6;  // GKB_STOP_RNS (eq. RNS): the relative change of the residual norm fell below the tolerance
  else if (dp[CD_REACH] != 0.0 && k > kReachWindow &&
           !(fma((ctl.rho[k - kReachWindow] - rho) / kReachWindow, (double)(ctl.K - k), dp[CD_TAUE]) >= rho))
    reason = 6;  // out of reach: at the mean decrease of the last kReachWindow iterations the residual
                 // would still be above tau ||e|| at k_max (a stop for the learned attempt)
  else if (!(tk1 > eta))
    reason = 3;  // GKB_STOP_BREAKDOWN
  else if (k >= ctl.K)
    reason = dp[CD_USEDP] != 0.0 ? 4 : 2;  // DP_NOT_REACHED / KMAX
  else if (!(ctl.alpha[k + 1] > eta))
    reason = 3;
  ctl.ip[CI_KSTOP] = k;
  if (reason) {
    ctl.ip[CI_REASON] = reason;
    ctl.ip[CI_STOP] = 1;
    if (ctl.host_stop) *(volatile int *)ctl.host_stop = 1;
  } else {
    ctl.ip[CI_K] = k + 1;
  }
}

// ---- GMRES (Algs. "AB-GMRES" and "BA-GMRES") -----------------------------------
// Arnoldi (eq. (Arn iter)) uses the reorthogonalisation kernels above: the two rounds'
// coefficients add up to the Hessenberg column, h_{k+1,k} = ||w|| is
// alpha[k+1] and q_{k+1} = w / alpha[k+1] (alpha[1] = ||r_0||).  The
// projected problem (eq. proj) min ||H_k u - ||r_0|| e_1|| is solved by
// Givens rotations updated once per iteration (the usual GMRES
// factorisation; the oracle takes the SVD of H_k): column k gets the k - 1
// earlier rotations and a new one that annihilates h_{k+1,k}, the rotated
// right-hand side g gains one entry, and u_k solves the k x k triangular
// system R u = g.  |g_{k+1}| is the projected residual.

// h_{1..k,k}: the reorthogonalisation coefficients of both rounds (c1 + c2)
__global__ __launch_bounds__(kBlock) void k_gm_hcol(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  const int k = ctl.ip[CI_K];
  double *col = ctl.hm + (long long)k * ctl.ldh;
  for (int i = threadIdx.x; i < k; i += kBlock) col[i] = ctl.c[i];
}

// One wavefront.  The serial rotation steps run in lane 0 on a copy of the
// column in LDS; the back substitution goes column by column with the rows
// spread over the lanes.
__global__ __launch_bounds__(64) void k_gm_solve(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double s_col[kGmMaxK + 2];
  __shared__ double s_g[kGmMaxK + 2];
  const int k = ctl.ip[CI_K];
  const int lane = threadIdx.x;
  double *col = ctl.hm + (long long)k * ctl.ldh;
  const double hk1 = ctl.alpha[k + 1];
  double ss = 0.0;
  for (int i = lane; i < k; i += 64) {
    const double v = col[i];
    s_col[i] = v;
    ss = fma(v, v, ss);
  }
  ss = wave_sum(ss);
  // g_1..g_{k-1} are final; lane 0 forms g_k and g_{k+1}
  for (int i = lane + 1; i < k; i += 64) s_g[i] = ctl.Rphi[i];
  __syncthreads();
  if (lane == 0) {
    double *dp = ctl.dp;
    // breakdown scale: the largest Hessenberg column norm so far
    dp[CD_BSCALE] = fmax(dp[CD_BSCALE], sqrt(fma(hk1, hk1, ss)));
    for (int i = 1; i < k; ++i) {            // rotation i acts on rows i-1, i
      const double c = ctl.Rd[i], sn = ctl.Rth[i];
      const double a = s_col[i - 1], b = s_col[i];
      s_col[i - 1] = c * a + sn * b;
      s_col[i] = c * b - sn * a;
    }
    const double a = s_col[k - 1];
    const double r = sqrt(fma(a, a, hk1 * hk1));
    const double c = r > 0.0 ? a / r : 1.0, sn = r > 0.0 ? hk1 / r : 0.0;
    ctl.Rd[k] = c;
    ctl.Rth[k] = sn;
    s_col[k - 1] = r;
    const double gk = (k == 1) ? ctl.alpha[1] : ctl.Rphi[k];  // g_1 = ||r_0||
    s_g[k] = c * gk;
    ctl.Rphi[k] = c * gk;
    ctl.Rphi[k + 1] = -sn * gk;
    ctl.pres[k] = fabs(sn * gk);
    dp[CD_PRES] = ctl.pres[k];
  }
  __syncthreads();
  for (int i = lane; i < k; i += 64) col[i] = s_col[i];
  // R u = g: u_j from the finished row j, then row j's column leaves the rows above
  for (int j = k; j >= 1; --j) {
    const double *cj = (j == k) ? s_col : ctl.hm + (long long)j * ctl.ldh;
    const double rjj = cj[j - 1];
    const double uj = rjj != 0.0 ? s_g[j] / rjj : 0.0;
    for (int i = lane + 1; i < j; i += 64) s_g[i] = fma(-cj[i - 1], uj, s_g[i]);
    if (lane == 0) ctl.u[j] = uj;
    __syncthreads();
  }
}

// rho_k = ||Y_k u_k - b||: partials of the squared norm, 4 rows per thread,
// four columns of Y per step; nt: Y's columns with nontemporal loads
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gm_resid(Ctl ctl, const T *__restrict__ Y, long long ld,
                                                     const T *__restrict__ bv, long long m, double *partials,
                                                     int nt) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[kBlock / 64];
  const int k = ctl.ip[CI_K];
  const long long r0 = ((long long)blockIdx.x * kBlock + threadIdx.x) * RPT;
  double acc[RPT];
  load_quad(bv, r0, m, acc);
#pragma unroll
  for (int i = 0; i < RPT; ++i) acc[i] = -acc[i];
  int j = 1;
  for (; j + 3 <= k; j += 4) {
    double y[4][RPT];
#pragma unroll
    for (int q = 0; q < 4; ++q) load_quad_q(Y + (long long)(j - 1 + q) * ld, r0, m, y[q], nt != 0);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double uq = ctl.u[j + q];
#pragma unroll
      for (int i = 0; i < RPT; ++i) acc[i] = fma(uq, y[q][i], acc[i]);
    }
  }
  for (; j <= k; ++j) {
    double y[RPT];
    load_quad_q(Y + (long long)(j - 1) * ld, r0, m, y, nt != 0);
    const double uj = ctl.u[j];
#pragma unroll
    for (int i = 0; i < RPT; ++i) acc[i] = fma(uj, y[i], acc[i]);
  }
  double ss = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) ss = fma(acc[i], acc[i], ss);
  const double tot = block_sum<kBlock>(ss, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// the GMRES stopping decision of iteration k: the discrepancy principle and
// residual norm stagnation on rho_k = ||A x_k - b||, then breakdown
// (h_{k+1,k} below 100 eps times the largest Hessenberg column norm), then k_max
__device__ inline void gm_stop_test(const Ctl &ctl, double rho) {
  double *dp = ctl.dp;
  const int k = ctl.ip[CI_K];
  ctl.rho[k] = rho;
  const double eta = dp[CD_ETAEPS] * dp[CD_BSCALE];
  int reason = 0;
  if (dp[CD_USEDP] != 0.0 && rho <= dp[CD_TAUE])
    reason = 1;  // GKB_STOP_DP
  else if (dp[CD_RNS] > 0.0 && k >= 2 && fabs(ctl.rho[k - 1] - rho) < dp[CD_RNS] * ctl.rho[k - 1])
    reason = 6;  // GKB_STOP_RNS
  else if (!(ctl.alpha[k + 1] > eta))
    reason = 3;  // GKB_STOP_BREAKDOWN: the Krylov space is invariant
  else if (k >= ctl.K)
    reason = dp[CD_USEDP] != 0.0 ? 4 : 2;
  ctl.ip[CI_KSTOP] = k;
  if (reason) {
    ctl.ip[CI_REASON] = reason;
    ctl.ip[CI_STOP] = 1;
    if (ctl.host_stop) *(volatile int *)ctl.host_stop = 1;
  } else {
    ctl.ip[CI_K] = k + 1;
  }
}

// ---- residual recurrences: Aw = (Y_k - Rth_k Aw) / Rd_k, r += Rphi_k Aw
// (Aw not read at k = 1), partials of ||r||^2 ----
template <typename T>
__device__ inline void resid_body(const Ctl &ctl, const T *__restrict__ yk, long long m, double *partials, Blk b) {
  __shared__ double lds[kBlock / 64];
  const int k = ctl.ip[CI_K];
  const double th = k > 1 ? ctl.Rth[k] : 0.0, inv = 1.0 / ctl.Rd[k], ph = ctl.Rphi[k];
  const long long r0 = ((long long)b.id * kBlock + threadIdx.x) * RPT;
  double y[RPT], aw[RPT], rr[RPT];
  load_quad(yk, r0, m, y);
  load_quad(ctl.r, r0, m, rr);
  if (k > 1) {
    load_quad(ctl.aw, r0, m, aw);
#pragma unroll
    for (int i = 0; i < RPT; ++i) aw[i] = fma(-th, aw[i], y[i]) * inv;
  } else {
#pragma unroll
    for (int i = 0; i < RPT; ++i) aw[i] = y[i] * inv;
  }
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    rr[i] = fma(ph, aw[i], rr[i]);
    acc = fma(rr[i], rr[i], acc);
  }
  if (r0 < m) {
    store_quad(ctl.aw, r0, m, aw);
    store_quad(ctl.r, r0, m, rr);
  }
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) partials[b.id] = s;
}

// ---- start-up: r_0 = -b, partials of ||b||^2 ----
template <typename T>
__device__ inline void resid_init_body(const Ctl &ctl, const T *__restrict__ bv, long long m, double *partials, Blk b) {
  __shared__ double lds[kBlock / 64];
  const long long r0 = ((long long)b.id * kBlock + threadIdx.x) * RPT;
  double y[RPT], rr[RPT];
  load_quad(bv, r0, m, y);
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    rr[i] = -y[i];
    acc = fma(y[i], y[i], acc);
  }
  if (r0 < m) store_quad(ctl.r, r0, m, rr);
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) partials[b.id] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_resid(Ctl ctl, const T *__restrict__ yk, long long m, double *partials) {
  if (ctl.ip[CI_STOP]) return;
  resid_body(ctl, yk, m, partials, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_resid_init(Ctl ctl, const T *__restrict__ bv, long long m,
                                                       double *partials) {
  resid_init_body(ctl, bv, m, partials, Blk{blockIdx.x, gridDim.x});
}

__global__ __launch_bounds__(kSolveThreads) void k_small_solve(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  small_solve_body(ctl);
}

// ---- hybrid regularisation: lambda_k chosen on C_k ------------------------------
// One pass of the damped reduction of [C_k; lambda I] (as in the projected
// solve, from column 1) carries three sums forward, so that one thread
// evaluates the rules at one lambda with O(k) work and no stored arrays:
//  * the residual of the damped problem, phibar_{k+1}^2 + sum psi_i^2 (psi_i
//    the parts rotated into the lambda rows);
//  * ||u||^2 = ||R^-1 f||^2: rotations from the right turn the upper
//    bidiagonal R into a lower bidiagonal L (the rotation that clears
//    R_{i,i+1} leaves delta_{i+1} = sn rho_{i+1} below the diagonal and
//    -cs rho_{i+1} on it), and ||R^-1 f|| = ||L^-1 f||, solved forward;
//  * ||R^-1||_F^2 = sum_j c_j, c_j = (1 + theta_j^2 c_{j-1}) / rho_j^2: column j
//    of R^-1 is e_j / rho_j plus -theta_j / rho_j times column j - 1.
// Then ||C_k u - t_1 e_1||^2 = damped residual^2 - lambda^2 ||u||^2 and, as
// R^T R = C_k^T C_k + lambda^2 I, trace(I_{k+1} - H(lambda)) = 1 + lambda^2 ||R^-1||_F^2.
struct HyVal {
  double phi2;  // ||C_k u_lambda - t_1 e_1||^2
  double tr;    // trace(I_{k+1} - H(lambda))
};

__device__ inline HyVal hy_eval(const double *__restrict__ a, const double *__restrict__ t, int k, double lam) {
  const double l2 = lam * lam;
  double rhobar = a[1], phibar = t[1], psi2 = 0.0;
  double zprev = 0.0, zz = 0.0, u2 = 0.0, cprev = 0.0, csum = 0.0, thprev = 0.0, cs2 = 1.0, sn2 = 0.0;
  for (int i = 1; i <= k; ++i) {
    double rhat = rhobar;
    if (lam > 0.0) {  // [rhobar; lambda] -> [rhat; 0]
      const double h2 = fma(rhobar, rhobar, l2);
      const double inv = rsqrt(h2);
      rhat = h2 * inv;
      psi2 = fma(l2 * inv * inv, phibar * phibar, psi2);
      phibar *= rhobar * inv;
    }
    // [rhat; t_{i+1}] -> [rho_i; 0]; R_{i,i+1} = theta = s alpha_{i+1}
    const double ti = t[i + 1];
    const double r2 = fma(rhat, rhat, ti * ti);
    const double irho = r2 > 0.0 ? rsqrt(r2) : 0.0;
    const double rho = r2 * irho;
    const double c = rhat * irho, sv = ti * irho;
    const double phi = c * phibar;
    phibar *= sv;
    double theta = 0.0;
    if (i < k) {
      theta = sv * a[i + 1];
      rhobar = -c * a[i + 1];
    }
    const double ci = fma(thprev * thprev, cprev, 1.0) * irho * irho;
    csum += ci;
    cprev = ci;
    const double gb = (i == 1) ? rho : -cs2 * rho;
    const double dl = (i == 1) ? 0.0 : sn2 * rho;
    const double rhs = fma(-dl, zprev, phi);
    if (i < k) {
      const double g2 = fma(gb, gb, theta * theta);
      const double ig = g2 > 0.0 ? rsqrt(g2) : 0.0;
      cs2 = g2 > 0.0 ? gb * ig : 1.0;
      sn2 = theta * ig;
      zprev = rhs * ig;
      zz = fma(zprev, zprev, zz);
    } else {
      const double zb = gb != 0.0 ? rhs / gb : 0.0;
      u2 = fma(zb, zb, zz);
    }
    thprev = theta;
  }
  HyVal v;
  v.phi2 = fmax(fma(phibar, phibar, psi2) - l2 * u2, 0.0);
  v.tr = fma(l2, csum, 1.0);
  return v;
}

// lambda_k on C_k: kHyPasses passes of kSolveThreads values of ln(lambda),
// equally spaced, first over [ln(1e-10 s), ln(10 s)] (s = max_i ||C_k e_i||),
// then over the bracket the previous pass found.
//  discrepancy: F = ||C_k u - t_1 e_1|| - tau eta grows with lambda; lambda = 0
//    when F(0) >= 0, the range's end where F has one sign over it, else the
//    first grid value with F >= 0 and its predecessor bracket the root, and
//    the last pass interpolates F linearly in ln(lambda);
//  GCV: G = ||C_k u - t_1 e_1||^2 / trace(I - H)^2; the grid minimum and its
//    neighbours bracket the next pass, and the last takes the vertex of the
//    parabola through the minimum and its neighbours.
constexpr int kHyPasses = 3;

__global__ __launch_bounds__(kSolveThreads) void k_hy_lambda(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double s_a[kHyMaxK + 2], s_t[kHyMaxK + 2];
  __shared__ double s_v[kSolveThreads];
  __shared__ double s_z[2], s_lam;
  __shared__ int s_done;
  const int k = ctl.ip[CI_K];
  const int tid = threadIdx.x;
  for (int i = 1 + tid; i <= k + 1; i += kSolveThreads) {
    s_a[i] = ctl.alpha[i];
    s_t[i] = ctl.t[i];
  }
  double sc = 0.0;
  for (int i = 1 + tid; i <= k; i += kSolveThreads) sc = fmax(sc, ctl.alpha[i] * ctl.alpha[i] + ctl.t[i + 1] * ctl.t[i + 1]);
  s_v[tid] = sc;
  __syncthreads();
  const int rule = (int)ctl.dp[CD_HRULE];
  const double target = ctl.dp[CD_HTARGET];
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < kSolveThreads; ++j) m = fmax(m, s_v[j]);
    m = sqrt(m);
    s_z[0] = log(1e-10 * m);
    s_z[1] = log(10.0 * m);
    s_done = 0;
    s_lam = 0.0;
    if (!(m > 0.0)) {
      s_done = 1;  // C_k = 0: nothing to regularise
    } else if (rule == HY_DP && sqrt(hy_eval(s_a, s_t, k, 0.0).phi2) >= target) {
      s_done = 1;  // the subspace cannot fit the data to the level yet
    }
  }
  __syncthreads();
  constexpr int N = kSolveThreads;
  for (int pass = 0; pass < kHyPasses && !s_done; ++pass) {
    const double za = s_z[0], zb = s_z[1];
    const double h = (zb - za) / (N - 1);
    const double z = za + h * tid;
    const HyVal v = hy_eval(s_a, s_t, k, exp(z));
    s_v[tid] = rule == HY_DP ? sqrt(v.phi2) - target : v.phi2 / (v.tr * v.tr);
    __syncthreads();
    if (tid == 0) {
      const bool last = pass == kHyPasses - 1;
      if (rule == HY_DP) {
        int j0 = N;
        for (int j = 0; j < N; ++j)
          if (s_v[j] >= 0.0) {
            j0 = j;
            break;
          }
        if (j0 == 0 || j0 == N) {
          s_lam = exp(j0 == 0 ? za : zb);  // the root lies outside the range (first pass only)
          s_done = 1;
        } else {
          const double z0 = za + h * (j0 - 1), fa = s_v[j0 - 1], fb = s_v[j0];
          if (last) {
            s_lam = exp(z0 + h * fa / (fa - fb));
          } else {
            s_z[0] = z0;
            s_z[1] = z0 + h;
          }
        }
      } else {
        int jm = 0;
        for (int j = 1; j < N; ++j)
          if (s_v[j] < s_v[jm]) jm = j;
        const int lo = jm > 0 ? jm - 1 : 0, hi = jm < N - 1 ? jm + 1 : N - 1;
        if (last) {
          double zm = za + h * jm;
          if (jm > 0 && jm < N - 1) {
            const double d2 = s_v[jm + 1] - 2.0 * s_v[jm] + s_v[jm - 1];
            if (d2 > 0.0) zm -= 0.5 * h * (s_v[jm + 1] - s_v[jm - 1]) / d2;
          }
          s_lam = exp(zm);
        } else {
          s_z[0] = za + h * lo;
          s_z[1] = za + h * hi;
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    ctl.dp[CD_LAMBDA] = s_lam;
    ctl.lamh[k] = s_lam;
  }
}

// the projected Tikhonov solution at lambda_k: [C_k; lambda I] reduced from
// column 1 (thread 0; Rth[i + 1] = R_{i,i+1}), then u and the projected residual
__global__ __launch_bounds__(kSolveThreads) void k_hy_solve(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  const int k = ctl.ip[CI_K];
  if (threadIdx.x == 0) {
    const double lam = ctl.dp[CD_LAMBDA];
    double rhobar = ctl.alpha[1], phibar = ctl.t[1];
    for (int i = 1; i <= k; ++i) {
      double rhat = rhobar;
      if (lam > 0.0) {
        rhat = sqrt(rhobar * rhobar + lam * lam);
        phibar *= rhobar / rhat;
      }
      const double ti = ctl.t[i + 1];
      const double rho = sqrt(rhat * rhat + ti * ti);
      const double c = rhat / rho, sv = ti / rho;
      ctl.Rd[i] = rho;
      ctl.Rphi[i] = c * phibar;
      phibar *= sv;
      if (i < k) {
        ctl.Rth[i + 1] = sv * ctl.alpha[i + 1];
        rhobar = -c * ctl.alpha[i + 1];
      }
    }
  }
  __syncthreads();
  finish_solve(ctl, k);
}

// ---- enlarged-subspace TSVD: one-sided Jacobi SVD of C_K (K = k_stop) -----------
// W = C_K (column-major, ld K + 1) and V = I; sweeps of rotations over all
// column pairs (round-robin: K/2 disjoint pairs per round) make the columns of
// W orthogonal, W = U Sigma, C_K = W V^T.  One wavefront takes one pair at a
// time: its lanes hold rows lane, lane + 64, ... of the two columns, the
// three inner products are reduced across the wavefront in a fixed order, and
// the rotation updates the rows in place.  Then
// u = sum over the `rank` largest sigma_i of (t_1 W_{1i} / sigma_i^2) v_i.
constexpr int kJacobiSweeps = 60;
constexpr int kTsvdThreads = 1024;

__device__ inline double wave_sum_all(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kTsvdThreads) void k_tsvd(Ctl ctl, double *__restrict__ W, double *__restrict__ V,
                                                       int rank) {
  __shared__ double s_sig[kHyMaxK + 2];
  __shared__ double s_coef[kHyMaxK + 2];
  __shared__ int s_rot;
  const int K = ctl.ip[CI_KSTOP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = kTsvdThreads / 64;
  const long long ldw = K + 1;
  for (long long e = tid; e < ldw * K; e += kTsvdThreads) {
    const int j = (int)(e / ldw), i = (int)(e - (long long)j * ldw);
    W[e] = i == j ? ctl.alpha[j + 1] : (i == j + 1 ? ctl.t[j + 2] : 0.0);
  }
  for (long long e = tid; e < (long long)K * K; e += kTsvdThreads) V[e] = (e / K == e % K) ? 1.0 : 0.0;
  __syncthreads();
  const int P = K + (K & 1);  // players of the round robin (one idle when K is odd)
  for (int sweep = 0; sweep < kJacobiSweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < P - 1; ++r) {
      for (int p = wave; p < P / 2; p += NW) {
        int i = p == 0 ? P - 1 : (r + p) % (P - 1);
        int j = p == 0 ? r : (r - p + P - 1) % (P - 1);
        if (i >= K || j >= K) continue;
        if (i > j) {
          const int tmp = i;
          i = j;
          j = tmp;
        }
        double *wi = W + (long long)i * ldw, *wj = W + (long long)j * ldw;
        double al = 0.0, be = 0.0, ga = 0.0;
        for (int q = lane; q <= K; q += 64) {
          al = fma(wi[q], wi[q], al);
          be = fma(wj[q], wj[q], be);
          ga = fma(wi[q], wj[q], ga);
        }
        al = wave_sum_all(al);
        be = wave_sum_all(be);
        ga = wave_sum_all(ga);
        if (!(fabs(ga) > 1e-15 * sqrt(al * be))) continue;
        if (lane == 0) s_rot = 1;
        const double zeta = (be - al) / (2.0 * ga);
        const double tn = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tn * tn), sn = cs * tn;
        for (int q = lane; q <= K; q += 64) {
          const double a = wi[q], b = wj[q];
          wi[q] = cs * a - sn * b;
          wj[q] = sn * a + cs * b;
        }
        double *vi = V + (long long)i * K, *vj = V + (long long)j * K;
        for (int q = lane; q < K; q += 64) {
          const double a = vi[q], b = vj[q];
          vi[q] = cs * a - sn * b;
          vj[q] = sn * a + cs * b;
        }
      }
      __syncthreads();
    }
    if (!s_rot) break;
    __syncthreads();
  }
  for (int i = tid; i < K; i += kTsvdThreads) {
    double ss = 0.0;
    for (int q = 0; q <= K; ++q) ss = fma(W[(long long)i * ldw + q], W[(long long)i * ldw + q], ss);
    s_sig[i] = ss;  // sigma_i^2
    s_coef[i] = 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    // the rank largest sigma (ties by index); a zero sigma takes no part
    for (int r = 0; r < rank; ++r) {
      int best = -1;
      for (int i = 0; i < K; ++i)
        if (s_coef[i] == 0.0 && s_sig[i] > 0.0 && (best < 0 || s_sig[i] > s_sig[best])) best = i;
      if (best < 0) break;
      s_coef[best] = ctl.t[1] * W[(long long)best * ldw] / s_sig[best];
    }
  }
  __syncthreads();
  for (int q = tid; q < K; q += kTsvdThreads) {
    double acc = 0.0;
    for (int i = 0; i < K; ++i)
      if (s_coef[i] != 0.0) acc = fma(s_coef[i], V[(long long)i * K + q], acc);
    ctl.u[q + 1] = acc;
  }
}

// ---- out = sum_{i=1..k_stop} u_i Q[:, i-1] -------------------------------------
template <typename T>
__device__ inline void solution_body(const Ctl &ctl, const T *__restrict__ Q, long long ld, long long dim,
                                     T *__restrict__ out, Blk b) {
  const int ks = ctl.ip[CI_KSTOP];
  const long long stride = (long long)b.n * kBlock;
  for (long long r = (long long)b.id * kBlock + threadIdx.x; r < dim; r += stride) {
    double acc = 0.0;
    for (int i = 1; i <= ks; ++i) acc = fma(ctl.u[i], (double)Q[(long long)(i - 1) * ld + r], acc);
    out[r] = (T)acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_solution(Ctl ctl, const T *__restrict__ Q, long long ld,
                                                     long long dim, T *__restrict__ out) {
  solution_body(ctl, Q, ld, dim, out, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__device__ inline void copy_body(const T *__restrict__ a, T *__restrict__ b, long long n, Blk blk) {
  const long long stride = (long long)blk.n * kBlock;
  for (long long r = (long long)blk.id * kBlock + threadIdx.x; r < n; r += stride) b[r] = a[r];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T *__restrict__ a, T *__restrict__ b, long long n) {
  copy_body(a, b, n, Blk{blockIdx.x, gridDim.x});
}

// partials of ||v||^2 (the finalising kernel writes ||v|| into t[k+1] or alpha[k+1])
template <typename T>
__device__ inline void norm_to_body(const T *__restrict__ v, long long dim, double *partials, Blk b) {
  __shared__ double lds[kBlock / 64];
  const long long stride = (long long)b.n * kBlock;
  double acc = 0.0;
  for (long long r = (long long)b.id * kBlock + threadIdx.x; r < dim; r += stride) {
    const double x = (double)v[r];
    acc = fma(x, x, acc);
  }
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) partials[b.id] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm_to(Ctl ctl, const T *__restrict__ v, long long dim,
                                                    double *partials) {
  if (ctl.ip[CI_STOP]) return;
  norm_to_body(v, dim, partials, Blk{blockIdx.x, gridDim.x});
}

// partials of ||a - b||^2 (the reconstruction error of x_k against x_true)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_diff_norm(const T *__restrict__ a, const T *__restrict__ b,
                                                      long long dim, double *partials) {
  __shared__ double lds[kBlock / 64];
  const long long stride = (long long)gridDim.x * kBlock;
  double acc = 0.0;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride) {
    const double d = (double)a[r] - (double)b[r];
    acc = fma(d, d, acc);
  }
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ void k_set_int(int *p, int v) { *p = v; }

// ---- batched launches (see proj2d.hip): one grid over every active slice ----
template <typename T>
__global__ __launch_bounds__(kBlock) void kb_copy(BatchDev<T> bd, int src_sel, int dst_sel) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VM, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  copy_body<T>(resolve(d, src_sel, k), resolve(d, dst_sel, k), d.g.m, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_norm_to(BatchDev<T> bd, int sel, int fam, int which) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, fam, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  (void)which;
  norm_to_body<T>(resolve(d, sel, k), fam == BF_VM ? d.g.m : d.dimq, d.partials, b);
}

// finalising kernel of a batched reduction: one workgroup per active slice
// sums the slice's partials of family fam
template <typename T>
__global__ __launch_bounds__(kBlock) void kb_norm_finalize(BatchDev<T> bd, int fam, int which) {
  const int a = blockIdx.x;
  const SliceDev<T> &d = bd.sd[bd.active[a]];
  if (skip(bd, d)) return;
  const int *pre = bd.pre + fam * (bd.na + 1);
  norm_finalize_body(d.ctl, d.partials, (unsigned)(pre[a + 1] - pre[a]), which);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_dots2(BatchDev<T> bd) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VQD, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  dots2_body<T>(d.ctl, d.Q, d.ldq, d.w, d.dimq, d.partials, b.id, blockIdx.y, d.reorth ? k : 0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_reduce_cols2(BatchDev<T> bd) {
  const int a = blockIdx.y;
  const SliceDev<T> &d = bd.sd[bd.active[a]];
  if (skip(bd, d)) return;
  const int *pre = bd.pre + BF_VQD * (bd.na + 1);
  const int k = d.ctl.ip[CI_K];
  // the launch covers 2 (kmax + 1) columns; this slice's two sets start at 0
  // and K + 1 of its own
  const int kmax1 = gridDim.x / 2;
  const int set = blockIdx.x >= (unsigned)kmax1 ? 1 : 0, j = blockIdx.x - set * kmax1;
  if (j > d.ctl.K) return;
  reduce_cols2_body(d.ctl, d.partials, pre[a + 1] - pre[a], set * (d.ctl.K + 1) + j, d.reorth ? k : 0);
}

template <typename T>
__global__ __launch_bounds__(kCoefThreads) void kb_dcgs_coef(BatchDev<T> bd) {
  const SliceDev<T> &d = bd.sd[bd.active[blockIdx.x]];
  if (skip(bd, d) || !d.reorth) return;
  dcgs_coef_body(d.ctl, d.ctl.ip[CI_K]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_resid(BatchDev<T> bd) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VM, blockIdx.x, b);
  if (skip(bd, d)) return;
  resid_body<T>(d.ctl, d.yk, d.g.m, d.partials, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_resid_init(BatchDev<T> bd) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VM, blockIdx.x, b);
  if (skip(bd, d)) return;
  resid_init_body<T>(d.ctl, d.b, d.g.m, d.partials, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_cgs_update(BatchDev<T> bd, int last) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VQU, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  cgs_update_body<T>(d.ctl, d.Q, d.ldq, d.w, d.dimq, last, d.partials, b, d.reorth ? k : 0);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_normalize(BatchDev<T> bd) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VQ, blockIdx.x, b);
  if (skip(bd, d)) return;
  normalize_body<T>(d.ctl, d.w, d.Q, d.ldq, d.dimq, b.id, PadOut<T>{}, d.ctl.alpha[d.ctl.ip[CI_K] + 1]);
}

template <typename T>
__global__ __launch_bounds__(kSolveThreads) void kb_small_solve(BatchDev<T> bd) {
  const SliceDev<T> &d = bd.sd[bd.active[blockIdx.x]];
  if (skip(bd, d)) return;
  small_solve_body(d.ctl);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void kb_solution(BatchDev<T> bd, int out_sel) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_VQ, blockIdx.x, b);
  solution_body<T>(d.ctl, d.Q, d.ldq, d.dimq, resolve(d, out_sel, 0), b);
}

// Per-slice scalars for the host, 4 per slice.  phase 0: t_1, alpha_1,
// ||b||; phase 1: k_stop, reason, rho[k_stop], pres[k_stop].
template <typename T>
__global__ void kb_report(const SliceDev<T> *sd, int ns, int phase, double *out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const Ctl &c = sd[s].ctl;
  if (phase == 0) {
    out[4 * s] = c.t[1];
    out[4 * s + 1] = c.alpha[1];
    out[4 * s + 2] = c.dp[CD_BNORM];
    out[4 * s + 3] = 0.0;
  } else {
    const int ks = c.ip[CI_KSTOP];
    out[4 * s] = ks;
    out[4 * s + 1] = c.ip[CI_REASON];
    out[4 * s + 2] = ks > 0 ? c.rho[ks] : 0.0;
    out[4 * s + 3] = ks > 0 ? c.pres[ks] : 0.0;
  }
}

template <typename T>
__global__ void kb_set_k(BatchDev<T> bd, int k) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= bd.na) return;
  const SliceDev<T> &d = bd.sd[bd.active[a]];
  if (!d.ctl.ip[CI_STOP]) d.ctl.ip[CI_K] = k;
}

}  // namespace

void launch_set_int(int *p, int v, hipStream_t s) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v); }

int vec_blocks(long long dim) {
  long long b = (dim + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
  return (int)std::max<long long>(b, 1);
}
int dots_blocks(long long dim) {
  const long long rows = (long long)kBlock * RPT * kDotsQuads;
  return (int)std::max<long long>((dim + rows - 1) / rows, 1);
}
int upd_blocks(long long dim) {
  const long long rows = 64LL * RPT * (kBlock / 64 / upd_split(dim));
  return (int)std::max<long long>((dim + rows - 1) / rows, 1);
}

template <typename T>
void launch_copy(const T *src, T *dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(vec_blocks(n)), dim3(kBlock), 0, s, src, dst, n);
}
void launch_norm_finalize(Ctl ctl, const double *partials, int nb, int which, const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_finalize, dim3(1), dim3(kBlock), 0, s, ctl, partials, nb, which, stop);
}
template <typename T>
void launch_norm_to(Ctl ctl, const T *v, long long dim, int which, double *partials, hipStream_t s) {
  const int nb = vec_blocks(dim);
  hipLaunchKernelGGL(k_norm_to<T>, dim3(nb), dim3(kBlock), 0, s, ctl, v, dim, partials);
  launch_norm_finalize(ctl, partials, nb, which, ctl.ip + CI_STOP, s);
}
template <typename T>
void launch_dcgs_dots(Ctl ctl, const T *Q, long long ld, const T *w, long long dim, double *partials,
                      hipStream_t s, bool nt) {
  const int nb = dots_blocks(dim);
  const dim3 grid(nb, (ctl.K + CH2) / CH2);
  hipLaunchKernelGGL(k_dots2<T>, grid, dim3(kBlock), 0, s, ctl, Q, ld, w, dim, partials, (int)nt);
  hipLaunchKernelGGL(k_reduce_cols2, dim3(2 * (ctl.K + 1)), dim3(kBlock), 0, s, ctl, (const double *)partials, nb);
}
void launch_dcgs_coef(Ctl ctl, hipStream_t s) { hipLaunchKernelGGL(k_dcgs_coef, dim3(1), dim3(kCoefThreads), 0, s, ctl); }
template <typename T>
void launch_cgs_update(Ctl ctl, const T *Q, long long ld, T *w, long long dim, int last, double *partials,
                       hipStream_t s, int reorth) {
  const int nb = upd_blocks(dim);
  hipLaunchKernelGGL(k_cgs_update<T>, dim3(nb), dim3(kBlock), 0, s, ctl, Q, ld, w, dim, last, partials, reorth, 0);
  if (last) launch_norm_finalize(ctl, partials, nb, NORM_ALPHA1, ctl.ip + CI_STOP, s);
}
template <typename T>
void launch_normalize(Ctl ctl, const T *w, T *Q, long long ld, long long dim, hipStream_t s, PadOut<T> pout) {
  hipLaunchKernelGGL(k_normalize<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, w, Q, ld, dim, pout);
}
template <typename T>
void launch_update_normalize(Ctl ctl, T *Q, long long ld, T *w, long long dim, double *partials, hipStream_t s,
                             int reorth, PadOut<T> pout, bool nt) {
  const int nb = upd_blocks(dim);
  hipLaunchKernelGGL(k_cgs_update<T>, dim3(nb), dim3(kBlock), 0, s, ctl, Q, ld, w, dim, 1, partials, reorth,
                     (int)nt);
  hipLaunchKernelGGL(k_normalize_fin<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, w, Q, ld, dim, pout,
                     (const double *)partials, nb);
}
template <typename T>
void launch_resid_init(Ctl ctl, const T *b, long long m, double *partials, hipStream_t s) {
  const int nb = vec_blocks(m);
  hipLaunchKernelGGL(k_resid_init<T>, dim3(nb), dim3(kBlock), 0, s, ctl, b, m, partials);
  launch_norm_finalize(ctl, partials, nb, NORM_BNORM, nullptr, s);
}
template <typename T>
void launch_resid(Ctl ctl, const T *yk, long long m, double *partials, hipStream_t s) {
  const int nb = vec_blocks(m);
  hipLaunchKernelGGL(k_resid<T>, dim3(nb), dim3(kBlock), 0, s, ctl, yk, m, partials);
  launch_norm_finalize(ctl, partials, nb, NORM_RHO, ctl.ip + CI_STOP, s);
}
template <typename T>
void launch_rre(Ctl ctl, const T *x, const T *x_true, long long n, double *partials, hipStream_t s) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_diff_norm<T>, dim3(nb), dim3(kBlock), 0, s, x, x_true, n, partials);
  launch_norm_finalize(ctl, partials, nb, NORM_RRE, nullptr, s);
}
void launch_small_solve(Ctl ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(kSolveThreads), 0, s, ctl);
}
void launch_gm_hcol(Ctl ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_hcol, dim3(1), dim3(kBlock), 0, s, ctl);
}
void launch_gm_solve(Ctl ctl, hipStream_t s) { hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(64), 0, s, ctl); }
template <typename T>
void launch_gm_resid(Ctl ctl, const T *Y, long long ld, const T *b, long long m, double *partials, hipStream_t s,
                     int which, bool nt) {
  const int nb = vec_blocks(m);
  hipLaunchKernelGGL(k_gm_resid<T>, dim3(nb), dim3(kBlock), 0, s, ctl, Y, ld, b, m, partials, (int)nt);
  launch_norm_finalize(ctl, partials, nb, which, ctl.ip + CI_STOP, s);
}
void launch_hy_lambda(Ctl ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_hy_lambda, dim3(1), dim3(kSolveThreads), 0, s, ctl);
}
void launch_hy_solve(Ctl ctl, hipStream_t s) { hipLaunchKernelGGL(k_hy_solve, dim3(1), dim3(kSolveThreads), 0, s, ctl); }
void launch_tsvd(Ctl ctl, double *W, double *V, int rank, hipStream_t s) {
  hipLaunchKernelGGL(k_tsvd, dim3(1), dim3(kTsvdThreads), 0, s, ctl, W, V, rank);
}
template <typename T>
void launch_final_residual(Ctl ctl, const T *ax, const T *b, long long m, double *partials, hipStream_t s) {
  const int nb = vec_blocks(m);
  hipLaunchKernelGGL(k_diff_norm<T>, dim3(nb), dim3(kBlock), 0, s, ax, b, m, partials);
  launch_norm_finalize(ctl, partials, nb, NORM_FINAL, nullptr, s);
}
template <typename T>
void launch_solution(Ctl ctl, const T *Q, long long ld, long long dim, T *out, hipStream_t s) {
  hipLaunchKernelGGL(k_solution<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, Q, ld, dim, out);
}

// ---- batched launchers ----
template <typename T>
void launch_b_copy(const BatchDev<T> &bd, const BatchLaunch &bl, int src_sel, int dst_sel, hipStream_t s) {
  if (bl.tot[BF_VM] > 0) hipLaunchKernelGGL(kb_copy<T>, dim3(bl.tot[BF_VM]), dim3(kBlock), 0, s, bd, src_sel, dst_sel);
}
template <typename T>
void launch_b_norm_finalize(const BatchDev<T> &bd, const BatchLaunch &bl, int fam, int which, hipStream_t s) {
  if (bl.na > 0) hipLaunchKernelGGL(kb_norm_finalize<T>, dim3(bl.na), dim3(kBlock), 0, s, bd, fam, which);
}
template <typename T>
void launch_b_norm_to(const BatchDev<T> &bd, const BatchLaunch &bl, int sel, int fam, int which, hipStream_t s) {
  if (bl.tot[fam] <= 0) return;
  hipLaunchKernelGGL(kb_norm_to<T>, dim3(bl.tot[fam]), dim3(kBlock), 0, s, bd, sel, fam, which);
  launch_b_norm_finalize(bd, bl, fam, which, s);
}
template <typename T>
void launch_b_dcgs(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s) {
  if (bl.tot[BF_VQ] <= 0) return;
  hipLaunchKernelGGL(kb_dots2<T>, dim3(bl.tot[BF_VQD], (bl.kmax + CH2) / CH2), dim3(kBlock), 0, s, bd);
  hipLaunchKernelGGL(kb_reduce_cols2<T>, dim3(2 * (bl.kmax + 1), bl.na), dim3(kBlock), 0, s, bd);
  hipLaunchKernelGGL(kb_dcgs_coef<T>, dim3(bl.na), dim3(kCoefThreads), 0, s, bd);
}
template <typename T>
void launch_b_cgs_update(const BatchDev<T> &bd, const BatchLaunch &bl, int last, hipStream_t s) {
  if (bl.tot[BF_VQU] <= 0) return;
  hipLaunchKernelGGL(kb_cgs_update<T>, dim3(bl.tot[BF_VQU]), dim3(kBlock), 0, s, bd, last);
  if (last) launch_b_norm_finalize(bd, bl, BF_VQU, NORM_ALPHA1, s);
}
template <typename T>
void launch_b_normalize(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s) {
  if (bl.tot[BF_VQ] > 0) hipLaunchKernelGGL(kb_normalize<T>, dim3(bl.tot[BF_VQ]), dim3(kBlock), 0, s, bd);
}
template <typename T>
void launch_b_resid(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s) {
  if (bl.tot[BF_VM] <= 0) return;
  hipLaunchKernelGGL(kb_resid<T>, dim3(bl.tot[BF_VM]), dim3(kBlock), 0, s, bd);
  launch_b_norm_finalize(bd, bl, BF_VM, NORM_RHO, s);
}
template <typename T>
void launch_b_resid_init(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s) {
  if (bl.tot[BF_VM] <= 0) return;
  hipLaunchKernelGGL(kb_resid_init<T>, dim3(bl.tot[BF_VM]), dim3(kBlock), 0, s, bd);
  launch_b_norm_finalize(bd, bl, BF_VM, NORM_BNORM, s);
}
template <typename T>
void launch_b_small_solve(const BatchDev<T> &bd, const BatchLaunch &bl, hipStream_t s) {
  if (bl.na > 0) hipLaunchKernelGGL(kb_small_solve<T>, dim3(bl.na), dim3(kSolveThreads), 0, s, bd);
}
template <typename T>
void launch_b_solution(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, hipStream_t s) {
  if (bl.tot[BF_VQ] > 0) hipLaunchKernelGGL(kb_solution<T>, dim3(bl.tot[BF_VQ]), dim3(kBlock), 0, s, bd, out_sel);
}
template <typename T>
void launch_b_set_k(const BatchDev<T> &bd, const BatchLaunch &bl, int k, hipStream_t s) {
  if (bl.na > 0) hipLaunchKernelGGL(kb_set_k<T>, dim3((bl.na + 255) / 256), dim3(256), 0, s, bd, k);
}
template <typename T>
void launch_b_report(const SliceDev<T> *sd, int ns, int phase, double *out, hipStream_t s) {
  if (ns > 0) hipLaunchKernelGGL(kb_report<T>, dim3((ns + 255) / 256), dim3(256), 0, s, sd, ns, phase, out);
}

#define GKB_INST(T)                                                                                         \
  template void launch_copy<T>(const T *, T *, long long, hipStream_t);                                    \
  template void launch_norm_to<T>(Ctl, const T *, long long, int, double *, hipStream_t);                  \
  template void launch_cgs_update<T>(Ctl, const T *, long long, T *, long long, int, double *, hipStream_t, \
                                     int);                                                                  \
  template void launch_normalize<T>(Ctl, const T *, T *, long long, long long, hipStream_t, PadOut<T>);               \
  template void launch_update_normalize<T>(Ctl, T *, long long, T *, long long, double *, hipStream_t, int, PadOut<T>, \
                                           bool);                                                                  \
  template void launch_resid<T>(Ctl, const T *, long long, double *, hipStream_t);                         \
  template void launch_rre<T>(Ctl, const T *, const T *, long long, double *, hipStream_t);                \
  template void launch_resid_init<T>(Ctl, const T *, long long, double *, hipStream_t);                    \
  template void launch_solution<T>(Ctl, const T *, long long, long long, T *, hipStream_t);                  \
  template void launch_gm_resid<T>(Ctl, const T *, long long, const T *, long long, double *, hipStream_t, int,  \
                                    bool);                                                                        \
  template void launch_final_residual<T>(Ctl, const T *, const T *, long long, double *, hipStream_t);       \
  template void launch_b_copy<T>(const BatchDev<T> &, const BatchLaunch &, int, int, hipStream_t);          \
  template void launch_b_norm_to<T>(const BatchDev<T> &, const BatchLaunch &, int, int, int, hipStream_t);  \
  template void launch_b_norm_finalize<T>(const BatchDev<T> &, const BatchLaunch &, int, int, hipStream_t); \
  template void launch_b_dcgs<T>(const BatchDev<T> &, const BatchLaunch &, hipStream_t);                    \
  template void launch_dcgs_dots<T>(Ctl, const T *, long long, const T *, long long, double *, hipStream_t, bool); \
  template void launch_b_cgs_update<T>(const BatchDev<T> &, const BatchLaunch &, int, hipStream_t);         \
  template void launch_b_normalize<T>(const BatchDev<T> &, const BatchLaunch &, hipStream_t);               \
  template void launch_b_resid<T>(const BatchDev<T> &, const BatchLaunch &, hipStream_t);                   \
  template void launch_b_resid_init<T>(const BatchDev<T> &, const BatchLaunch &, hipStream_t);              \
  template void launch_b_small_solve<T>(const BatchDev<T> &, const BatchLaunch &, hipStream_t);             \
  template void launch_b_solution<T>(const BatchDev<T> &, const BatchLaunch &, int, hipStream_t);           \
  template void launch_b_set_k<T>(const BatchDev<T> &, const BatchLaunch &, int, hipStream_t);              \
  template void launch_b_report<T>(const SliceDev<T> *, int, int, double *, hipStream_t);
GKB_INST(float)
GKB_INST(double)
#undef GKB_INST

}  // namespace gkb
