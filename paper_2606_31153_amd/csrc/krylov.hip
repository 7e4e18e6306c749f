// Krylov vector kernels for the AB-/BA-GKB iteration on gfx950.
//
// Precision split: vectors (Q, Y, s, w) are stored in T (float or double);
// every inner product, norm and reorthogonalisation update is formed and
// accumulated in double; alpha, t, the projected solve and the discrepancy
// test are double.  All reductions are deterministic (fixed-order wave
// butterflies, fixed-order sum over workgroups by the last workgroup to
// arrive).
//
// Reorthogonalisation (one-sided, on q only; Alg. "GKB" step 9 and its
// AB/BA counterparts) is classical Gram-Schmidt applied twice:
//   c1 = Q^T w;  w -= Q c1;  c2 = Q^T w;  w -= Q c2;  alpha = ||w||.
// The discrepancy residual ||A x_k - b|| is obtained from the Gram matrix of
// the stored A-images Y_i (BA, GKB: A q_i; AB: A B q_i) and b:
//   ||Y u - b||^2 = u^T (Y^T Y) u - 2 u^T (Y^T b) + ||b||^2,
// which equals ||A x_k - b||^2 because A x_k = sum_i u_i Y_i.
// The projected problem min ||C_k u - t_1 e_1||^2 + lambda^2 ||u||^2
// (eq. proj GKB) is solved by Givens rotations updated once per iteration
// (the factorisation Paige and Saunders use for LSQR, with the damping rows
// for lambda); this gives the same minimiser as the SVD route of the paper
// in O(k) work per iteration.

#include "internal.h"
#include "reduce.h"

namespace gkb {

namespace {

constexpr int CH = 8;  // columns per pass of the multi-dot loops

int g_max_vec_blocks = 512;

// Sum CH values over the block; results valid in threads 0..CH-1 (value j in thread j).
__device__ inline double block_sum_vec(double (&v)[CH], double *lds /* [4][CH] */) {
#pragma unroll
  for (int j = 0; j < CH; ++j) v[j] = wave_sum(v[j]);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < CH; ++j) lds[wid * CH + j] = v[j];
  }
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x < CH) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) r += lds[w * CH + threadIdx.x];
  }
  return r;
}

// Partial inner products of w with columns [0, ncol) of V over this block's
// rows, written to partials[blockIdx.x * ldp + c].
template <typename T>
__device__ inline void block_dots(const T *__restrict__ V, long long ld, int ncol, const T *__restrict__ w,
                                  long long dim, double *partials, int ldp, double *lds) {
  const long long stride = (long long)gridDim.x * kBlock;
  for (int c0 = 0; c0 < ncol; c0 += CH) {
    double acc[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) acc[j] = 0.0;
    for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride) {
      const double wv = (double)w[r];
#pragma unroll
      for (int j = 0; j < CH; ++j)
        if (c0 + j < ncol) acc[j] = fma((double)V[(long long)(c0 + j) * ld + r], wv, acc[j]);
    }
    const double s = block_sum_vec(acc, lds);
    if (threadIdx.x < CH && c0 + (int)threadIdx.x < ncol) partials[(long long)blockIdx.x * ldp + c0 + threadIdx.x] = s;
  }
}

// Last block: out[c] = sum over blocks of partials[b*ldp + c], fixed order.
__device__ inline void finish_dots(int ncol, const double *partials, int ldp, double *out, long long out_stride,
                                   double *out2, long long out2_stride) {
  const unsigned nb = gridDim.x;
  for (int c = threadIdx.x; c < ncol; c += kBlock) {
    double acc = 0.0;
    for (unsigned b = 0; b < nb; ++b) acc += partials[(long long)b * ldp + c];
    out[(long long)c * out_stride] = acc;
    if (out2) out2[(long long)c * out2_stride] = acc;
  }
}

// ---- c = Q[:, 0..k-1]^T w -------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_dots(Ctl ctl, const T *__restrict__ Q, long long ld,
                                                     const T *__restrict__ w, long long dim, double *partials,
                                                     unsigned *counter) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[(kBlock / 64) * CH];
  const int k = ctl.ip[CI_K];
  const int ldp = ctl.K + 2;
  block_dots(Q, ld, k, w, dim, partials, ldp, lds);
  if (arrive_last(counter, gridDim.x)) {
    finish_dots(k, partials, ldp, ctl.c, 1, nullptr, 0);
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// ---- w -= Q c; then (last == 0) c = Q^T w, or (last == 1) alpha[k+1] = ||w|| ----
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_update(Ctl ctl, const T *__restrict__ Q, long long ld,
                                                       T *__restrict__ w, long long dim, int last,
                                                       double *partials, unsigned *counter) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[(kBlock / 64) * CH];
  const int k = ctl.ip[CI_K];
  const int ldp = ctl.K + 2;
  const long long stride = (long long)gridDim.x * kBlock;
  const double *__restrict__ cc = ctl.c;
  double nrm = 0.0;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride) {
    double acc = (double)w[r];
    for (int c = 0; c < k; ++c) acc = fma(-cc[c], (double)Q[(long long)c * ld + r], acc);
    const T v = (T)acc;
    w[r] = v;
    nrm = fma((double)v, (double)v, nrm);
  }
  if (!last) {
    block_dots(Q, ld, k, (const T *)w, dim, partials, ldp, lds);
    if (arrive_last(counter, gridDim.x)) {
      finish_dots(k, partials, ldp, ctl.c, 1, nullptr, 0);
      if (threadIdx.x == 0) *counter = 0u;
    }
  } else {
    const double s = block_sum<kBlock>(nrm, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
    if (arrive_last(counter, gridDim.x)) {
      double acc = 0.0;
      for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock) acc += partials[b];
      const double tot = block_sum<kBlock>(acc, lds);
      if (threadIdx.x == 0) {
        ctl.alpha[k + 1] = sqrt(tot);
        *counter = 0u;
      }
    }
  }
}

// ---- Q[:, k] = w / alpha[k+1] ------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_normalize(Ctl ctl, const T *__restrict__ w, T *__restrict__ Q,
                                                      long long ld, long long dim) {
  if (ctl.ip[CI_STOP]) return;
  const int k = ctl.ip[CI_K];
  const double inv = 1.0 / ctl.alpha[k + 1];
  T *q = Q + (long long)k * ld;
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride)
    q[r] = (T)((double)w[r] * inv);
}

// ---- Gram row k: G[k][c] = G[c][k] = Y_k . Y_c, c = 0..k (Y_0 = b) ------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram(Ctl ctl, const T *__restrict__ Y, long long ld, long long dim,
                                                 double *partials, unsigned *counter) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[(kBlock / 64) * CH];
  const int k = ctl.ip[CI_K];
  const int ldp = ctl.K + 2;
  block_dots(Y, ld, k + 1, Y + (long long)k * ld, dim, partials, ldp, lds);
  if (arrive_last(counter, gridDim.x)) {
    finish_dots(k + 1, partials, ldp, ctl.G + (long long)k * ctl.ldG, 1, ctl.G + k, ctl.ldG);
    if (threadIdx.x == 0) *counter = 0u;
  }
}

// ---- projected solve, discrepancy test, advance --------------------------------
// One wavefront.  Iteration k has alpha[1..k], t[1..k+1] (and alpha[k+1]
// unless k == K).  Givens rotations G = [[c, s], [-s, c]] reduce
// [C_k; lambda I] to upper bidiagonal R (diagonal Rd, superdiagonal Rth) with
// right-hand side Rphi; u_k solves R u = Rphi.
__global__ __launch_bounds__(64) void k_small_solve(Ctl ctl) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double s_u[1];
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
    const double phibar_next = -s * phibar;
    dp[CD_CPREV] = c;
    dp[CD_SPREV] = s;
    dp[CD_PHIBAR] = phibar_next;
    // back substitution
    double un = ctl.Rphi[k] / ctl.Rd[k];
    ctl.u[k] = un;
    for (int i = k - 1; i >= 1; --i) {
      un = (ctl.Rphi[i] - ctl.Rth[i + 1] * un) / ctl.Rd[i];
      ctl.u[i] = un;
    }
    // projected residual ||C_k u - t_1 e_1|| (without the Tikhonov rows):
    // row i of C_k u is alpha_i u_i + t_i u_{i-1}
    double pr = 0.0;
    for (int i = 1; i <= k + 1; ++i) {
      double r = (i <= k ? ctl.alpha[i] * ctl.u[i] : 0.0) + (i >= 2 ? ctl.t[i] * ctl.u[i - 1] : 0.0);
      if (i == 1) r -= ctl.t[1];
      pr = fma(r, r, pr);
    }
    dp[CD_PRES] = sqrt(pr);
    ctl.pres[k] = dp[CD_PRES];
  }
  __syncthreads();
  // ||Y u - b||^2 = sum_ij u_i u_j G_ij - 2 sum_i u_i G_i0 + G_00  (i, j = 1..k)
  double part = 0.0;
  for (int i = 1 + threadIdx.x; i <= k; i += 64) {
    const double *Gi = ctl.G + (long long)i * ctl.ldG;
    double acc = -2.0 * Gi[0];
    for (int j = 1; j <= k; ++j) acc = fma(Gi[j], ctl.u[j], acc);
    part = fma(ctl.u[i], acc, part);
  }
  part = wave_sum(part);
  if (threadIdx.x == 0) {
    const double rho2 = part + ctl.G[0];
    const double rho = sqrt(fmax(rho2, 0.0));
    ctl.rho[k] = rho;
    // breakdown scale: max_i sqrt(alpha_i^2 + t_{i+1}^2)
    const double ak = ctl.alpha[k], tk1 = ctl.t[k + 1];
    const double sc = fmax(dp[CD_BSCALE], sqrt(ak * ak + tk1 * tk1));
    dp[CD_BSCALE] = sc;
    const double eta = dp[CD_ETAEPS] * sc;
    int reason = 0;
    if (dp[CD_USEDP] != 0.0 && rho <= dp[CD_TAUE])
      reason = 1;  // GKB_STOP_DP
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
  (void)s_u;
}

// ---- out = sum_{i=1..k_stop} u_i Q[:, i-1] -------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_solution(Ctl ctl, const T *__restrict__ Q, long long ld,
                                                     long long dim, T *__restrict__ out) {
  const int ks = ctl.ip[CI_KSTOP];
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride) {
    double acc = 0.0;
    for (int i = 1; i <= ks; ++i) acc = fma(ctl.u[i], (double)Q[(long long)(i - 1) * ld + r], acc);
    out[r] = (T)acc;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T *__restrict__ a, T *__restrict__ b, long long n) {
  const long long stride = (long long)gridDim.x * kBlock;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < n; r += stride) b[r] = a[r];
}

// ||v|| into t[k+1] (which == NORM_T1) or alpha[k+1] (NORM_ALPHA1)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_norm_to(Ctl ctl, const T *__restrict__ v, long long dim, int which,
                                                    double *partials, unsigned *counter) {
  if (ctl.ip[CI_STOP]) return;
  __shared__ double lds[kBlock / 64];
  const long long stride = (long long)gridDim.x * kBlock;
  double acc = 0.0;
  for (long long r = (long long)blockIdx.x * kBlock + threadIdx.x; r < dim; r += stride) {
    const double x = (double)v[r];
    acc = fma(x, x, acc);
  }
  const double s = block_sum<kBlock>(acc, lds);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
  if (arrive_last(counter, gridDim.x)) {
    double a = 0.0;
    for (unsigned b = threadIdx.x; b < gridDim.x; b += kBlock) a += partials[b];
    const double tot = block_sum<kBlock>(a, lds);
    if (threadIdx.x == 0) {
      const int k = ctl.ip[CI_K];
      if (which == NORM_T1)
        ctl.t[k + 1] = sqrt(tot);
      else
        ctl.alpha[k + 1] = sqrt(tot);
      *counter = 0u;
    }
  }
}

__global__ void k_set_int(int *p, int v) { *p = v; }

}  // namespace

void launch_set_int(int *p, int v, hipStream_t s) { hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v); }

int vec_blocks(long long dim) {
  long long b = (dim + kBlock - 1) / kBlock;
  if (b > g_max_vec_blocks) b = g_max_vec_blocks;
  if (b < 1) b = 1;
  return (int)b;
}

template <typename T>
void launch_copy(const T *src, T *dst, long long n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy<T>, dim3(vec_blocks(n)), dim3(kBlock), 0, s, src, dst, n);
}
template <typename T>
void launch_norm_to(Ctl ctl, const T *v, long long dim, int which, double *partials, unsigned *counter,
                    hipStream_t s) {
  hipLaunchKernelGGL(k_norm_to<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, v, dim, which, partials,
                     counter);
}
template <typename T>
void launch_cgs_dots(Ctl ctl, const T *Q, long long ld, const T *w, long long dim, double *partials,
                     unsigned *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_dots<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, Q, ld, w, dim, partials,
                     counter);
}
template <typename T>
void launch_cgs_update(Ctl ctl, const T *Q, long long ld, T *w, long long dim, int last, double *partials,
                       unsigned *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_update<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, Q, ld, w, dim, last,
                     partials, counter);
}
template <typename T>
void launch_normalize(Ctl ctl, const T *w, T *Q, long long ld, long long dim, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, w, Q, ld, dim);
}
template <typename T>
void launch_gram(Ctl ctl, const T *Y, long long ld, long long dim, int init, double *partials, unsigned *counter,
                 hipStream_t s) {
  (void)init;
  hipLaunchKernelGGL(k_gram<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, Y, ld, dim, partials, counter);
}
void launch_small_solve(Ctl ctl, hipStream_t s) {
  hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(64), 0, s, ctl);
}
template <typename T>
void launch_solution(Ctl ctl, const T *Q, long long ld, long long dim, T *out, hipStream_t s) {
  hipLaunchKernelGGL(k_solution<T>, dim3(vec_blocks(dim)), dim3(kBlock), 0, s, ctl, Q, ld, dim, out);
}

#define GKB_INST(T)                                                                                         \
  template void launch_copy<T>(const T *, T *, long long, hipStream_t);                                    \
  template void launch_norm_to<T>(Ctl, const T *, long long, int, double *, unsigned *, hipStream_t);      \
  template void launch_cgs_dots<T>(Ctl, const T *, long long, const T *, long long, double *, unsigned *,  \
                                   hipStream_t);                                                           \
  template void launch_cgs_update<T>(Ctl, const T *, long long, T *, long long, int, double *, unsigned *, \
                                     hipStream_t);                                                         \
  template void launch_normalize<T>(Ctl, const T *, T *, long long, long long, hipStream_t);               \
  template void launch_gram<T>(Ctl, const T *, long long, long long, int, double *, unsigned *, hipStream_t); \
  template void launch_solution<T>(Ctl, const T *, long long, long long, T *, hipStream_t);
GKB_INST(float)
GKB_INST(double)
#undef GKB_INST

}  // namespace gkb
