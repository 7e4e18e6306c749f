// Kernels of the learned sinogram filter (gfx950): a bias-free 1D
// convolutional network along the detector axis, 1 -> 32 -> 32 -> 32 -> 1
// channels, kernel 9, zero "same" padding, ReLU after the first three
// layers.  Inside BA-GKB it acts through its frozen-mask linearisation F
// (M = B F A, M^T = A^T F^T B^T; BA-GKB needs only B and B^T, Sec. 3.2).
//
// Activations are position-major, a[row][p][c] (32 floats per detector
// position), rows = views x detector rows, p = detector column.
//  * k_net_c1:  1 -> 32 channels on the vector ALUs (9 taps per output).
//  * k_net_c32: 32 -> 32 channels on the matrix cores: per tap t and half of
//    the input channels, one v_mfma_f32_32x32x16_bf16 multiplies the 32 x 16
//    weight block (output channel x input channel) by the 16 x 32 block of
//    activations (input channel x position), accumulating in FP32; 18 such
//    products per 32 x 32 output tile.  Activations are staged in LDS as
//    NSPLIT bfloat16 terms: 1 for training (bfloat16 operands), 3 for the
//    filter inside GKB (hi + mid + lo reproduces every FP32 activation
//    exactly, so F is applied at FP32 accuracy).
//  * k_net_c4:  32 -> 1 channel on the vector ALUs.
//  The transposed filter F^T and the backward pass run through the same
//  three kernels with flipped, channel-transposed weights.
//  * mask modes: none; compute (ReLU, and the 32 mask bits per position
//    written as one word); apply (zero the channels whose frozen bit is 0).
//  * k_net_wgrad32 (matrix cores) and k_net_wgrad_edge (vector ALUs):
//    weight gradients as per-workgroup partial sums over positions, reduced
//    in a fixed order in FP64 by k_net_reduce; k_net_adam, k_net_prep.

#include <algorithm>
#include <cmath>

#include "internal.h"
#include "reduce.h"

namespace gkb {

namespace {

constexpr int NC = 32, NK = 9, NH = 4;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// 1 -> 32 channels: z[c] = sum_t w[c][t] s[p + t - 4]
// ---------------------------------------------------------------------------
constexpr int TP1 = 256;

template <int MODE>
__global__ __launch_bounds__(256) void k_net_c1(Col<const float> sc, float *__restrict__ out,
                                                unsigned *__restrict__ mask, const float *__restrict__ w, int L,
                                                int segs, long long rows, const int *stop) {
  if (stop && *stop) return;
  const float *__restrict__ s = sc.get();
  __shared__ float sw[NC * NK];
  __shared__ float ss[TP1 + 2 * NH];
  const long long blk = blockIdx.x;
  const long long row = blk / segs;
  const int p0 = (int)(blk - row * segs) * TP1;
  for (int i = threadIdx.x; i < NC * NK; i += 256) sw[i] = w[i];
  for (int i = threadIdx.x; i < TP1 + 2 * NH; i += 256) {
    const int p = p0 - NH + i;
    ss[i] = (p >= 0 && p < L) ? s[row * L + p] : 0.f;
  }
  __syncthreads();
  const int p = p0 + threadIdx.x;
  if (p >= L) return;
  float z[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < NK; ++t) acc = fmaf(sw[c * NK + t], ss[threadIdx.x + t], acc);
    z[c] = acc;
  }
  const long long pos = row * L + p;
  if (MODE == 1) {
    unsigned bits = 0u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bits |= (z[c] > 0.f ? 1u : 0u) << c;
      z[c] = fmaxf(z[c], 0.f);
    }
    mask[pos] = bits;
  } else if (MODE == 2) {
    const unsigned bits = mask[pos];
#pragma unroll
    for (int c = 0; c < NC; ++c) z[c] = ((bits >> c) & 1u) ? z[c] : 0.f;
  }
  float4 *o = reinterpret_cast<float4 *>(out + pos * NC);
#pragma unroll
  for (int q = 0; q < NC / 4; ++q) o[q] = make_float4(z[4 * q], z[4 * q + 1], z[4 * q + 2], z[4 * q + 3]);
}

// ---------------------------------------------------------------------------
// 32 -> 1 channel: out[p] = sum_t sum_c w[c][t] a[p + t - 4][c]
// ---------------------------------------------------------------------------
constexpr int TP4 = 256;

__global__ __launch_bounds__(256) void k_net_c4(const float *__restrict__ a, float *__restrict__ out,
                                                const float *__restrict__ w, int L, int segs, long long rows,
                                                const int *stop) {
  if (stop && *stop) return;
  __shared__ float sw[NC * NK];
  __shared__ float sa[(TP4 + 2 * NH) * (NC + 1)];
  const long long blk = blockIdx.x;
  const long long row = blk / segs;
  const int p0 = (int)(blk - row * segs) * TP4;
  for (int i = threadIdx.x; i < NC * NK; i += 256) sw[i] = w[i];
  const float *__restrict__ arow = a + row * L * NC;
  for (int i = threadIdx.x; i < (TP4 + 2 * NH) * (NC / 4); i += 256) {
    const int pw = i / (NC / 4), c4 = (i % (NC / 4)) * 4;
    const int p = p0 - NH + pw;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p >= 0 && p < L) v = *reinterpret_cast<const float4 *>(arow + (long long)p * NC + c4);
    float *d = sa + pw * (NC + 1) + c4;
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
  __syncthreads();
  const int p = p0 + threadIdx.x;
  if (p >= L) return;
  float acc = 0.f;
#pragma unroll 1
  for (int t = 0; t < NK; ++t) {
    const float *r = sa + (threadIdx.x + t) * (NC + 1);
#pragma unroll
    for (int c = 0; c < NC; ++c) acc = fmaf(sw[c * NK + t], r[c], acc);
  }
  out[row * L + p] = acc;
}

// ---------------------------------------------------------------------------
// 32 -> 32 channels on the matrix cores
// ---------------------------------------------------------------------------
constexpr int TPC = 128;            // output positions per workgroup (4 waves x 32)
constexpr int WINC = TPC + 2 * NH;  // staged input positions
constexpr int LDC = 40;             // LDS row stride in bfloat16 (80 bytes)

template <int NSPLIT>
__device__ inline void split_store(__bf16 *dst, int stride_split, float4 v) {
  float r[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int sp = 0; sp < NSPLIT; ++sp) {
    bf16x4 h;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      h[q] = (__bf16)r[q];
      r[q] = r[q] - (float)h[q];
    }
    *reinterpret_cast<bf16x4 *>(dst + sp * stride_split) = h;
  }
}

template <int NSPLIT, int MODE>
__global__ __launch_bounds__(256) void k_net_c32(const float *__restrict__ a, float *__restrict__ out,
                                                 unsigned *__restrict__ mask, const __bf16 *__restrict__ wb, int L,
                                                 int segs, long long rows, const int *stop) {
  if (stop && *stop) return;
  __shared__ __bf16 sa[NSPLIT * WINC * LDC];
  const long long blk = blockIdx.x;
  const long long row = blk / segs;
  const int p0 = (int)(blk - row * segs) * TPC;
  const float *__restrict__ arow = a + row * L * NC;
  for (int i = threadIdx.x; i < WINC * (NC / 4); i += 256) {
    const int pw = i / (NC / 4), c4 = (i % (NC / 4)) * 4;
    const int p = p0 - NH + pw;
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (p >= 0 && p < L) v = *reinterpret_cast<const float4 *>(arow + (long long)p * NC + c4);
    split_store<NSPLIT>(sa + pw * LDC + c4, WINC * LDC, v);
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int hi = lane >> 5, col = lane & 31;
  // weight fragments: output channel col, taps t, input channels 16h + 8hi .. +7
  bf16x8 wf[2 * NK];
#pragma unroll
  for (int s = 0; s < 2 * NK; ++s) {
    const int t = s >> 1, h = s & 1;
    wf[s] = *reinterpret_cast<const bf16x8 *>(wb + (col * NK + t) * NC + 16 * h + 8 * hi);
  }
  __syncthreads();
  f32x16 acc = {};
  const int pw = wave * 32 + col;
#pragma unroll
  for (int s = 0; s < 2 * NK; ++s) {
    const int t = s >> 1, h = s & 1;
    const __bf16 *src = sa + (pw + t) * LDC + 16 * h + 8 * hi;
#pragma unroll
    for (int sp = 0; sp < NSPLIT; ++sp) {
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(src + sp * WINC * LDC);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[s], bv, acc, 0, 0, 0);
    }
  }
  // lane holds output channels 8 (r/4) + 4 hi + r%4 of position p
  const int p = p0 + pw;
  const bool valid = p < L;
  const long long pos = row * L + p;
  if (MODE == 1) {
    unsigned bits = 0u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = 8 * (r >> 2) + 4 * hi + (r & 3);
      bits |= (acc[r] > 0.f ? 1u : 0u) << c;
      acc[r] = fmaxf(acc[r], 0.f);
    }
    bits |= __shfl_xor(bits, 32, 64);
    if (valid && hi == 0) mask[pos] = bits;
  } else if (MODE == 2) {
    const unsigned bits = valid ? mask[pos] : 0u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int c = 8 * (r >> 2) + 4 * hi + (r & 3);
      acc[r] = ((bits >> c) & 1u) ? acc[r] : 0.f;
    }
  }
  if (valid) {
    float *o = out + pos * NC + 4 * hi;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<float4 *>(o + 8 * q) = make_float4(acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]);
  }
}

// ---------------------------------------------------------------------------
// weight gradient of a 32 -> 32 layer on the matrix cores:
// dW[co][ci][t] = sum_{row, p} g[p][co] a[p + t - 4][ci] (bfloat16 operands)
// Workgroups loop over (row, segment) items; wave w accumulates the taps
// t = w, w + 4, w + 8 as 32 x 32 (co x ci) tiles.
// ---------------------------------------------------------------------------
constexpr int TPW = 128;
constexpr int LDG = TPW + 8;  // [co][p] stride (272 bytes)

__global__ __launch_bounds__(256) void k_net_wgrad32(const float *__restrict__ g, const float *__restrict__ a,
                                                     float *__restrict__ partials, int L, int segs, long long rows) {
  __shared__ __bf16 gT[NC * LDG];
  __shared__ __bf16 aP[(TPW + 2 * NH) * LDC];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int hi = lane >> 5, col = lane & 31;
  f32x16 acc[3] = {};
  const long long items = rows * segs;
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const long long row = it / segs;
    const int p0 = (int)(it - row * segs) * TPW;
    __syncthreads();
    for (int i = threadIdx.x; i < TPW * (NC / 4); i += 256) {
      const int pw = i / (NC / 4), c4 = (i % (NC / 4)) * 4;
      const int p = p0 + pw;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < L) v = *reinterpret_cast<const float4 *>(g + (row * L + p) * NC + c4);
      gT[(c4 + 0) * LDG + pw] = (__bf16)v.x;
      gT[(c4 + 1) * LDG + pw] = (__bf16)v.y;
      gT[(c4 + 2) * LDG + pw] = (__bf16)v.z;
      gT[(c4 + 3) * LDG + pw] = (__bf16)v.w;
    }
    for (int i = threadIdx.x; i < (TPW + 2 * NH) * (NC / 4); i += 256) {
      const int pw = i / (NC / 4), c4 = (i % (NC / 4)) * 4;
      const int p = p0 - NH + pw;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p >= 0 && p < L) v = *reinterpret_cast<const float4 *>(a + (row * L + p) * NC + c4);
      split_store<1>(aP + pw * LDC + c4, 0, v);
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < TPW; kb += 16) {
      const bf16x8 af = *reinterpret_cast<const bf16x8 *>(gT + col * LDG + kb + 8 * hi);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int t = wave + 4 * j;
        if (t < NK) {
          bf16x8 bv;
#pragma unroll
          for (int e = 0; e < 8; ++e) bv[e] = aP[(kb + 8 * hi + e + t) * LDC + col];
          acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af, bv, acc[j], 0, 0, 0);
        }
      }
    }
  }
  // tile element (co, ci) of tap t -> partial [co][ci][t]
  float *dst = partials + (long long)blockIdx.x * (NC * NC * NK);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const int t = wave + 4 * j;
    if (t < NK) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int co = 8 * (r >> 2) + 4 * hi + (r & 3);
        dst[(co * NC + col) * NK + t] = acc[j][r];
      }
    }
  }
}

// weight gradient of an edge layer (1 <-> 32 channels), FP32:
// dW[c][t] = sum_{row, p} G[p][c] S[p + sgn (t - 4)]
constexpr int TPE = 256;

__global__ __launch_bounds__(256) void k_net_wgrad_edge(const float *__restrict__ G, const float *__restrict__ S,
                                                        float *__restrict__ partials, int L, int segs, long long rows,
                                                        int sgn) {
  __shared__ float sG[TPE * (NC + 1)];
  __shared__ float sS[TPE + 2 * NH];
  float acc[2] = {0.f, 0.f};
  const long long items = rows * segs;
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const long long row = it / segs;
    const int p0 = (int)(it - row * segs) * TPE;
    __syncthreads();
    for (int i = threadIdx.x; i < TPE * (NC / 4); i += 256) {
      const int pw = i / (NC / 4), c4 = (i % (NC / 4)) * 4;
      const int p = p0 + pw;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (p < L) v = *reinterpret_cast<const float4 *>(G + (row * L + p) * NC + c4);
      float *d = sG + pw * (NC + 1) + c4;
      d[0] = v.x;
      d[1] = v.y;
      d[2] = v.z;
      d[3] = v.w;
    }
    for (int i = threadIdx.x; i < TPE + 2 * NH; i += 256) {
      const int p = p0 - NH + i;
      sS[i] = (p >= 0 && p < L) ? S[row * L + p] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int slot = threadIdx.x + 256 * j;
      if (slot < NC * NK) {
        const int c = slot / NK, t = slot % NK;
        const int sh = NH + sgn * (t - NH);
        float a = acc[j];
        for (int pw = 0; pw < TPE; ++pw) a = fmaf(sG[pw * (NC + 1) + c], sS[pw + sh], a);
        acc[j] = a;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int slot = threadIdx.x + 256 * j;
    if (slot < NC * NK) partials[(long long)blockIdx.x * (NC * NK) + slot] = acc[j];
  }
}

// out[j] = scale * sum_i partials[i][j], FP64, fixed order
__global__ __launch_bounds__(256) void k_net_reduce(const float *__restrict__ partials, int nparts, int count,
                                                    float *__restrict__ out, double scale) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  double s = 0.0;
  for (int i = 0; i < nparts; ++i) s += (double)partials[(long long)i * count + j];
  out[j] = (float)(s * scale);
}

// Adam with bias correction, FP32 state, FP64 arithmetic
__global__ __launch_bounds__(256) void k_net_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ g, int n, double lr, double b1, double b2,
                                                  double eps, double bc1, double bc2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double gi = g[i];
  const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
  const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
  m[i] = (float)mi;
  v[i] = (float)vi;
  w[i] = (float)((double)w[i] - lr * (mi / bc1) / (sqrt(vi / bc2) + eps));
}

// Derived layouts of the master weights W1 [32][1][9], W2, W3 [32][32][9],
// W4 [1][32][9] (bfloat16-rounded values):
//  fwd: w1 [c][t], w2b/w3b [co][t][ci], w4 [c][t]
//  transposed (flipped taps): w4t [c][t] = W4[0][c][8-t], w3t/w2t [ci][t][co] = W[co][ci][8-t],
//  w1t [c][t] = W1[c][0][8-t]
__global__ __launch_bounds__(256) void k_net_prep(const float *__restrict__ W, NetW nw) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n1 = NC * NK, n2 = NC * NC * NK;
  if (i < n1) {
    const int c = i / NK, t = i % NK;
    const float w1 = (float)(__bf16)W[i];
    nw.w1[i] = w1;
    nw.w1t[c * NK + (NK - 1 - t)] = w1;
    const float w4 = (float)(__bf16)W[n1 + 2 * n2 + i];
    nw.w4[i] = w4;
    nw.w4t[c * NK + (NK - 1 - t)] = w4;
  }
  if (i < n2) {
    const int co = i / (NC * NK), rem = i % (NC * NK), ci = rem / NK, t = rem % NK;
    const __bf16 a2 = (__bf16)W[n1 + i], a3 = (__bf16)W[n1 + n2 + i];
    nw.w2b[(co * NK + t) * NC + ci] = a2;
    nw.w3b[(co * NK + t) * NC + ci] = a3;
    nw.w2t[(ci * NK + (NK - 1 - t)) * NC + co] = a2;
    nw.w3t[(ci * NK + (NK - 1 - t)) * NC + co] = a3;
  }
}

// r = xhat - x with per-workgroup partials of the FP64 sums ||r||^2 and ||x||^2
__global__ __launch_bounds__(256) void k_net_resid(const float *__restrict__ xhat, const float *__restrict__ x,
                                                   float *__restrict__ r, long long n, double *partials) {
  __shared__ double red[4];
  double rr = 0.0, xx = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const float d = xhat[i] - x[i];
    r[i] = d;
    rr = fma((double)d, (double)d, rr);
    xx = fma((double)x[i], (double)x[i], xx);
  }
  const double brr = block_sum<256>(rr, red);
  const double bxx = block_sum<256>(xx, red);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = brr;
    partials[2 * blockIdx.x + 1] = bxx;
  }
}

// sums[0], sums[1] from the nb partial pairs of k_net_resid (fixed order)
__global__ __launch_bounds__(256) void k_net_resid_finalize(const double *__restrict__ partials, int nb,
                                                            double *sums) {
  __shared__ double red[4];
  const double ta = partial_total<256>(partials, (unsigned)nb, 2, red);
  const double tb = partial_total<256>(partials + 1, (unsigned)nb, 2, red);
  if (threadIdx.x == 0) {
    sums[0] = ta;
    sums[1] = tb;
  }
}

__global__ __launch_bounds__(256) void k_net_scale(float *__restrict__ r, long long n, const double *sums, int batch) {
  const double sc = 2.0 / (sums[1] * batch);
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
    r[i] = (float)((double)r[i] * sc);
}

}  // namespace

int net_segments(int L, int tile) { return (L + tile - 1) / tile; }

void launch_net_resid(const float *xhat, const float *x, float *r, long long n, double *partials, double *sums,
                      hipStream_t st) {
  const int nb = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_net_resid, dim3(nb), dim3(256), 0, st, xhat, x, r, n, partials);
  hipLaunchKernelGGL(k_net_resid_finalize, dim3(1), dim3(256), 0, st, (const double *)partials, nb, sums);
}

void launch_net_scale(float *r, long long n, const double *sums, int batch, hipStream_t st) {
  const int nb = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_net_scale, dim3(nb), dim3(256), 0, st, r, n, sums, batch);
}

void launch_net_c1(Col<const float> s, float *out, unsigned *mask, const float *w, int L, long long rows, int mode,
                   const int *stop, hipStream_t st) {
  const int segs = net_segments(L, TP1);
  const dim3 grid((unsigned)(rows * segs));
  if (mode == 1)
    hipLaunchKernelGGL(k_net_c1<1>, grid, dim3(256), 0, st, s, out, mask, w, L, segs, rows, stop);
  else if (mode == 2)
    hipLaunchKernelGGL(k_net_c1<2>, grid, dim3(256), 0, st, s, out, mask, w, L, segs, rows, stop);
  else
    hipLaunchKernelGGL(k_net_c1<0>, grid, dim3(256), 0, st, s, out, mask, w, L, segs, rows, stop);
}

void launch_net_c4(const float *a, float *out, const float *w, int L, long long rows, const int *stop,
                   hipStream_t st) {
  const int segs = net_segments(L, TP4);
  hipLaunchKernelGGL(k_net_c4, dim3((unsigned)(rows * segs)), dim3(256), 0, st, a, out, w, L, segs, rows, stop);
}

void launch_net_c32(const float *a, float *out, unsigned *mask, const __bf16 *wb, int L, long long rows, int nsplit,
                    int mode, const int *stop, hipStream_t st) {
  const int segs = net_segments(L, TPC);
  const dim3 grid((unsigned)(rows * segs)), blk(256);
#define NET_C32(S, M) hipLaunchKernelGGL((k_net_c32<S, M>), grid, blk, 0, st, a, out, mask, wb, L, segs, rows, stop)
  if (nsplit == 3) {
    if (mode == 1)
      NET_C32(3, 1);
    else if (mode == 2)
      NET_C32(3, 2);
    else
      NET_C32(3, 0);
  } else {
    if (mode == 1)
      NET_C32(1, 1);
    else if (mode == 2)
      NET_C32(1, 2);
    else
      NET_C32(1, 0);
  }
#undef NET_C32
}

int net_wgrad_blocks() { return 1024; }

void launch_net_wgrad32(const float *g, const float *a, float *partials, int L, long long rows, hipStream_t st) {
  const int segs = net_segments(L, TPW);
  hipLaunchKernelGGL(k_net_wgrad32, dim3(net_wgrad_blocks()), dim3(256), 0, st, g, a, partials, L, segs, rows);
}

void launch_net_wgrad_edge(const float *G, const float *S, float *partials, int L, long long rows, int sgn,
                           hipStream_t st) {
  const int segs = net_segments(L, TPE);
  hipLaunchKernelGGL(k_net_wgrad_edge, dim3(net_wgrad_blocks()), dim3(256), 0, st, G, S, partials, L, segs, rows,
                     sgn);
}

void launch_net_reduce(const float *partials, int nparts, int count, float *out, double scale, hipStream_t st) {
  hipLaunchKernelGGL(k_net_reduce, dim3((count + 255) / 256), dim3(256), 0, st, partials, nparts, count, out, scale);
}

void launch_net_adam(float *w, float *m, float *v, const float *g, int n, double lr, double b1, double b2,
                     double eps, int step, hipStream_t st) {
  const double bc1 = 1.0 - std::pow(b1, step), bc2 = 1.0 - std::pow(b2, step);
  hipLaunchKernelGGL(k_net_adam, dim3((n + 255) / 256), dim3(256), 0, st, w, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
}

void launch_net_prep(const float *W, const NetW &nw, hipStream_t st) {
  hipLaunchKernelGGL(k_net_prep, dim3((NC * NC * NK + 255) / 256), dim3(256), 0, st, W, nw);
}

}  // namespace gkb
