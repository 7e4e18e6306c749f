// Epilogue shared by the projector kernels (2D and 3D).
#pragma once

#include "internal.h"
#include "reduce.h"

namespace gkb {

// Element idx of a vector into its padded copy (see PadOut).
template <typename T>
__device__ inline void pad_store(const PadOut<T> &p, long long idx, T v) {
  // 2D vectors have fewer than 2^31 elements
  const unsigned a = (unsigned)idx / (unsigned)p.n1, b = (unsigned)idx - a * (unsigned)p.n1;
  if (p.kind == PADK_IMAGE) {  // a = row j, b = column i
    p.dst[(long long)a * p.lead + p.off0 + b] = v;
    if (p.offT >= 0) p.dst[p.offT + (long long)b * p.ldT + p.off0 + a] = v;
  } else {  // a = view, b = bin
    const long long q = (long long)a * p.lead + p.off0 + b;
    if (p.kind == PADK_SINO) {
      p.dst[q] = v;
    } else {
      const T w = p.w[idx];
      p.dst[2 * q] = w * v;
      p.dst[2 * q + 1] = w;
    }
  }
}

// Epilogue shared by all projector kernels.  Every thread of the block calls
// it (the norm reduction needs the whole block).
template <typename T>
__device__ inline void epilogue(const Epi<T> &e, long long idx, bool valid, T raw, T *outp, Blk b) {
  __shared__ double red[kBlock / 64];
  double out = (double)raw;
  int k = 0;
  if (e.use_ctl) {
    k = e.ctl.ip[CI_K];
    if (e.in_sel == IN_INV_TNEXT) out = out / e.ctl.t[k + 1];
    if (e.prev_sel != PREV_NONE && valid) {
      const double pc =
          (e.prev_sel == PREV_NEG_ALPHA_OVER_T) ? -e.ctl.alpha[k] / e.ctl.t[k] : -e.ctl.t[k + 1];
      out = fma(pc, (double)e.prev.get()[idx], out);
    }
  }
  const T outT = (T)out;
  if (valid) {
    outp[idx] = outT;
    if (e.out_raw.base) e.out_raw.get()[idx] = raw;
    if (e.pout.dst) pad_store(e.pout, idx, outT);
  }
  // ||out||^2: one partial per workgroup; a finalising kernel launched after
  // the projector sums them into t[k+1]
  if (e.norm_to_t) {
    const double v = valid ? (double)outT * (double)outT : 0.0;
    const double bs = block_sum<kBlock>(v, red);
    if (threadIdx.x == 0) e.partials[b.id] = bs;
  }
}

}  // namespace gkb
