// Device helpers of the batched launches: which slice a workgroup belongs to,
// and the slice's vector operands.
#pragma once

#include "internal.h"

namespace gkb {

// Active-slice index a with pre[a] <= blk < pre[a+1] (pre: na+1 ascending
// entries, pre[0] = 0).  The search is uniform across the workgroup.
__device__ inline int find_slice(const int *__restrict__ pre, int na, unsigned blk) {
  int lo = 0, hi = na;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if ((unsigned)pre[mid] <= blk)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Slice and local workgroup of this workgroup in a launch of family fam.
template <typename T>
__device__ inline const SliceDev<T> &slice_of(const BatchDev<T> &bd, int fam, unsigned blk, Blk &b) {
  const int *pre = bd.pre + fam * (bd.na + 1);
  const int a = find_slice(pre, bd.na, blk);
  b.id = blk - (unsigned)pre[a];
  b.n = (unsigned)(pre[a + 1] - pre[a]);
  return bd.sd[bd.active[a]];
}

// Launches made after a solve has stopped (solution assembly) run on stopped
// slices too.
template <typename T>
__device__ inline bool skip(const BatchDev<T> &bd, const SliceDev<T> &d) {
  return !bd.ignore_stop && d.ctl.ip[CI_STOP];
}

template <typename T>
__device__ inline T *resolve(const SliceDev<T> &d, int sel, int k) {
  switch (sel) {
    case BS_B: return const_cast<T *>(d.b);
    case BS_X: return d.x;
    case BS_S: return d.s;
    case BS_W: return d.w;
    case BS_TN: return d.tn;
    case BS_TM: return d.tm;
    case BS_Q_PREV: return d.Q + (long long)(k - 1) * d.ldq;
    case BS_Y_CUR: return d.yk;
    default: return nullptr;
  }
}

}  // namespace gkb
