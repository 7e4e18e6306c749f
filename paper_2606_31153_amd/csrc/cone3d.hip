// 3D cone-beam projector kernels for gfx950 (flat detector): Joseph forward
// A and its exact adjoint A^T, voxel-driven bilinear back projector B and its
// exact adjoint B^T.  These are the cone-beam counterparts of the 2D pair of
// Sec. 1 (A x ~= b with B != A^T); the GKB recurrences of Sec. 3 apply them
// unchanged.
//
// Geometry (voxel pitch 1, voxel (i,j,l) centred at (i-(nx-1)/2, j-(ny-1)/2,
// l-(nz-1)/2)): source S = D (cos b, sin b, 0); the detector plane is
// perpendicular to the central ray c = -(cos b, sin b, 0) at distance SDD
// from the source, with axes e_u = (-sin b, cos b, 0) and e_z; the ray of
// detector pixel (k, r) has direction d = SDD c + u_k e_u + v_r e_z with
// u_k = (k - (nu-1)/2) du and v_r = (r - (nw-1)/2) dw.
//
//  * A: Joseph's method in 3D.  Each ray steps through the voxel planes
//    perpendicular to its dominant axis (x or y; geometries in which z could
//    dominate are rejected on the host); in every plane the volume is
//    interpolated bilinearly at the crossing; the sum is scaled by
//    |d| / |d_dom|.
//  * B: every voxel centre is projected onto the detector (perspective
//    division by its depth along c) and the view is interpolated bilinearly.
//  * A^T, B^T: exact transposes, both as gathers (no atomics, fixed order).
//    A^T runs over voxels: for view v the rays that sample voxel p are the
//    columns k near p's detector coordinate u_p; in p's plane along the ray's
//    dominant axis, ray k passes at the in-plane offset
//    depth * du * (k - u_p) / d_dom(k) from p (similar triangles through the
//    source), and row r at height lambda_k v_r with lambda_k the ray
//    parameter of that plane.  B^T runs over rays: in each plane along the
//    ray, the voxels whose projection lies within one detector pixel of
//    (k, r), found from the ray's crossing and a per-ray half-width.
//
// Layouts (all zero padded so that every tap is in bounds without a test):
//  * volume x[l][j][i]; for A and B^T two copies: x-dominant rays read
//    [i][l+P][j+P] (the in-plane coordinate that changes along a detector row
//    is contiguous), y-dominant rays read [j][l+P][i+P];
//  * sinogram y[v][r][k]; B reads a copy padded to [v][r+PY][k+PY];
//  * A^T reads w * y, w = |d| / |d_dom| of each ray, precomputed per call.

#include <algorithm>

#include "devmath.h"
#include "epilogue.h"
#include "internal.h"

namespace gkb {

namespace {

// ray (view v, row r, column k) of detector index rr
struct RayIdx {
  int v, r, k;
  long long vk;
};
__device__ inline RayIdx ray_index(const GeomDev &g, long long rr) {
  RayIdx q;
  q.k = (int)(rr % g.nu);
  const long long vr = rr / g.nu;
  q.r = (int)(vr % g.nw);
  q.v = (int)(vr / g.nw);
  q.vk = (long long)q.v * g.nu + q.k;
  return q;
}

// depth along the central ray and the numerator of the detector u coordinate
// of the point (x, y, .) in view (cb, sb): u = unum * SDD / (du * depth) + offu
template <typename T>
__device__ inline void cone_project(T x, T y, T cb, T sb, T D, T &unum, T &depth) {
  depth = D - fma(x, cb, y * sb);
  unum = fma(y, cb, -(x * sb));
}

// voxel of this thread: 32 x 8 tiles in (i, j), one slab l per tile row
__device__ inline void voxel_of(const GeomDev &g, unsigned blk, int &i, int &j, int &l) {
  const int tiles_x = (g.nx + 31) >> 5, tiles = tiles_x * ((g.ny + 7) >> 3);
  l = (int)blk / tiles;
  const int t = (int)blk - l * tiles;
  i = (t % tiles_x) * 32 + (threadIdx.x & 31);
  j = (t / tiles_x) * 8 + (threadIdx.x >> 5);
}

// ---------------------------------------------------------------------------
// padded copies
// ---------------------------------------------------------------------------
// x-dominant copy [i][lp][jp] (lp = l + P, jp = j + P): tiles of 32 (jp) x 32 (i)
// in padded slab lp, transposed through LDS
template <typename T>
__global__ __launch_bounds__(256) void k_cone_pad_x(Col<const T> xc, T *__restrict__ pad, GeomDev g,
                                                    const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ x = xc.get();
  __shared__ T tile[32][33];
  const int P = g.P3;
  const int jp0 = blockIdx.x * 32, i0 = blockIdx.y * 32, lp = blockIdx.z;
  const int l = lp - P;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const bool lin = (unsigned)l < (unsigned)g.nz;
  for (int q = ty; q < 32; q += 8) {
    const int j = jp0 + q - P, i = i0 + tx;
    tile[q][tx] = (lin && (unsigned)j < (unsigned)g.ny && i < g.nx) ? x[((long long)l * g.ny + j) * g.nx + i] : T(0);
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int i = i0 + q, jp = jp0 + tx;
    if (i < g.nx && jp < g.ldX) pad[(long long)i * g.planeX + (long long)lp * g.ldX + jp] = tile[tx][q];
  }
}

// y-dominant copy [j][lp][ip] at offYD: rows of the original volume, padded
template <typename T>
__global__ __launch_bounds__(256) void k_cone_pad_y(Col<const T> xc, T *__restrict__ pad, GeomDev g,
                                                    const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ x = xc.get();
  const int P = g.P3;
  const long long rows = (long long)g.ny * (g.nz + 2 * P);
  const long long total = rows * g.ldV;
  for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
    const long long row = idx / g.ldV;
    const int ip = (int)(idx - row * g.ldV);
    const int j = (int)(row / (g.nz + 2 * P)), lp = (int)(row - (long long)j * (g.nz + 2 * P));
    const int i = ip - P, l = lp - P;
    pad[g.offYD + idx] = ((unsigned)i < (unsigned)g.nx && (unsigned)l < (unsigned)g.nz)
                             ? x[((long long)l * g.ny + j) * g.nx + i]
                             : T(0);
  }
}

// sinogram padded by PY zeros in r and k: [v][r+PY][k+PY]
template <typename T>
__global__ __launch_bounds__(256) void k_cone_pad_sino(Col<const T> yc, T *__restrict__ pad, GeomDev g,
                                                       const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ y = yc.get();
  const int PY = g.PY3, rows = g.nw + 2 * PY;
  const long long total = (long long)g.nv * g.sliceY;
  for (long long idx = (long long)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (long long)gridDim.x * 256) {
    const long long row = idx / g.ldSu;
    const int kp = (int)(idx - row * g.ldSu);
    const int v = (int)(row / rows), rp = (int)(row - (long long)v * rows);
    const int k = kp - PY, r = rp - PY;
    pad[idx] = ((unsigned)k < (unsigned)g.nu && (unsigned)r < (unsigned)g.nw)
                   ? y[((long long)v * g.nw + r) * g.nu + k]
                   : T(0);
  }
}

// w * y with w = |d| / |d_dom| of each ray (input of A^T)
template <typename T>
__global__ __launch_bounds__(256) void k_cone_weight(Col<const T> yc, ConeTab<T> ct, T *__restrict__ wy, GeomDev g,
                                                     const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ y = yc.get();
  for (long long rr = (long long)blockIdx.x * 256 + threadIdx.x; rr < g.m; rr += (long long)gridDim.x * 256) {
    const RayIdx q = ray_index(g, rr);
    const T vv = (T(q.r) - T(g.offw)) * T(g.dw);
    const T w = sqrt(fma(vv, vv, ct.dxy2[q.vk])) * fabs(ct.lslope[q.vk]);
    wy[rr] = w * y[rr];
  }
}

// ---------------------------------------------------------------------------
// A: Joseph forward, one thread per ray
// ---------------------------------------------------------------------------
constexpr int kConeFwdPlanes = 12;  // planes whose tap loads are in flight together

template <typename T>
__device__ inline void cone_fwd_body(const GeomDev &g, const ConeTab<T> &ct, const T *__restrict__ pad, T *yo,
                                     const Epi<T> &e, Blk b) {
  const long long rr = (long long)b.id * kBlock + threadIdx.x;
  const bool valid = rr < g.m;
  T acc = T(0);
  if (valid) {
    const RayIdx q = ray_index(g, rr);
    const int meta = ct.meta[q.vk];
    int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
    const bool ydom = (meta >> 30) & 1;
    const T base1 = ct.base1[q.vk], slope1 = ct.slope1[q.vk], lsl = ct.lslope[q.vk];
    const T vv = (T(q.r) - T(g.offw)) * T(g.dw);
    const T midz = T(0.5) * T(g.nz - 1);
    const T base2 = fma(vv, ct.lmid[q.vk], midz), slope2 = vv * lsl;
    const T mid = ydom ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
    // planes where the height is inside [-1, nz] (one plane of margin: the
    // taps there read the zero padding)
    if (slope2 != T(0)) {
      T ta = (T(-1) - base2) / slope2, tb = (T(g.nz) - base2) / slope2;
      if (ta > tb) {
        const T tt = ta;
        ta = tb;
        tb = tt;
      }
      lo = max(lo, (int)fmin(fmax(ceil(ta + mid) - T(1), T(-1)), T(32767)));
      hi = min(hi, (int)fmin(fmax(floor(tb + mid) + T(1), T(-1)), T(32767)));
    } else if (!(base2 > T(-1) && base2 < T(g.nz))) {
      hi = lo - 1;
    }
    const int n1 = ydom ? g.nx : g.ny;
    const int ld = ydom ? g.ldV : g.ldX;
    const unsigned plane = (unsigned)(ydom ? g.planeY : g.planeX);
    const T *__restrict__ vol = pad + (ydom ? g.offYD : 0LL);
    const T c1lo = T(-1.5), c1hi = T(n1) + T(0.5), c2lo = T(-1.5), c2hi = T(g.nz) + T(0.5);
    unsigned poff = (unsigned)max(lo, 0) * plane + (unsigned)(g.P3 * ld + g.P3);
    T tf = T(lo) - mid;
    T a[kConeFwdPlanes];
#pragma unroll
    for (int u = 0; u < kConeFwdPlanes; ++u) a[u] = T(0);
    int t = lo;
    // kConeFwdPlanes planes per step: the pair loads of all of them are
    // issued before any is interpolated
    for (; t + kConeFwdPlanes - 1 <= hi; t += kConeFwdPlanes) {
      typename Pair<T>::v2 pa[kConeFwdPlanes], pb[kConeFwdPlanes];
      T fr[kConeFwdPlanes], fz[kConeFwdPlanes];
#pragma unroll
      for (int u = 0; u < kConeFwdPlanes; ++u) {
        const T p1 = clampv(fma(tf + T(u), slope1, base1), c1lo, c1hi);
        const T p2 = clampv(fma(tf + T(u), slope2, base2), c2lo, c2hi);
        const T f1 = floor(p1), f2 = floor(p2);
        const unsigned o = poff + (unsigned)u * plane + (unsigned)((int)f2 * ld + (int)f1);
        pa[u] = load_pair(vol + o);
        pb[u] = load_pair(vol + o + ld);
        fr[u] = p1 - f1;
        fz[u] = p2 - f2;
      }
#pragma unroll
      for (int u = 0; u < kConeFwdPlanes; ++u) {
        const T va = fma(fr[u], pa[u].y - pa[u].x, pa[u].x), vb = fma(fr[u], pb[u].y - pb[u].x, pb[u].x);
        a[u] += fma(fz[u], vb - va, va);
      }
      tf += T(kConeFwdPlanes);
      poff += (unsigned)kConeFwdPlanes * plane;
    }
    for (; t <= hi; ++t) {
      const T p1 = clampv(fma(tf, slope1, base1), c1lo, c1hi);
      const T p2 = clampv(fma(tf, slope2, base2), c2lo, c2hi);
      const T f1 = floor(p1), f2 = floor(p2);
      const unsigned o = poff + (unsigned)((int)f2 * ld + (int)f1);
      const auto pa = load_pair(vol + o);
      const auto pb = load_pair(vol + o + ld);
      const T fr = p1 - f1;
      const T va = fma(fr, pa.y - pa.x, pa.x), vb = fma(fr, pb.y - pb.x, pb.x);
      a[0] += fma(p2 - f2, vb - va, va);
      tf += T(1);
      poff += plane;
    }
#pragma unroll
    for (int u = 1; u < kConeFwdPlanes; ++u) a[0] += a[u];
    const T w = sqrt(fma(vv, vv, ct.dxy2[q.vk])) * fabs(lsl);
    acc = a[0] * w;
  }
  epilogue(e, rr, valid, acc, yo, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cone_fwd(GeomDev g, ConeTab<T> ct, const T *__restrict__ pad, Col<T> yc,
                                                     Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  cone_fwd_body(g, ct, pad, yc.get(), e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// B^T: transpose of the voxel-driven back projector, one thread per ray.
// Ray (v, r, k) collects every voxel whose detector coordinates (u, w) are
// within one pixel of (k, r), with the weight (1 - |u - k|)(1 - |w - r|).
// On each dominant plane those voxels lie within the ray's in-plane
// half-width h1 of its crossing, and in the rows whose projected row
// coordinate can reach r at the depths of those columns.
// ---------------------------------------------------------------------------
constexpr int kConeBtRows = 4;    // most rows of the uniform window
constexpr int kConeBtPlanes = 6;  // planes whose loads are in flight together

// Generic form: the exact candidate columns and rows of every plane, with
// data-dependent loops.  Used where the uniform windows would be too large.
template <typename T>
__device__ inline T cone_bt_ray_generic(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt,
                                        const T *__restrict__ pad, const RayIdx &q) {
  const int meta = ct.meta_bt[q.vk];
  const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
  const bool ydom = (meta >> 30) & 1;
  const T base1 = ct.base1[q.vk], slope1 = ct.slope1[q.vk], h1 = ct.h1[q.vk];
  const T cb = vt.p0[q.v], sb = vt.p1[q.v], D = T(g.D);
  const T midx = T(0.5) * T(g.nx - 1), midy = T(0.5) * T(g.ny - 1), midz = T(0.5) * T(g.nz - 1);
  const T mid = ydom ? midy : midx, mid1 = ydom ? midx : midy;
  const int n1 = ydom ? g.nx : g.ny;
  const int ld = ydom ? g.ldV : g.ldX;
  const long long plane = ydom ? g.planeY : g.planeX;
  const T *__restrict__ vol = pad + (ydom ? g.offYD : 0LL) + (g.P3 * ld + g.P3);
  const T Su = T(g.Su), Sw = T(g.Sw), offu = T(g.off), offw = T(g.offw);
  const T kf = T(q.k), rf = T(q.r);
  const T inv_sw = T(1) / Sw;
  const T eps = T(1e-3);
  T acc = T(0);
  for (int t = lo; t <= hi; ++t) {
    const T tf = T(t) - mid;
    const T c1 = fma(tf, slope1, base1);
    const int j0 = max((int)ceil(c1 - h1), 0), j1 = min((int)floor(c1 + h1), n1 - 1);
    const T *__restrict__ pl = vol + (long long)t * plane;
    for (int jj = j0; jj <= j1; ++jj) {
      const T o = T(jj) - mid1;
      T unum, depth;
      cone_project(ydom ? o : tf, ydom ? tf : o, cb, sb, D, unum, depth);
      const T inv = fast_rcp(depth);
      const T u = fma(unum, Su * inv, offu);
      const T wu = T(1) - fabs(u - kf);
      if (wu > T(0)) {
        const T mw = Sw * inv;
        // heights whose row coordinate z mw + offw is within one row of r
        const T zh = depth * inv_sw, zc = (rf - offw) * zh + midz;
        const int l0 = max((int)ceil(zc - zh - eps), 0), l1 = min((int)floor(zc + zh + eps), g.nz - 1);
        for (int l = l0; l <= l1; ++l) {
          const T ww = T(1) - fabs(fma(T(l) - midz, mw, offw) - rf);
          if (ww > T(0)) acc = fma(wu * ww, pl[(long long)l * ld + jj], acc);
        }
      }
    }
  }
  return acc;
}

// Windowed form: on every plane NJ consecutive columns from ceil(c1 - h1)
// and nl consecutive rows (NJ and nl uniform over the wavefront), every
// weight a clamped hat, no data-dependent branches.  The first row is the
// lowest that the projected row coordinate can bring within one row of r at
// the window's depths: the row interval of a column at depth d is
// midz + (rho -+ 1) d / Sw (rho = r - offw), linear in d, and the depth is
// linear along the window, so its extremes sit at the window's ends.  Both
// window starts are clamped into the padded volume; since each window is at
// least as long as the set of voxels with nonzero weight, the clamp keeps
// every such voxel of the volume inside it.  Planes where the ray's height
// is farther than the window's reach from the volume are skipped.
template <typename T, int NJ>
__device__ inline T cone_bt_ray_win(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt,
                                    const T *__restrict__ pad, const RayIdx &q, int nl) {
  const int meta = ct.meta_bt[q.vk];
  int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
  const bool ydom = (meta >> 30) & 1;
  const T base1 = ct.base1[q.vk], slope1 = ct.slope1[q.vk], h1 = ct.h1[q.vk];
  const T cb = vt.p0[q.v], sb = vt.p1[q.v], D = T(g.D);
  const T midx = T(0.5) * T(g.nx - 1), midy = T(0.5) * T(g.ny - 1), midz = T(0.5) * T(g.nz - 1);
  const T mid = ydom ? midy : midx, mid1 = ydom ? midx : midy;
  const int n1 = ydom ? g.nx : g.ny;
  const int ld = ydom ? g.ldV : g.ldX;
  const long long plane = ydom ? g.planeY : g.planeX;
  const T *__restrict__ vol = pad + (ydom ? g.offYD : 0LL) + (g.P3 * ld + g.P3);
  const T Su = T(g.Su), Sw = T(g.Sw), inv_sw = T(1) / Sw;
  const T rho = T(q.r) - T(g.offw);
  const T eps = T(1e-3);
  // depth D - (x cos + y sin) and Su (y cos - x sin) of the voxel at in-plane
  // offset o on the plane at offset tf: affine in o and in tf
  const T ddo = ydom ? -cb : -sb, duo = (ydom ? -sb : cb) * Su;
  const T dtt = ydom ? -sb : -cb, utt = (ydom ? cb : -sb) * Su;
  {
    // height of the ray at plane offset tf: base2 + slope2 tf; a voxel of the
    // window is within zm rows of it
    const T vv = rho * T(g.dw);
    const T base2 = fma(vv, ct.lmid[q.vk], midz), slope2 = vv * ct.lslope[q.vk];
    const T zm = fma(T(g.dmax3), inv_sw, fabs(rho) * inv_sw * (h1 + T(1))) + T(1);
    if (slope2 != T(0)) {
      T ta = (T(-1) - zm - base2) / slope2, tb = (T(g.nz) + zm - base2) / slope2;
      if (ta > tb) {
        const T tt = ta;
        ta = tb;
        tb = tt;
      }
      lo = max(lo, (int)fmin(fmax(ceil(ta + mid) - T(1), T(-1)), T(32767)));
      hi = min(hi, (int)fmin(fmax(floor(tb + mid) + T(1), T(-1)), T(32767)));
    } else if (!(base2 > T(-1) - zm && base2 < T(g.nz) + zm)) {
      hi = lo - 1;
    }
  }
  // lowest row reachable: midz + rm d at the window end that minimises it
  const T rm = (rho - T(1)) * inv_sw;
  const bool last_end = (rm >= T(0)) != (ddo >= T(0));
  const T cmin = (last_end ? rm * (T(NJ - 1) * ddo) : T(0)) + (midz - eps);
  const T cu = T(g.off) - T(q.k), cw = T(g.offw) - T(q.r);
  const T jlo = T(-g.P3), jhi = T(n1 - 1 + g.P3 - (NJ - 1));
  const T llo = T(-g.P3), lhi = T(g.nz - 1 + g.P3 - (nl - 1));
  // plane t's window: the depth and Su * unum of its first column, the
  // height offset of its first row, and its values
  auto window = [&](int t, T &dep0, T &uns0, T &z0, T (&v)[kConeBtRows][NJ]) {
    const T tf = T(t) - mid;
    const T j0f = clampv(T(ceil(T(fma(tf, slope1, base1)) - h1)), jlo, jhi);
    const T o0 = j0f - mid1;
    dep0 = T(fma(o0, ddo, T(fma(tf, dtt, D))));
    uns0 = T(fma(o0, duo, tf * utt));
    const T l0f = clampv(T(ceil(T(fma(rm, dep0, cmin)))), llo, lhi);
    z0 = l0f - midz;
    const T *__restrict__ pl = vol + (long long)t * plane + ((int)l0f * ld + (int)j0f);
#pragma unroll
    for (int p = 0; p < kConeBtRows; ++p)
      if (p < nl) {
#pragma unroll
        for (int c = 0; c < NJ; ++c) v[p][c] = pl[p * ld + c];
      }
  };
  auto weigh = [&](T dep0, T uns0, T z0, const T (&v)[kConeBtRows][NJ], T &acc) {
#pragma unroll
    for (int c = 0; c < NJ; ++c) {
      const T dep = c == 0 ? dep0 : T(fma(T(c), ddo, dep0));
      const T uns = c == 0 ? uns0 : T(fma(T(c), duo, uns0));
      const T inv = fast_rcp(dep);
      const T wu = hat_clamp(T(T(1) - fabs(T(fma(uns, inv, cu)))));
      const T mw = Sw * inv;
      const T b0 = T(fma(z0, mw, cw));
      T col = T(0);
#pragma unroll
      for (int p = 0; p < kConeBtRows; ++p)
        if (p < nl) {
          const T wr = p == 0 ? b0 : T(fma(T(p), mw, b0));
          col = T(fma(hat_clamp(T(T(1) - fabs(wr))), v[p][c], col));
        }
      acc = T(fma(wu, col, acc));
    }
  };
  // kConeBtPlanes planes per step: the loads of all of them are issued
  // before any is weighed
  T acc = T(0);
  int t = lo;
  for (; t + kConeBtPlanes - 1 <= hi; t += kConeBtPlanes) {
    T d[kConeBtPlanes], u[kConeBtPlanes], z[kConeBtPlanes];
    T v[kConeBtPlanes][kConeBtRows][NJ];
#pragma unroll
    for (int i = 0; i < kConeBtPlanes; ++i) window(t + i, d[i], u[i], z[i], v[i]);
#pragma unroll
    for (int i = 0; i < kConeBtPlanes; ++i) weigh(d[i], u[i], z[i], v[i], acc);
  }
  for (; t <= hi; ++t) {
    T da, ua, za;
    T va[kConeBtRows][NJ];
    window(t, da, ua, za, va);
    weigh(da, ua, za, va, acc);
  }
  return acc;
}

template <typename T>
__device__ inline void cone_back_adj_body(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt,
                                          const T *__restrict__ pad, T *yo, const Epi<T> &e, Blk b) {
  const long long rr = (long long)b.id * kBlock + threadIdx.x;
  const bool valid = rr < g.m;
  const RayIdx q = ray_index(g, valid ? rr : 0);
  // uniform window sizes: columns floor(2 h1) + 1 (at least 2); rows from the
  // largest row interval over the window's depth range
  const T h1 = ct.h1[q.vk];
  const int nj = max(wave_max(valid ? (int)floor(T(2) * h1) + 1 : 0), 2);
  const bool ydom = (ct.meta_bt[q.vk] >> 30) & 1;
  const T ddo = fabs(ydom ? vt.p0[q.v] : vt.p1[q.v]);
  const T rho = fabs(T(q.r) - T(g.offw));
  const int nl_ray = (int)floor(fma(T(2), T(g.dmax3), rho * ddo * T(nj - 1)) / T(g.Sw) + T(2e-3)) + 1;
  const int nl = wave_max(valid ? nl_ray : 0);
  T acc = T(0);
  if (valid) {
    const bool fits = nl <= kConeBtRows && nl <= g.nz + 2 * g.P3 && nj <= min(g.nx, g.ny) + 2 * g.P3;
    if (fits && nj == 2)
      acc = cone_bt_ray_win<T, 2>(g, ct, vt, pad, q, nl);
    else if (fits && nj == 3)
      acc = cone_bt_ray_win<T, 3>(g, ct, vt, pad, q, nl);
    else if (fits && nj == 4)
      acc = cone_bt_ray_win<T, 4>(g, ct, vt, pad, q, nl);
    else if (fits && nj == 5)
      acc = cone_bt_ray_win<T, 5>(g, ct, vt, pad, q, nl);
    else
      acc = cone_bt_ray_generic(g, ct, vt, pad, q);
  }
  epilogue(e, rr, valid, acc, yo, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cone_back_adj(GeomDev g, ConeTab<T> ct, ViewTab<T> vt,
                                                          const T *__restrict__ pad, Col<T> yc, Epi<T> e,
                                                          const int *stop) {
  if (stop && *stop) return;
  cone_back_adj_body(g, ct, vt, pad, yc.get(), e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// B: voxel-driven bilinear back projection, one thread per voxel
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void cone_back_body(const GeomDev &g, const ViewTab<T> &vt, const T *__restrict__ ypad, T *xo,
                                      const Epi<T> &e, Blk b) {
  int i, j, l;
  voxel_of(g, b.id, i, j, l);
  const bool valid = i < g.nx && j < g.ny;
  T acc = T(0);
  if (valid) {
    const T x = T(i) - T(0.5) * T(g.nx - 1), y = T(j) - T(0.5) * T(g.ny - 1), z = T(l) - T(0.5) * T(g.nz - 1);
    const T D = T(g.D), Su = T(g.Su), Sw = T(g.Sw), offu = T(g.off), offw = T(g.offw);
    const T ulo = T(-2), uhi = T(g.nu), wlo = T(-2), whi = T(g.nw);
    const int ld = g.ldSu;
    unsigned voff = (unsigned)(g.PY3 * ld + g.PY3);
    T a0 = T(0), a1 = T(0);
    int v = 0;
    for (; v + 1 < g.nv; v += 2) {
      T s[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        T unum, depth;
        cone_project(x, y, vt.p0[v + q], vt.p1[v + q], D, unum, depth);
        const T inv = fast_rcp(depth);
        const T u = clampv(fma(unum, Su * inv, offu), ulo, uhi);
        const T w = clampv(fma(z, Sw * inv, offw), wlo, whi);
        const T fu = floor(u), fw = floor(w);
        const unsigned o = voff + (unsigned)q * (unsigned)g.sliceY + (unsigned)((int)fw * ld + (int)fu);
        const auto pa = load_pair(ypad + o);
        const auto pb = load_pair(ypad + o + ld);
        const T fr = u - fu;
        const T va = fma(fr, pa.y - pa.x, pa.x), vb = fma(fr, pb.y - pb.x, pb.x);
        s[q] = fma(w - fw, vb - va, va);
      }
      a0 += s[0];
      a1 += s[1];
      voff += 2u * (unsigned)g.sliceY;
    }
    if (v < g.nv) {
      T unum, depth;
      cone_project(x, y, vt.p0[v], vt.p1[v], D, unum, depth);
      const T inv = fast_rcp(depth);
      const T u = clampv(fma(unum, Su * inv, offu), ulo, uhi);
      const T w = clampv(fma(z, Sw * inv, offw), wlo, whi);
      const T fu = floor(u), fw = floor(w);
      const unsigned o = voff + (unsigned)((int)fw * ld + (int)fu);
      const auto pa = load_pair(ypad + o);
      const auto pb = load_pair(ypad + o + ld);
      const T fr = u - fu;
      const T va = fma(fr, pa.y - pa.x, pa.x), vb = fma(fr, pb.y - pb.x, pb.x);
      a0 += fma(w - fw, vb - va, va);
    }
    acc = a0 + a1;
  }
  epilogue(e, valid ? ((long long)l * g.ny + j) * g.nx + i : 0, valid, acc, xo, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cone_back(GeomDev g, ViewTab<T> vt, const T *__restrict__ ypad,
                                                      T *__restrict__ xo, Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  cone_back_body(g, vt, ypad, xo, e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// A^T: transpose of Joseph's projector, one thread per voxel
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void cone_fwd_adj_body(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt,
                                         const T *__restrict__ wy, T *xo, const Epi<T> &e, Blk b) {
  int i, j, l;
  voxel_of(g, b.id, i, j, l);
  const bool valid = i < g.nx && j < g.ny;
  T acc = T(0);
  if (valid) {
    const T x = T(i) - T(0.5) * T(g.nx - 1), y = T(j) - T(0.5) * T(g.ny - 1), z = T(l) - T(0.5) * T(g.nz - 1);
    const T D = T(g.D), Su = T(g.Su), offu = T(g.off), offw = T(g.offw), du = T(g.du), dw = T(g.dw);
    const T hk_fac = T(g.hk_fac);
    const T eps = T(1e-3);
    for (int v = 0; v < g.nv; ++v) {
      const T cb = vt.p0[v], sb = vt.p1[v];
      T unum, depth;
      cone_project(x, y, cb, sb, D, unum, depth);
      const T inv = fast_rcp(depth);
      const T u = fma(unum, Su * inv, offu);
      // columns whose rays pass within one voxel (in the ray's plane) of p
      const T hk = fma(hk_fac, inv, T(1e-4));
      const int k0 = max((int)ceil(u - hk), 0), k1 = min((int)floor(u + hk), g.nu - 1);
      const T dd = depth * du;
      const T dxs = x - D * cb, dys = y - D * sb;
      const typename Pair<T>::v2 *pk = reinterpret_cast<const typename Pair<T>::v2 *>(ct.pk) + (long long)v * g.nu;
      const T *__restrict__ wv = wy + (long long)v * g.nw * g.nu;
      for (int k = k0; k <= k1; ++k) {
        const auto pq = pk[k];  // (1/d_dom, y-dominant)
        const T wxy = T(1) - fabs(dd * (T(k) - u) * pq.x);
        if (wxy > T(0)) {
          // ray parameter of p's plane along this ray's dominant axis; the
          // row-r ray is at height lam * v_r there
          const T lam = (pq.y != T(0) ? dys : dxs) * pq.x;
          const T ldw = lam * dw;
          const T rh = fast_rcp(ldw), rc = fma(z, rh, offw);
          const int r0 = max((int)ceil(rc - rh - eps), 0), r1 = min((int)floor(rc + rh + eps), g.nw - 1);
          for (int r = r0; r <= r1; ++r) {
            const T wz = T(1) - fabs(fma(ldw, T(r) - offw, -z));
            if (wz > T(0)) acc = fma(wxy * wz, wv[(long long)r * g.nu + k], acc);
          }
        }
      }
    }
  }
  epilogue(e, valid ? ((long long)l * g.ny + j) * g.nx + i : 0, valid, acc, xo, b);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cone_fwd_adj(GeomDev g, ConeTab<T> ct, ViewTab<T> vt,
                                                         const T *__restrict__ wy, T *__restrict__ xo, Epi<T> e,
                                                         const int *stop) {
  if (stop && *stop) return;
  cone_fwd_adj_body(g, ct, vt, wy, xo, e, Blk{blockIdx.x, gridDim.x});
}

int grid_stride_blocks(long long total) { return (int)std::min<long long>((total + 255) / 256, 8192); }

}  // namespace

int cone_voxel_blocks(const GeomDev &g) { return ((g.nx + 31) / 32) * ((g.ny + 7) / 8) * g.nz; }

template <typename T>
void launch_cone_pad_volume(const GeomDev &g, Col<const T> x, T *pad, int want_x, int want_y, const int *stop,
                            hipStream_t s) {
  if (want_x) {
    const dim3 grid((g.ldX + 31) / 32, (g.nx + 31) / 32, g.nz + 2 * g.P3);
    hipLaunchKernelGGL(k_cone_pad_x<T>, grid, dim3(256), 0, s, x, pad, g, stop);
  }
  if (want_y) {
    const long long tot = (long long)g.ny * (g.nz + 2 * g.P3) * g.ldV;
    hipLaunchKernelGGL(k_cone_pad_y<T>, dim3(grid_stride_blocks(tot)), dim3(256), 0, s, x, pad, g, stop);
  }
}

template <typename T>
void launch_cone_pad_sino(const GeomDev &g, Col<const T> y, T *pad, const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_cone_pad_sino<T>, dim3(grid_stride_blocks(g.sino_pad_elems)), dim3(256), 0, s, y, pad, g,
                     stop);
}

template <typename T>
void launch_cone_weight_sino(const GeomDev &g, const ConeTab<T> &ct, Col<const T> y, T *wy, const int *stop,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cone_weight<T>, dim3(grid_stride_blocks(g.m)), dim3(256), 0, s, y, ct, wy, g, stop);
}

template <typename T>
void launch_cone_fwd(const GeomDev &g, const ConeTab<T> &ct, const T *pad, Col<T> y, const Epi<T> &e,
                     const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_cone_fwd<T>, dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, ct, pad, y, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, ray_blocks(g), NORM_T1, stop, s);
}

template <typename T>
void launch_cone_back_adj(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt, const T *pad, Col<T> y,
                          const Epi<T> &e, const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_cone_back_adj<T>, dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, ct, vt, pad, y, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, ray_blocks(g), NORM_T1, stop, s);
}

template <typename T>
void launch_cone_back(const GeomDev &g, const ViewTab<T> &vt, const T *ypad, T *x, const Epi<T> &e,
                      const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_cone_back<T>, dim3(cone_voxel_blocks(g)), dim3(kBlock), 0, s, g, vt, ypad, x, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, cone_voxel_blocks(g), NORM_T1, stop, s);
}

template <typename T>
void launch_cone_fwd_adj(const GeomDev &g, const ConeTab<T> &ct, const ViewTab<T> &vt, const T *wy, T *x,
                         const Epi<T> &e, const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_cone_fwd_adj<T>, dim3(cone_voxel_blocks(g)), dim3(kBlock), 0, s, g, ct, vt, wy, x, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, cone_voxel_blocks(g), NORM_T1, stop, s);
}

#define GKB_INST(T)                                                                                             \
  template void launch_cone_pad_volume<T>(const GeomDev &, Col<const T>, T *, int, int, const int *,          \
                                          hipStream_t);                                                       \
  template void launch_cone_pad_sino<T>(const GeomDev &, Col<const T>, T *, const int *, hipStream_t);        \
  template void launch_cone_weight_sino<T>(const GeomDev &, const ConeTab<T> &, Col<const T>, T *,            \
                                           const int *, hipStream_t);                                         \
  template void launch_cone_fwd<T>(const GeomDev &, const ConeTab<T> &, const T *, Col<T>, const Epi<T> &,    \
                                   const int *, hipStream_t);                                                 \
  template void launch_cone_back_adj<T>(const GeomDev &, const ConeTab<T> &, const ViewTab<T> &, const T *,   \
                                        Col<T>, const Epi<T> &, const int *, hipStream_t);                    \
  template void launch_cone_back<T>(const GeomDev &, const ViewTab<T> &, const T *, T *, const Epi<T> &,      \
                                    const int *, hipStream_t);                                                \
  template void launch_cone_fwd_adj<T>(const GeomDev &, const ConeTab<T> &, const ViewTab<T> &, const T *,    \
                                       T *, const Epi<T> &, const int *, hipStream_t);
GKB_INST(float)
GKB_INST(double)
#undef GKB_INST

}  // namespace gkb
