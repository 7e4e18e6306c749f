// 2D projector kernels for gfx950: Joseph forward A and its exact adjoint
// A^T, pixel-driven linear-interpolation back projector B and its exact
// adjoint B^T, for parallel-beam and curved equiangular fan-beam geometry.
//
// Operator definitions: the forward model A x ~= b with an unmatched back
// projector B != A^T (Sec. 1, eq. (1)); A^T and B^T are the transposes the
// AB-/BA-GKB recurrences apply (Algs. "AB-GKB", "BA-GKB").
//
// Mapping:
//  * ray-driven kernels (A, B^T): one thread per ray (view, bin), bins of a
//    view on consecutive lanes; the loop runs over the lines of the ray's
//    dominant image axis.  Row-stepping rays read the image row-major,
//    column-stepping rays read a transposed copy, so the taps of a wavefront
//    stay within a few cache lines of one image line.
//  * pixel-driven kernels (B, A^T): one thread per pixel, 32x8 pixel tiles
//    per 256-thread workgroup, loop over views; per-view constants are
//    uniform across the workgroup (scalar loads).
//  * gathers only: every output element is written by one thread, the sum
//    order is fixed, results are bitwise reproducible.
//  * epilogue: out = raw * in_scale + coef * prev, optional copy of raw, and
//    a deterministic FP64 reduction of ||out||^2 (last-arriving workgroup
//    finalises).

#include "internal.h"
#include "reduce.h"

namespace gkb {

namespace {

template <typename T>
__device__ inline T load_or_zero(const T *line, int i, int len) {
  const int ic = min(max(i, 0), len - 1);
  const T v = line[ic];
  return ((unsigned)i < (unsigned)len) ? v : T(0);
}

// atan of the small angle between a ray and the direction to a pixel
// (|z| <= tan of one bin pitch).  float: the series z - z^3/3 + z^5/5, whose
// relative error z^6/7 stays below float rounding for |z| < 0.05; double:
// the library atan.
__device__ inline float small_atan(float z) {
  const float z2 = z * z;
  return z * fmaf(z2, fmaf(z2, 0.2f, -1.0f / 3.0f), 1.0f);
}
__device__ inline double small_atan(double z) { return atan(z); }

// Epilogue shared by all projector kernels.  Every thread of the block calls
// it (the norm reduction needs the whole block).
template <typename T>
__device__ inline void epilogue(const Epi<T> &e, long long idx, bool valid, T raw, T *outp) {
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
  }
  if (e.norm_to_t) {
    const double v = valid ? (double)outT * (double)outT : 0.0;
    const double bs = block_sum<kBlock>(v, red);
    const unsigned nb = gridDim.x;
    if (threadIdx.x == 0) e.partials[blockIdx.x] = bs;
    if (arrive_last(e.counter, nb)) {
      double acc = 0.0;
      for (unsigned b = threadIdx.x; b < nb; b += kBlock) acc += e.partials[b];
      const double tot = block_sum<kBlock>(acc, red);
      if (threadIdx.x == 0) {
        e.ctl.t[k + 1] = sqrt(tot);
        *e.counter = 0u;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// ray-driven: A (Joseph forward)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd(GeomDev g, RayTab<T> rt, Col<const T> xc,
                                                const T *__restrict__ xT, Col<T> yc, Epi<T> e,
                                                const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ x = xc.get();
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = r < g.m;
  T acc = T(0);
  if (valid) {
    const int meta = rt.meta[r];
    const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
    const bool rowdom = (meta >> 30) & 1;
    const T base = rt.base[r], slope = rt.slope[r];
    const T *img = rowdom ? x : xT;
    const int len = rowdom ? g.nx : g.ny;
    const T mid = rowdom ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
    for (int j = lo; j <= hi; ++j) {
      const T c = fma(T(j) - mid, slope, base);
      const T fl = floor(c);
      const int i0 = (int)fl;
      const T f = c - fl;
      const T *line = img + (long long)j * len;
      const T v0 = load_or_zero(line, i0, len);
      const T v1 = load_or_zero(line, i0 + 1, len);
      acc += fma(f, v1 - v0, v0);
    }
    acc *= rt.w[r];
  }
  epilogue(e, r, valid, acc, yc.get());
}

// ---------------------------------------------------------------------------
// ray-driven: B^T (transpose of the pixel-driven back projector)
// Ray (v,k) collects every pixel whose detector coordinate is within one bin
// of k, with the hat weight 1 - |u(p) - k|.  On each line the candidates lie
// within h of the ray's crossing.
// ---------------------------------------------------------------------------
template <typename T, bool FAN>
__global__ __launch_bounds__(kBlock) void k_back_adj(GeomDev g, RayTab<T> rt, Col<const T> xc,
                                                     const T *__restrict__ xT, Col<T> yc, Epi<T> e,
                                                     const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ x = xc.get();
  const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = r < g.m;
  T acc = T(0);
  if (valid) {
    const int meta = rt.meta[r];
    const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
    const bool rowdom = (meta >> 30) & 1;
    const T base = rt.base[r], slope = rt.slope[r];
    const T h = rt.h[r];
    const T *img = rowdom ? x : xT;
    const int len = rowdom ? g.nx : g.ny;
    const T mid = rowdom ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
    if (!FAN) {
      const T inv_h = T(1) / h;
      for (int j = lo; j <= hi; ++j) {
        const T c = fma(T(j) - mid, slope, base);
        const int ilo = (int)ceil(c - h), ihi = (int)floor(c + h);
        const T *line = img + (long long)j * len;
        for (int i = ilo; i <= ihi; ++i) {
          const T wt = T(1) - fabs(c - T(i)) * inv_h;
          const T v = load_or_zero(line, i, len);
          acc += (wt > T(0)) ? wt * v : T(0);
        }
      }
    } else {
      const T t0 = rt.t0[r], dt = rt.dt[r], dperp = rt.dperp[r], dpar = rt.dpar[r];
      const T inv_dg = T(g.inv_du);
      for (int j = lo; j <= hi; ++j) {
        const T c = fma(T(j) - mid, slope, base);
        const T along0 = fma(T(j) - mid, dt, t0);
        const int ilo = (int)ceil(c - h), ihi = (int)floor(c + h);
        const T *line = img + (long long)j * len;
        for (int i = ilo; i <= ihi; ++i) {
          const T d = T(i) - c;
          const T z = (dperp * d) / fma(dpar, d, along0);
          const T wt = T(1) - fabs(small_atan(z)) * inv_dg;
          const T v = load_or_zero(line, i, len);
          acc += (wt > T(0)) ? wt * v : T(0);
        }
      }
    }
  }
  epilogue(e, r, valid, acc, yc.get());
}

// ---------------------------------------------------------------------------
// pixel-driven: B (back projection by linear interpolation on the detector)
// ---------------------------------------------------------------------------
__device__ inline void tile_pixel(const GeomDev &g, int &i, int &j) {
  const int tiles_x = (g.nx + 31) >> 5;
  const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
  i = tx * 32 + (threadIdx.x & 31);
  j = ty * 8 + (threadIdx.x >> 5);
}

template <typename T, bool FAN>
__global__ __launch_bounds__(kBlock) void k_back(GeomDev g, ViewTab<T> vt, Col<const T> yc, T *__restrict__ xo,
                                                 Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  int i, j;
  tile_pixel(g, i, j);
  const bool valid = i < g.nx && j < g.ny;
  const T *__restrict__ y = yc.get();
  T acc = T(0);
  if (valid) {
    const T px = T(i) - T(0.5) * T(g.nx - 1);
    const T py = T(j) - T(0.5) * T(g.ny - 1);
    const T off = T(g.off);
    const int nu = g.nu;
    if (!FAN) {
      for (int v = 0; v < g.nv; ++v) {
        const T u = fma(px, vt.p0[v], fma(py, vt.p1[v], off));
        const T fl = floor(u);
        const int k0 = (int)fl;
        const T f = u - fl;
        const T *row = y + (long long)v * nu;
        const T y0 = load_or_zero(row, k0, nu);
        const T y1 = load_or_zero(row, k0 + 1, nu);
        acc += fma(f, y1 - y0, y0);
      }
    } else {
      const T D = T(g.D), inv_dg = T(g.inv_du);
      for (int v = 0; v < g.nv; ++v) {
        const T cb = vt.p0[v], sb = vt.p1[v];
        const T a = D - fma(px, cb, py * sb);
        const T bb = fma(px, sb, -py * cb);
        const T u = fma(atan2(bb, a), inv_dg, off);
        const T fl = floor(u);
        const int k0 = (int)fl;
        const T f = u - fl;
        const T *row = y + (long long)v * nu;
        const T y0 = load_or_zero(row, k0, nu);
        const T y1 = load_or_zero(row, k0 + 1, nu);
        acc += fma(f, y1 - y0, y0);
      }
    }
  }
  epilogue(e, valid ? (long long)j * g.nx + i : 0, valid, acc, xo);
}

// ---------------------------------------------------------------------------
// pixel-driven: A^T (exact adjoint of Joseph's projector)
// A ray with unit direction d passing at signed perpendicular distance delta
// from pixel p gives p the Joseph weight max(0, 1 - |delta|/|d_dom|)/|d_dom|.
// Parallel beam: delta = (s_k - s(p)), so the candidates are the bins within
// |d_dom|/du of u(p).  Fan beam: delta = b cos(g_k) - a sin(g_k) with (a, b)
// the coordinates of p - S along and across the central ray; the candidates
// are the bins within asin(1/|p - S|) of the pixel's fan angle.
// ---------------------------------------------------------------------------
template <typename T, bool FAN>
__global__ __launch_bounds__(kBlock) void k_fwd_adj(GeomDev g, ViewTab<T> vt, RayTab<T> rt, Col<const T> yc,
                                                    T *__restrict__ xo, Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  int i, j;
  tile_pixel(g, i, j);
  const bool valid = i < g.nx && j < g.ny;
  const T *__restrict__ y = yc.get();
  T acc = T(0);
  if (valid) {
    const T px = T(i) - T(0.5) * T(g.nx - 1);
    const T py = T(j) - T(0.5) * T(g.ny - 1);
    const T off = T(g.off);
    const int nu = g.nu;
    if (!FAN) {
      for (int v = 0; v < g.nv; ++v) {
        const T u = fma(px, vt.p0[v], fma(py, vt.p1[v], off));
        const T w = vt.p2[v], slope = vt.p3[v], h = vt.p4[v];
        const int klo = max((int)ceil(u - h), 0), khi = min((int)floor(u + h), nu - 1);
        const T *row = y + (long long)v * nu;
        for (int k = klo; k <= khi; ++k) {
          const T wt = T(1) - fabs(u - T(k)) * slope;
          acc += (wt > T(0)) ? w * wt * row[k] : T(0);
        }
      }
    } else {
      const T D = T(g.D), inv_dg = T(g.inv_du), hfac = T(g.hmax_fan);
      for (int v = 0; v < g.nv; ++v) {
        const T cb = vt.p0[v], sb = vt.p1[v];
        const T a = D - fma(px, cb, py * sb);
        const T bb = fma(px, sb, -py * cb);
        const T up = fma(atan2(bb, a), inv_dg, off);
        // candidates: |g_k - g_p| < asin(1/|p-S|) <= z/sqrt(1-z^2), z = 1/|p-S|
        const T z = rsqrt(fma(a, a, bb * bb));
        const T h = hfac * z * rsqrt(T(1) - z * z) + T(1e-3);
        const int klo = max((int)ceil(up - h), 0), khi = min((int)floor(up + h), nu - 1);
        const T *row = y + (long long)v * nu;
        const T *wv = rt.w + (long long)v * nu;
        for (int k = klo; k <= khi; ++k) {
          const T delta = fma(bb, vt.gcos[k], -a * vt.gsin[k]);
          const T w = wv[k];
          const T wt = T(1) - fabs(delta) * w;
          acc += (wt > T(0)) ? w * wt * row[k] : T(0);
        }
      }
    }
  }
  epilogue(e, valid ? (long long)j * g.nx + i : 0, valid, acc, xo);
}

// ---------------------------------------------------------------------------
// transpose (32x32 LDS tiles) for column-stepping rays
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(Col<const T> xc, T *__restrict__ xT, int nx, int ny,
                                                   const int *stop) {
  if (stop && *stop) return;
  const T *__restrict__ x = xc.get();
  __shared__ T tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + tx, j = by + r;
    if (i < nx && j < ny) tile[r][tx] = x[(long long)j * nx + i];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = by + tx, i = bx + r;
    if (i < nx && j < ny) xT[(long long)i * ny + j] = tile[tx][r];
  }
}

}  // namespace

int pixel_blocks(const GeomDev &g) { return ((g.nx + 31) / 32) * ((g.ny + 7) / 8); }
int ray_blocks(const GeomDev &g) { return (int)((g.m + kBlock - 1) / kBlock); }

template <typename T>
void launch_transpose(Col<const T> x, T *xT, int nx, int ny, const int *stop, hipStream_t s) {
  dim3 grid((nx + 31) / 32, (ny + 31) / 32);
  hipLaunchKernelGGL(k_transpose<T>, grid, dim3(256), 0, s, x, xT, nx, ny, stop);
}

template <typename T>
void launch_fwd(const GeomDev &g, const RayTab<T> &rt, Col<const T> x, const T *xT, Col<T> y, const Epi<T> &e,
                const int *stop, hipStream_t s) {
  hipLaunchKernelGGL(k_fwd<T>, dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, rt, x, xT, y, e, stop);
}

template <typename T>
void launch_back_adj(const GeomDev &g, const RayTab<T> &rt, Col<const T> x, const T *xT, Col<T> y,
                     const Epi<T> &e, const int *stop, hipStream_t s) {
  if (g.kind == 1)
    hipLaunchKernelGGL((k_back_adj<T, true>), dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, rt, x, xT, y, e, stop);
  else
    hipLaunchKernelGGL((k_back_adj<T, false>), dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, rt, x, xT, y, e, stop);
}

template <typename T>
void launch_back(const GeomDev &g, const ViewTab<T> &vt, const RayTab<T> &rt, Col<const T> y, T *x,
                 const Epi<T> &e, const int *stop, hipStream_t s) {
  (void)rt;
  if (g.kind == 1)
    hipLaunchKernelGGL((k_back<T, true>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, y, x, e, stop);
  else
    hipLaunchKernelGGL((k_back<T, false>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, y, x, e, stop);
}

template <typename T>
void launch_fwd_adj(const GeomDev &g, const ViewTab<T> &vt, const RayTab<T> &rt, Col<const T> y, T *x,
                    const Epi<T> &e, const int *stop, hipStream_t s) {
  if (g.kind == 1)
    hipLaunchKernelGGL((k_fwd_adj<T, true>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, rt, y, x, e, stop);
  else
    hipLaunchKernelGGL((k_fwd_adj<T, false>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, rt, y, x, e, stop);
}

#define GKB_INST(T)                                                                                             \
  template void launch_transpose<T>(Col<const T>, T *, int, int, const int *, hipStream_t);                   \
  template void launch_fwd<T>(const GeomDev &, const RayTab<T> &, Col<const T>, const T *, Col<T>,              \
                              const Epi<T> &, const int *, hipStream_t);                                       \
  template void launch_back_adj<T>(const GeomDev &, const RayTab<T> &, Col<const T>, const T *, Col<T>,         \
                                   const Epi<T> &, const int *, hipStream_t);                                  \
  template void launch_back<T>(const GeomDev &, const ViewTab<T> &, const RayTab<T> &, Col<const T>, T *,       \
                               const Epi<T> &, const int *, hipStream_t);                                      \
  template void launch_fwd_adj<T>(const GeomDev &, const ViewTab<T> &, const RayTab<T> &, Col<const T>, T *,    \
                                  const Epi<T> &, const int *, hipStream_t);
GKB_INST(float)
GKB_INST(double)
#undef GKB_INST

}  // namespace gkb
