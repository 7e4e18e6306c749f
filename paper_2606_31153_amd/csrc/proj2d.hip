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
//    dominant image axis.  They read a zero-padded copy of the image that
//    holds both a row-major and a column-major layout, so row-stepping and
//    column-stepping rays both read along one padded line, every tap is in
//    bounds without a test, and the two taps of a crossing are one 8-byte
//    load addressed by a 32-bit offset from a uniform base.
//  * pixel-driven kernels (B, A^T): a 256-thread workgroup per 32x2 pixel
//    tile, four threads per pixel (views of one residue mod 4 each, summed
//    through LDS), each looping over its views; per-view constants are
//    uniform across a wavefront (scalar loads).  They read a zero-padded
//    copy of the sinogram; the detector coordinate is clamped into the padded
//    range (taps outside the detector read zeros).
//  * gathers only: every output element is written by one thread, the sum
//    order is fixed, results are bitwise reproducible.
//  * epilogue: out = raw * in_scale + coef * prev, optional copy of raw, and
//    a deterministic FP64 reduction of ||out||^2 (last-arriving workgroup
//    finalises).

#include <algorithm>

#include "batch.h"
#include "devmath.h"
#include "epilogue.h"
#include "internal.h"
#include "reduce.h"

namespace gkb {

namespace {

// atan of |z| <= 0.5: z * P(z^2), P of degree 5 with P(0) = 1, fitted to the
// relative error of atan by Lawson's iteratively reweighted least squares on
// Chebyshev nodes, its coefficients rounded to float one at a time with the
// higher ones refitted (fit_angle_poly.py beside this file).  With the
// coefficients as printed the relative error is at most 5.4e-9 in exact
// arithmetic, below float rounding.
__device__ inline float atan_poly(float z) {
  const float t = z * z;
  float p = -0.05125048f;
  p = fmaf(p, t, 0.10155799f);
  p = fmaf(p, t, -0.14174211f);
  p = fmaf(p, t, 0.19994168f);
  p = fmaf(p, t, -0.33333233f);
  p = fmaf(p, t, 1.0f);
  return z * p;
}

// atan_poly with P's coefficients times a scale: eval(z, off) = off +
// scale * atan(z) with one multiply fewer than fma(atan_poly(z), scale, off).
struct AtanScaled {
  float c[6];
  __device__ explicit AtanScaled(float scale) {
    const float q[6] = {1.0f, -0.33333233f, 0.19994168f, -0.14174211f, 0.10155799f, -0.05125048f};
#pragma unroll
    for (int j = 0; j < 6; ++j) c[j] = q[j] * scale;
  }
  __device__ float eval(float z, float off) const {
    const float t = z * z;
    float p = c[5];
#pragma unroll
    for (int j = 4; j >= 0; --j) p = fmaf(p, t, c[j]);
    return fmaf(z, p, off);
  }
};

// The same for asin(s) = s * Q(s^2), |s| <= 1/sqrt(5) (the sine of an angle of
// tangent 0.5): relative error at most 1.1e-9.  The struct holds Q's
// coefficients times a scale, and eval(s, off) = off + scale * asin(s).
struct AsinScaled {
  float c[6];
  __device__ explicit AsinScaled(float scale) {
    const float q[6] = {1.0f, 0.16666691f, 0.074983247f, 0.04501405f, 0.026861863f, 0.036772124f};
#pragma unroll
    for (int j = 0; j < 6; ++j) c[j] = q[j] * scale;
  }
  __device__ float eval(float s, float off) const {
    const float t = s * s;
    float p = c[5];
#pragma unroll
    for (int j = 4; j >= 0; --j) p = fmaf(p, t, c[j]);
    return fmaf(s, p, off);
  }
};

// Fan angle of a pixel from its coordinates (a along, b across the central ray).
template <typename T>
__device__ inline T fan_angle(T bb, T a, bool fast);
template <>
__device__ inline float fan_angle<float>(float bb, float a, bool fast) {
  return fast ? atan_poly(bb * __builtin_amdgcn_rcpf(a)) : atan2f(bb, a);
}
template <>
__device__ inline double fan_angle<double>(double bb, double a, bool) {
  return atan2(bb, a);
}

// atan of the small angle between a ray and the direction to a pixel
// (|z| <= tan of one bin pitch).  float: z - z^3/3 + z^5/5, relative error
// z^6/7 (below float rounding for |z| < 0.05); double: the library atan.
__device__ inline float small_atan(float z) {
  const float z2 = z * z;
  return z * fmaf(z2, fmaf(z2, 0.2f, -1.0f / 3.0f), 1.0f);
}
__device__ inline double small_atan(double z) { return atan(z); }


// ---------------------------------------------------------------------------
// padded copies
// ---------------------------------------------------------------------------
// row-major region: ny lines of ldR = nx + 2P (image row j at line j)
template <typename T>
__device__ inline void pad_rows_body(const T *__restrict__ x, T *__restrict__ pad, int nx, int ny, int P, int ldR,
                                     Blk b) {
  const long long total = (long long)ny * ldR;
  for (long long idx = (long long)b.id * 256 + threadIdx.x; idx < total; idx += (long long)b.n * 256) {
    const int j = (int)(idx / ldR), i = (int)(idx - (long long)j * ldR) - P;
    pad[idx] = ((unsigned)i < (unsigned)nx) ? x[(long long)j * nx + i] : T(0);
  }
}

// column-major region at offset offT: nx lines of ldT = ny + 2P (image column
// i at line i); tile (bx, by) covers padded rows 32 bx.. and columns 32 by..
template <typename T>
__device__ inline void pad_cols_body(const T *__restrict__ x, T *__restrict__ pad, int nx, int ny, int P, int ldT,
                                     long long offT, int bx, int by) {
  __shared__ T tile[32][33];
  const int jp0 = bx * 32, i0 = by * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int j = jp0 + r - P, i = i0 + tx;  // source pixel (i, j)
    tile[r][tx] = ((unsigned)j < (unsigned)ny && i < nx) ? x[(long long)j * nx + i] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = i0 + r, jp = jp0 + tx;
    if (i < nx && jp < ldT) pad[offT + (long long)i * ldT + jp] = tile[tx][r];
  }
}

// sinogram rows padded by PY zeros on both sides: nv lines of ldY = nu + 2 PY
template <typename T>
__device__ inline void pad_sino_body(const T *__restrict__ y, T *__restrict__ pad, int nv, int nu, int PY, int ldY,
                                     Blk b) {
  const long long total = (long long)nv * ldY;
  for (long long idx = (long long)b.id * 256 + threadIdx.x; idx < total; idx += (long long)b.n * 256) {
    const int v = (int)(idx / ldY), k = (int)(idx - (long long)v * ldY) - PY;
    pad[idx] = ((unsigned)k < (unsigned)nu) ? y[(long long)v * nu + k] : T(0);
  }
}

// (w y, w) per padded bin for the fan-beam A^T: w = 1/|d_dom| per ray in padded layout
template <typename T>
__device__ inline void pad_sino_w_body(const T *__restrict__ y, const T *__restrict__ wpad, T *__restrict__ out,
                                       int nv, int nu, int PY, int ldY, Blk b) {
  const long long total = (long long)nv * ldY;
  for (long long idx = (long long)b.id * 256 + threadIdx.x; idx < total; idx += (long long)b.n * 256) {
    const int v = (int)(idx / ldY), k = (int)(idx - (long long)v * ldY) - PY;
    const T yv = ((unsigned)k < (unsigned)nu) ? y[(long long)v * nu + k] : T(0);
    const T w = wpad[idx];
    out[2 * idx] = w * yv;
    out[2 * idx + 1] = w;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_pad_rows(Col<const T> xc, T *__restrict__ pad, int nx, int ny, int P,
                                                  int ldR, const int *stop) {
  if (stop && *stop) return;
  pad_rows_body(xc.get(), pad, nx, ny, P, ldR, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ __launch_bounds__(256) void k_pad_cols(Col<const T> xc, T *__restrict__ pad, int nx, int ny, int P,
                                                  int ldT, long long offT, const int *stop) {
  if (stop && *stop) return;
  pad_cols_body(xc.get(), pad, nx, ny, P, ldT, offT, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(256) void k_pad_sino(Col<const T> yc, T *__restrict__ pad, int nv, int nu, int PY,
                                                  int ldY, const int *stop) {
  if (stop && *stop) return;
  pad_sino_body(yc.get(), pad, nv, nu, PY, ldY, Blk{blockIdx.x, gridDim.x});
}

template <typename T>
__global__ __launch_bounds__(256) void k_pad_sino_w(Col<const T> yc, const T *__restrict__ wpad, T *__restrict__ out,
                                                    int nv, int nu, int PY, int ldY, const int *stop) {
  if (stop && *stop) return;
  pad_sino_w_body(yc.get(), wpad, out, nv, nu, PY, ldY, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// ray-driven: A (Joseph forward)
// ---------------------------------------------------------------------------
// One line's taps of every lane from a segment of the line: each lane loads
// one element of the 64 from s0 (the wavefront's smallest left tap, from its
// first and last lanes, whose crossings bound the others') and the lanes
// exchange them, so the texture path sees one contiguous load instead of 64
// scattered pairs.  Where some lane's pair is not inside the segment (the
// rays spread over more than 63 pixels, or are not ordered) the pair is
// gathered instead; the test is uniform over the wavefront.  The staged form
// below takes whole blocks of lines; this one takes the lines after the last
// block (all of them with the staged form switched off).
__device__ inline float seg_lerp(const float *__restrict__ line, float c, int lane) {
  const float f = floorf(c);
  const int fi = (int)f;
  const int s0 = min(__builtin_amdgcn_readlane(fi, 0), __builtin_amdgcn_readlane(fi, 63));
  const int dl = fi - s0;
  const float v = line[s0 + lane];
  float t0, t1;
  if (__ballot((unsigned)dl > 62u) == 0) {
    t0 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(dl * 4, __builtin_bit_cast(int, v)));
    t1 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(dl * 4 + 4, __builtin_bit_cast(int, v)));
  } else {
    const auto p = load_pair(line + fi);
    t0 = p.x;
    t1 = p.y;
  }
  return fmaf(c - f, t1 - t0, t0);
}

// A for a wavefront of 64 valid rays that all step along the same axis: one
// loop over the lines any of them crosses (a ray's crossings outside its own
// range fall into the zero padding and add nothing), in blocks of
// kFwdStageLines (or eight) lines, then line by line.

// SW: segment width in elements, 64 (fan beam: adjacent rays cross a line
// under a pixel apart) or 128 (parallel beam: up to sqrt(2) pixels apart).
template <int SW>
__device__ inline float fwd_ray_seg(const GeomDev &g, const RayTab<float> &rt, const float *__restrict__ pad,
                                    long long r) {
  static_assert(SW == 64 || SW == 128, "segment width");
  const int meta = rt.meta[r];
  const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
  const bool rowdom = (meta >> 30) & 1;
  // lines any lane crosses; none when every ray misses the image
  const int wlo = wave_min(lo <= hi ? lo : (1 << 20)), whi = wave_max(lo <= hi ? hi : -1);
  if (wlo > whi) return 0.f;
  const float base = rt.base[r], slope = rt.slope[r];
  const int ld = rowdom ? g.ldR : g.ldT;
  const float mid = rowdom ? 0.5f * float(g.ny - 1) : 0.5f * float(g.nx - 1);
  const float *__restrict__ line0 = pad + (rowdom ? 0LL : g.offT) + g.pad;
  const float clo = -1.5f, chi = float(rowdom ? g.nx : g.ny) + 0.5f;
  const int lane = threadIdx.x & 63;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  int j = wlo;
  if constexpr (kFwdSegStage) {
    // kFwdStageLines lines per step.  LPL = SW / 4 lanes load line
    // h * LPS + q' of the step (q' = lane / LPL), four consecutive elements
    // each, so that one 16-byte load per lane covers the SW-element segments
    // of LPS = 64 / LPL lines, into this wavefront's LDS rows; a lane then
    // reads its two taps from the row.  The rays of a wavefront cross every
    // line in the same order (that of their bins, or the reverse), so a
    // segment starts at the crossing of lane 0 or of lane 63, whichever lies
    // first at the middle line; a line where some lane falls outside its
    // segment gathers instead.
    constexpr int LPL = SW / 4, LPS = 64 / LPL, NL = kFwdStageLines;
    static_assert(NL % LPS == 0, "whole loads per step");
    __shared__ __align__(16) float stage[kBlock / 64][NL * SW];
    float *__restrict__ rows = stage[threadIdx.x >> 6];
    const int sub = lane / LPL, e4 = (lane % LPL) * 4;
    // lane masks of the line groups 1 .. LPS - 1 (a branch-free choice of
    // each lane's segment start)
    int msk[LPS];
#pragma unroll
    for (int u = 1; u < LPS; ++u) msk[u] = sub == u ? -1 : 0;
    const float b0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, base), 0));
    const float b63 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, base), 63));
    const int lead = b0 <= b63 ? 0 : 63;
    // element offsets from pad (never negative: a crossing's floor is at
    // least -2 and every line has pad >= 2 leading elements)
    const unsigned lbase = (unsigned)((rowdom ? 0LL : g.offT) + g.pad);
    const unsigned lane_off = (unsigned)(sub * ld + e4);
    float jm = float(j) - mid;  // line coordinate relative to the middle line (exact)
    for (; j <= whi - (NL - 1); j += NL, jm += float(NL)) {
      float c[NL], f[NL];
      int fi[NL], s0[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        c[q] = clampv(fmaf(q == 0 ? jm : jm + float(q), slope, base), clo, chi);
        f[q] = floorf(c[q]);
        fi[q] = (int)f[q];
        s0[q] = __builtin_amdgcn_readlane(fi[q], lead);
      }
      const unsigned rowj = lbase + (unsigned)(j * ld);
      float4 v[NL / LPS];
#pragma unroll
      for (int h = 0; h < NL / LPS; ++h) {
        int s = s0[LPS * h];
#pragma unroll
        for (int u = 1; u < LPS; ++u) s = (msk[u] & s0[LPS * h + u]) | (~msk[u] & s);
        v[h] = *reinterpret_cast<const float4 *>(pad + (rowj + (unsigned)(LPS * h * ld) + lane_off + (unsigned)s));
      }
#pragma unroll
      for (int h = 0; h < NL / LPS; ++h) *reinterpret_cast<float4 *>(rows + (LPS * h + sub) * SW + e4) = v[h];
      __builtin_amdgcn_wave_barrier();
      float sv[NL];
#pragma unroll
      for (int q = 0; q < NL; ++q) {
        const int dl = fi[q] - s0[q];
        float t0, t1;
        if (__ballot((unsigned)dl > unsigned(SW - 2)) == 0) {
          t0 = rows[q * SW + dl];
          t1 = rows[q * SW + dl + 1];
        } else {
          const auto p = load_pair(pad + (rowj + (unsigned)(q * ld) + (unsigned)fi[q]));
          t0 = p.x;
          t1 = p.y;
        }
        sv[q] = fmaf(c[q] - f[q], t1 - t0, t0);
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int q = 0; q < NL; q += 4) {
        a0 += sv[q];
        a1 += sv[q + 1];
        a2 += sv[q + 2];
        a3 += sv[q + 3];
      }
    }
  }
  for (; j <= whi - 7; j += 8) {
    float s[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float c = clampv(fmaf(float(j + q) - mid, slope, base), clo, chi);
      s[q] = seg_lerp(line0 + (long long)(j + q) * ld, c, lane);
    }
    a0 += s[0];
    a1 += s[1];
    a2 += s[2];
    a3 += s[3];
    a0 += s[4];
    a1 += s[5];
    a2 += s[6];
    a3 += s[7];
  }
  for (; j <= whi; ++j) {
    const float c = clampv(fmaf(float(j) - mid, slope, base), clo, chi);
    a0 += seg_lerp(line0 + (long long)j * ld, c, lane);
  }
  return ((a0 + a1) + (a2 + a3)) * rt.w[r];
}

// SW: the segment width the launch was built for (64 fan beam, 128 parallel
// beam); a geometry flagged for the other width takes the per-ray gathers.
template <typename T, int SW>
__device__ inline void fwd_body(const GeomDev &g, const RayTab<T> &rt, const T *__restrict__ pad, T *yo,
                                const Epi<T> &e, Blk b) {
  const unsigned wg = rt.order_fwd ? (unsigned)rt.order_fwd[b.id] : b.id;
  const long long r = (long long)wg * kBlock + threadIdx.x;
  const bool valid = r < g.m;
  T acc = T(0);
  bool seg = false;
  if constexpr (sizeof(T) == 4) {
    if (g.fwd_seg == (SW == 128 ? 2 : 1)) {
      // every lane a ray, all stepping along the same axis
      const bool rd = valid && ((rt.meta[r] >> 30) & 1);
      seg = __ballot(!valid) == 0 && (__ballot(rd) == 0 || __ballot(!rd) == 0);
    }
    if (seg) acc = fwd_ray_seg<SW>(g, rt, pad, r);
  }
  if (valid && !seg) {
    const int meta = rt.meta[r];
    const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
    const bool rowdom = (meta >> 30) & 1;
    const T base = rt.base[r], slope = rt.slope[r];
    const int ld = rowdom ? g.ldR : g.ldT;
    const T mid = rowdom ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
    unsigned off = (rowdom ? 0u : (unsigned)g.offT) + (unsigned)(lo * ld + g.pad);
    T jf = T(lo) - mid;
    // crossings outside [-1, len] only meet the zero padding; the clamp keeps
    // every tap inside the padded line whatever the rounding of c
    const T clo = T(-1.5), chi = T(rowdom ? g.nx : g.ny) + T(0.5);
    T a0 = T(0), a1 = T(0), a2 = T(0), a3 = T(0);
    int j = lo;
    // eight lines per step: the sixteen taps are in flight together
    for (; j + 7 <= hi; j += 8) {
      T c[8], fl[8];
      typename Pair<T>::v2 p[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        c[q] = clampv(fma(jf + T(q), slope, base), clo, chi);
        fl[q] = floor(c[q]);
        p[q] = load_pair(pad + (off + (unsigned)(q * ld) + (unsigned)(int)fl[q]));
      }
      a0 += fma(c[0] - fl[0], p[0].y - p[0].x, p[0].x);
      a1 += fma(c[1] - fl[1], p[1].y - p[1].x, p[1].x);
      a2 += fma(c[2] - fl[2], p[2].y - p[2].x, p[2].x);
      a3 += fma(c[3] - fl[3], p[3].y - p[3].x, p[3].x);
      a0 += fma(c[4] - fl[4], p[4].y - p[4].x, p[4].x);
      a1 += fma(c[5] - fl[5], p[5].y - p[5].x, p[5].x);
      a2 += fma(c[6] - fl[6], p[6].y - p[6].x, p[6].x);
      a3 += fma(c[7] - fl[7], p[7].y - p[7].x, p[7].x);
      jf += T(8);
      off += 8u * (unsigned)ld;
    }
    for (; j + 3 <= hi; j += 4) {
      T c[4], fl[4];
      typename Pair<T>::v2 p[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = clampv(fma(jf + T(q), slope, base), clo, chi);
        fl[q] = floor(c[q]);
        p[q] = load_pair(pad + (off + (unsigned)(q * ld) + (unsigned)(int)fl[q]));
      }
      a0 += fma(c[0] - fl[0], p[0].y - p[0].x, p[0].x);
      a1 += fma(c[1] - fl[1], p[1].y - p[1].x, p[1].x);
      a2 += fma(c[2] - fl[2], p[2].y - p[2].x, p[2].x);
      a3 += fma(c[3] - fl[3], p[3].y - p[3].x, p[3].x);
      jf += T(4);
      off += 4u * (unsigned)ld;
    }
    for (; j <= hi; ++j) {
      const T c0 = clampv(fma(jf, slope, base), clo, chi);
      const T f0l = floor(c0);
      const auto p0 = load_pair(pad + (off + (unsigned)(int)f0l));
      a0 += fma(c0 - f0l, p0.y - p0.x, p0.x);
      jf += T(1);
      off += (unsigned)ld;
    }
    a0 += a1;
    a2 += a3;
    a0 += a2;
    acc = a0 * rt.w[r];
  }
  epilogue(e, r, valid, acc, yo, b);
}

template <typename T, int SW>
__global__ __launch_bounds__(kBlock) void k_fwd(GeomDev g, RayTab<T> rt, const T *__restrict__ pad, Col<T> yc,
                                                Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  fwd_body<T, SW>(g, rt, pad, yc.get(), e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// ray-driven: B^T (transpose of the pixel-driven back projector)
// Ray (v,k) collects every pixel whose detector coordinate is within one bin
// of k, with the hat weight 1 - |u(p) - k|.  On each line those pixels lie
// within the ray's half-width h of its crossing c, so the window of
// floor(2h) + 1 consecutive pixels from ceil(c - h) holds all of them (h
// bounds the half-width on every line of the ray).  The window length is
// taken as the wavefront's maximum, which makes the candidate loop uniform;
// candidates outside the support get a negative weight, clamped to zero.
// ---------------------------------------------------------------------------
// Sum over the lines lo..hi of one ray (half < 0), or over half of them
// (half 0: the first floor(len / 2), half 1: the rest), with n candidates per
// line: n = CNT, or the wave-uniform runtime count `nrt` (at most MAXC) when
// CNT == 0.
// kBtLines lines per step, the taps of all of them loaded before any is
// weighted: 8 for parallel rays, 6 for fan rays (whose kernel would need 110
// instead of 94 VGPRs with 8, four waves per SIMD instead of five).
template <bool FAN>
constexpr int kBtLines = FAN ? 6 : 8;
template <typename T, bool FAN, int CNT, int MAXC>
__device__ inline T back_adj_ray(const GeomDev &g, const RayTab<T> &rt, const T *__restrict__ pad, long long r,
                                 T hr, int nrt, int half) {
  constexpr int NQ = CNT ? CNT : MAXC;
  const int n = CNT ? CNT : nrt;
  const int meta = rt.meta_bt[r];
  int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
  if (half >= 0) {
    const int mdl = lo + max(hi - lo + 1, 0) / 2;
    if (half == 0)
      hi = mdl - 1;
    else
      lo = mdl;
  }
  const bool rowdom = (meta >> 30) & 1;
  const T base = rt.base[r], slope = rt.slope[r];
  const int ld = rowdom ? g.ldR : g.ldT;
  const T mid = rowdom ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
  unsigned off = (rowdom ? 0u : (unsigned)g.offT) + (unsigned)(lo * ld + g.pad);
  T jf = T(lo) - mid;
  // crossings farther than h from the image only meet zero weights; the
  // clamp keeps every candidate inside the padded line
  const T clo = -hr - T(0.5), chi = T((rowdom ? g.nx : g.ny) - 1) + hr + T(0.5);
  T t0 = T(0), dt = T(0), dperp = T(0), dpar = T(0);
  if (FAN) {
    t0 = rt.t0[r];
    dt = rt.dt[r];
    dperp = rt.dperp[r];
    dpar = rt.dpar[r];
  }
  const T inv_h = FAN ? T(0) : T(1) / hr;
  const T inv_dg = T(g.inv_du);
  const T kzr = fabs(dperp) * inv_dg;
  const bool series = sizeof(T) == 4 && g.bt_fast;
  // the line at jfl (padded-line offset offl): offset d0 of the window's
  // first pixel from the crossing, and the window's taps
  auto taps = [&](T jfl, unsigned offl, T &d0, T (&v)[NQ]) {
    const T c = clampv(T(fma(jfl, slope, base)), clo, chi);
    const T i0f = ceil(c - hr);
    d0 = i0f - c;
    const T *p = pad + (offl + (unsigned)(int)i0f);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (q < n) v[q] = p[q];
  };
  auto weigh = [&](T jfl, T d0, const T (&v)[NQ], T &acc) {
    if (!FAN) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        if (q < n) {
          const T wt = fma(-fabs(q == 0 ? d0 : d0 + T(q)), inv_h, T(1));
          acc = fma(hat_clamp(wt), v[q], acc);
        }
      }
    } else {
      const T along0 = fma(jfl, dt, t0);
      if (series) {
        // |angle| / dg = kz |d| (1 - e + e^2) with e = kd d, written as
        // |d| (kz + d (a1 + d a2)): one reciprocal per line
        const T inv0 = fast_rcp(along0);
        const T kd = dpar * inv0, kz = kzr * inv0;
        const T a1 = -kz * kd, a2 = -a1 * kd;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q < n) {
            const T d = q == 0 ? d0 : d0 + T(q);
            const T gq = fma(fma(a2, d, a1), d, kz);
            const T wt = fma(-fabs(d), gq, T(1));
            acc = fma(hat_clamp(wt), v[q], acc);
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          if (q < n) {
            const T d = q == 0 ? d0 : d0 + T(q);
            // tangent of the angle between the ray and the pixel, seen from the source
            const T z = dperp * d * fast_rcp(fma(dpar, d, along0));
            const T wt = T(1) - fabs(small_atan(z)) * inv_dg;
            acc = fma(hat_clamp(wt), v[q], acc);
          }
        }
      }
    }
  };
  T acc = T(0);
  int j = lo;
  constexpr int NL = kBtLines<FAN>;
  for (; j + NL - 1 <= hi; j += NL) {
    T d0[NL], v[NL][NQ];
#pragma unroll
    for (int i = 0; i < NL; ++i) taps(jf + T(i), off + (unsigned)(i * ld), d0[i], v[i]);
#pragma unroll
    for (int i = 0; i < NL; ++i) weigh(jf + T(i), d0[i], v[i], acc);
    jf += T(NL);
    off += (unsigned)(NL * ld);
  }
  for (; j <= hi; ++j) {
    T d0a, va[NQ];
    taps(jf, off, d0a, va);
    weigh(jf, d0a, va, acc);
    jf += T(1);
    off += (unsigned)ld;
  }
  return acc;
}

template <typename T, bool FAN, int NC>
__device__ inline void back_adj_body(const GeomDev &g, const RayTab<T> &rt, const T *__restrict__ pad, T *yo,
                                     const Epi<T> &e, Blk b) {
  // workgroup = 64 consecutive bins of consecutive views, one view per
  // wavefront, so that its wavefronts cross nearly the same image lines.
  // Parallel beam: 4 views of whole rays.  Fan beam: 2 views, each ray split
  // into two halves of its line range (wavefront 2 v + h takes half h of view
  // v's rays): fan rays differ much in length, a workgroup lasts as long as
  // its longest ray, and halving them shortens the launch's tail.
  constexpr int VPW = FAN ? 2 : 4;
  const int tiles_u = (g.nu + 63) >> 6;
  const unsigned wg = rt.order_bt ? (unsigned)rt.order_bt[b.id] : b.id;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int half = FAN ? (wave & 1) : -1, lane = threadIdx.x & 63;
  const int view = (int)(wg / tiles_u) * VPW + (FAN ? wave >> 1 : wave), bin = (int)(wg % tiles_u) * 64 + lane;
  const bool valid = view < g.nv && bin < g.nu;
  const long long r = valid ? (long long)view * g.nu + bin : 0;
  const T hr = valid ? rt.h[r] : T(0);
  // window length: the wavefront's largest floor(2h) + 1.  It is at most the
  // slice's own candidate count (plus one where h rounds up in float), which
  // its padding is sized for; a longer window than a ray needs only adds zero
  // weights.  NC is the largest count of the launch (of all its slices).
  const int cnt = min(wave_max(valid ? (int)floor(T(2) * hr) + 1 : 0), NC);
  T acc = T(0);
  if (valid) {
    // the three largest counts have straight-line code; the generic count
    // guards every tap with a branch
    if (cnt == NC)
      acc = back_adj_ray<T, FAN, NC, NC>(g, rt, pad, r, hr, cnt, half);
    else if (cnt == NC - 1)
      acc = back_adj_ray<T, FAN, NC - 1, NC>(g, rt, pad, r, hr, cnt, half);
    else if (NC > 3 && cnt == NC - 2)
      acc = back_adj_ray<T, FAN, (NC > 3 ? NC - 2 : 0), NC>(g, rt, pad, r, hr, cnt, half);
    else
      acc = back_adj_ray<T, FAN, 0, NC>(g, rt, pad, r, hr, cnt, half);
  }
  bool own = valid;
  if constexpr (FAN) {
    // the halves meet in LDS: first half + second half, in the first half's wavefront
    __shared__ T second[2][64];
    if (half == 1) second[wave >> 1][lane] = acc;
    __syncthreads();
    if (half == 0) acc += second[wave >> 1][lane];
    own = valid && half == 0;
  }
  epilogue(e, own ? r : 0, own, acc, yo, b);
}

template <typename T, bool FAN, int NC>
__global__ __launch_bounds__(kBlock) void k_back_adj(GeomDev g, RayTab<T> rt, const T *__restrict__ pad, Col<T> yc,
                                                     Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  back_adj_body<T, FAN, NC>(g, rt, pad, yc.get(), e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// pixel-driven: B (back projection by linear interpolation on the detector)
// ---------------------------------------------------------------------------
// Pixel of this thread in tile blk, and the thread's view group.  A group is
// a whole number of wavefronts, so the group index, and with it every view
// index, is uniform across a wavefront: it is returned as such, which keeps
// the per-view constants in scalar loads.
__device__ inline int tile_pixel(const GeomDev &g, unsigned blk, int &i, int &j) {
  const int tiles_x = (g.nx + kPixTileX - 1) / kPixTileX;
  const int tx = (int)blk % tiles_x, ty = (int)blk / tiles_x;
  constexpr int tpix = kPixTileX * kPixTileY;
  static_assert(tpix % 64 == 0, "a view group must be whole wavefronts");
  i = tx * kPixTileX + (int)(threadIdx.x % kPixTileX);
  j = ty * kPixTileY + (int)((threadIdx.x % tpix) / kPixTileX);
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / tpix));
}

// Sum of the view groups' partial sums of a pixel, in group order, returned
// to group 0 (other groups get 0).  Every thread of the workgroup calls it.
template <typename T>
__device__ inline T gather_view_groups(T acc) {
  constexpr int tpix = kPixTileX * kPixTileY;
  __shared__ T xch[(kViewGroups - 1) * tpix];
  const int grp = (int)(threadIdx.x / tpix), pix = (int)(threadIdx.x % tpix);
  if (grp > 0) xch[(grp - 1) * tpix + pix] = acc;
  __syncthreads();
  if (grp > 0) return T(0);
#pragma unroll
  for (int q = 1; q < kViewGroups; ++q) acc += xch[(q - 1) * tpix + pix];
  return acc;
}

// Parallel beam: VU = 4 or 8 views per step (the loads of all in flight
// together), summed into four accumulators by view index mod 4, so that both
// choices add the same terms in the same order.
template <typename T, bool FAN, int VU = 4>
__device__ inline void back_body(const GeomDev &g, const ViewTab<T> &vt, const T *__restrict__ ypad, T *xo,
                                 const Epi<T> &e, Blk b) {
  static_assert(VU == 4 || VU == 8, "B: 4 or 8 views per step");
  int i, j;
  const int grp = tile_pixel(g, b.id, i, j);
  const bool valid = i < g.nx && j < g.ny;
  T acc = T(0);
  if (valid) {
    const T px = T(i) - T(0.5) * T(g.nx - 1);
    const T py = T(j) - T(0.5) * T(g.ny - 1);
    const T off = T(g.off);
    const T ulo = T(-2), uhi = T(g.nu + 1);
    // this group's views: grp, grp + VS, ...
    constexpr int VS = kViewGroups;
    const unsigned ldY = (unsigned)g.ldY;
    unsigned roff = (unsigned)g.padY + (unsigned)grp * ldY;
    if (!FAN) {
      T a[4] = {T(0), T(0), T(0), T(0)};
      int v = grp;
      if (VU == 8) {
        for (; v + 7 * VS < g.nv; v += 8 * VS) {
          T u[8], fl[8];
          typename Pair<T>::v2 p[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            u[q] = clampv(fma(px, vt.p0[v + q * VS], fma(py, vt.p1[v + q * VS], off)), ulo, uhi);
            fl[q] = floor(u[q]);
            p[q] = load_pair(ypad + (roff + (unsigned)(q * VS) * ldY + (unsigned)(int)fl[q]));
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) a[q & 3] += fma(u[q] - fl[q], p[q].y - p[q].x, p[q].x);
          roff += (unsigned)(8 * VS) * ldY;
        }
      }
      for (; v + 3 * VS < g.nv; v += 4 * VS) {
        T u[4], fl[4];
        typename Pair<T>::v2 p[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          u[q] = clampv(fma(px, vt.p0[v + q * VS], fma(py, vt.p1[v + q * VS], off)), ulo, uhi);
          fl[q] = floor(u[q]);
          p[q] = load_pair(ypad + (roff + (unsigned)(q * VS) * ldY + (unsigned)(int)fl[q]));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) a[q] += fma(u[q] - fl[q], p[q].y - p[q].x, p[q].x);
        roff += (unsigned)(4 * VS) * ldY;
      }
      for (; v < g.nv; v += VS) {
        const T u0 = clampv(fma(px, vt.p0[v], fma(py, vt.p1[v], off)), ulo, uhi);
        const T f0l = floor(u0);
        const auto p0 = load_pair(ypad + (roff + (unsigned)(int)f0l));
        a[0] += fma(u0 - f0l, p0.y - p0.x, p0.x);
        roff += (unsigned)VS * ldY;
      }
      acc = (a[0] + a[1]) + (a[2] + a[3]);
    } else {
      const T D = T(g.D), inv_dg = T(g.inv_du);
      const bool fast = g.fast_atan != 0;
      const AtanScaled atn((float)inv_dg);
      // the pixel's detector coordinate in view (cb, sb); float with the fast
      // angle: the atan polynomial yields bins directly
      auto u_of = [&](T cb, T sb) -> T {
        if constexpr (sizeof(T) == 4) {
          if (fast) {
            const T a = fma(-px, cb, fma(-py, sb, D));
            const T bb = fma(px, sb, -py * cb);
            return clampv(T(atn.eval(bb * fast_rcp(a), off)), ulo, uhi);
          }
        }
        const T a = D - fma(px, cb, py * sb);
        const T bb = fma(px, sb, -py * cb);
        return clampv(T(fma(fan_angle<T>(bb, a, fast), inv_dg, off)), ulo, uhi);
      };
      T a0 = T(0), a1 = T(0);
      int v = grp;
      for (; v + VS < g.nv; v += 2 * VS) {
        T u[2], fl[2];
        typename Pair<T>::v2 p[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          u[q] = u_of(vt.p0[v + q * VS], vt.p1[v + q * VS]);
          fl[q] = floor(u[q]);
          p[q] = load_pair(ypad + (roff + (unsigned)(q * VS) * ldY + (unsigned)(int)fl[q]));
        }
        a0 += fma(u[0] - fl[0], p[0].y - p[0].x, p[0].x);
        a1 += fma(u[1] - fl[1], p[1].y - p[1].x, p[1].x);
        roff += (unsigned)(2 * VS) * ldY;
      }
      if (v < g.nv) {
        const T u = u_of(vt.p0[v], vt.p1[v]);
        const T fl = floor(u);
        const auto p = load_pair(ypad + (roff + (unsigned)(int)fl));
        a0 += fma(u - fl, p.y - p.x, p.x);
      }
      acc = a0 + a1;
    }
  }
  acc = gather_view_groups(acc);
  const bool own = valid && grp == 0;
  epilogue(e, own ? (long long)j * g.nx + i : 0, own, acc, xo, b);
}

template <typename T, bool FAN, int VU>
__global__ __launch_bounds__(kBlock) void k_back(GeomDev g, ViewTab<T> vt, const T *__restrict__ ypad,
                                                 T *__restrict__ xo, Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  back_body<T, FAN, VU>(g, vt, ypad, xo, e, Blk{blockIdx.x, gridDim.x});
}

// ---------------------------------------------------------------------------
// pixel-driven: A^T (exact adjoint of Joseph's projector)
// A ray with unit direction d passing at signed perpendicular distance delta
// from pixel p gives p the Joseph weight max(0, 1 - |delta|/|d_dom|)/|d_dom|.
// Parallel beam: delta = (s_k - s(p)), so the candidates are the bins within
// |d_dom|/du of u(p).  Fan beam: delta = b cos(g_k) - a sin(g_k) with (a, b)
// the coordinates of p - S along and across the central ray; the candidates
// are the bins within asin(|d_dom|/|p - S|) of the pixel's fan angle, with
// |d_dom| bounded by that of the pixel's own ray plus the fan spread of the
// candidates.
// ---------------------------------------------------------------------------
// Parallel-beam A^T: hat-weighted sum of n consecutive bins from `row`, the
// first at distance d0 (in bins) from the pixel's detector coordinate;
// n = CNT, or the uniform runtime count nrt (at most MAXC) when CNT == 0.
template <typename T, int CNT, int MAXC>
__device__ inline T at_par_bins(const T *__restrict__ row, T d0, T slope, int nrt) {
  constexpr int NQ = CNT ? CNT : MAXC;
  const int n = CNT ? CNT : nrt;
  T yv[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (q < n) yv[q] = row[q];
  T part = T(0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < n) {
      const T wt = fma(-fabs(d0 - T(q)), slope, T(1));
      part = fma(hat_clamp(wt), yv[q], part);
    }
  }
  return part;
}

// Fan-beam A^T in float: sum over n bins of (w y)_k max(0, 1 - |delta_k| w_k)
// with the pairs (w y, w) from yw, the first bin at distance d0 below the
// pixel's coordinate and delta = d (c1 + c3 d^2) for d = u_p - k; n = CNT, or
// the uniform runtime count nrt (at most MAXC) when CNT == 0.
template <typename T, int CNT, int MAXC>
__device__ inline T at_fan_bins(const typename Pair<T>::v2 *__restrict__ yw, T d0, T c1, T c3, int nrt) {
  constexpr int NQ = CNT ? CNT : MAXC;
  const int n = CNT ? CNT : nrt;
  typename Pair<T>::v2 pw[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (q < n) pw[q] = yw[q];
  T part = T(0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < n) {
      const T d = d0 - T(q);
      const T delta = d * fma(c3, d * d, c1);
      const T wt = fma(-fabs(delta), pw[q].y, T(1));
      part = fma(hat_clamp(wt), pw[q].x, part);
    }
  }
  return part;
}

// As at_fan_bins with the first-order sine, delta = c1 d, and the offsets
// scaled by c1: the first bin at distance dc1 = c1 d0.  Adds to acc.
template <typename T, int CNT, int MAXC>
__device__ inline T at_fan_bins_lin(const typename Pair<T>::v2 *__restrict__ yw, T dc1, T c1, int nrt, T acc) {
  constexpr int NQ = CNT ? CNT : MAXC;
  const int n = CNT ? CNT : nrt;
  typename Pair<T>::v2 pw[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
    if (q < n) pw[q] = yw[q];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q < n) {
      const T delta = q == 0 ? dc1 : fma(T(-q), c1, dc1);
      const T wt = fma(-fabs(delta), pw[q].y, T(1));
      acc = fma(hat_clamp(wt), pw[q].x, acc);
    }
  }
  return acc;
}

// Parallel beam: VU views per step.  With VU > 1 every view of a step reads
// the full window of NC bins (the candidates past a view's own floor(2h) + 1
// get zero weight), so that the loads of all VU views are in flight
// together; the terms are added in the same order as with VU = 1.
template <typename T, bool FAN, int NC, int VU = 1>
__device__ inline void fwd_adj_body(const GeomDev &g, const ViewTab<T> &vt, const T *__restrict__ ypad, T *xo,
                                    const Epi<T> &e, Blk b) {
  int i, j;
  const int grp = tile_pixel(g, b.id, i, j);
  const bool valid = i < g.nx && j < g.ny;
  T acc = T(0);
  const T px = T(i) - T(0.5) * T(g.nx - 1);
  const T py = T(j) - T(0.5) * T(g.ny - 1);
  const T off = T(g.off);
  // this group's views: grp, grp + VS, ...
  constexpr int VS = kViewGroups;
  const unsigned ldY = (unsigned)g.ldY;
  unsigned roff = (unsigned)g.padY + (unsigned)grp * ldY;
  // bins farther than the candidate half-width from the detector have zero
  // weight; the clamp keeps every candidate inside the padded row
  const T ulo = -T(g.uclamp_at), uhi = T(g.nu - 1) + T(g.uclamp_at);
  if (!FAN) {
    if (valid) {
      int v = grp;
      if (VU > 1) {
        // a slice's padding is sized for its own candidate count (NC is the
        // launch's largest): the bins past it are not read
        const int ncs = min(g.nc_at, NC);
        for (; v + (VU - 1) * VS < g.nv; v += VU * VS) {
          T d0[VU], yv[VU][NC];
#pragma unroll
          for (int q = 0; q < VU; ++q) {
            const int vq = v + q * VS;
            const T u = clampv(fma(px, vt.p0[vq], fma(py, vt.p1[vq], off)), ulo, uhi);
            const T k0f = ceil(u - vt.p4[vq]);
            d0[q] = u - k0f;
            const T *row = ypad + (roff + (unsigned)(q * VS) * ldY + (unsigned)(int)k0f);
#pragma unroll
            for (int c = 0; c < NC; ++c) yv[q][c] = c < ncs ? row[c] : T(0);
          }
#pragma unroll
          for (int q = 0; q < VU; ++q) {
            const int vq = v + q * VS;
            const T slope = vt.p3[vq];
            T part = T(0);
#pragma unroll
            for (int c = 0; c < NC; ++c) {
              const T wt = fma(-fabs(d0[q] - T(c)), slope, T(1));
              part = fma(hat_clamp(wt), yv[q][c], part);
            }
            acc = fma(vt.p2[vq], part, acc);
          }
          roff += (unsigned)(VU * VS) * ldY;
        }
      }
      for (; v < g.nv; v += VS) {
        T u = fma(px, vt.p0[v], fma(py, vt.p1[v], off));
        u = clampv(u, ulo, uhi);
        const T w = vt.p2[v], slope = vt.p3[v], h = vt.p4[v];
        // the bins within h of u lie in the floor(2h) + 1 bins from ceil(u - h);
        // h is the view's, so the count is uniform
        const int cv = min((int)floor(T(2) * h) + 1, NC);
        const T k0f = ceil(u - h);
        const T d0 = u - k0f;  // offset of u from the first candidate
        const T *row = ypad + (roff + (unsigned)(int)k0f);
        const T part = cv == NC       ? at_par_bins<T, NC, NC>(row, d0, slope, cv)
                       : cv == NC - 1 ? at_par_bins<T, NC - 1, NC>(row, d0, slope, cv)
                                      : at_par_bins<T, 0, NC>(row, d0, slope, cv);
        acc = fma(w, part, acc);
        roff += (unsigned)VS * ldY;
      }
    }
  } else {
    // ypad holds (w y, w) per padded bin, w = 1/|d_dom| of the ray (0 in the
    // pads); vt.gcos holds (cos g_k, sin g_k) per padded bin.  The candidate
    // window of every pixel of the tile is floor(2H) + 1 bins from ceil(u_p - H),
    // H the tile's half-width bound for the view, which a lane of the wavefront
    // holds for 64 of the group's views at a time.  Every lane runs the loop
    // (pixels outside the image too: the clamp keeps their reads inside the
    // padded rows, and their sums are discarded).
    const T D = T(g.D), inv_dg = T(g.inv_du);
    const bool fast = g.fast_atan != 0;
    const int lane = threadIdx.x & 63;
    const T *__restrict__ ht = vt.htile + (long long)b.id * g.nv;
    const int nvg = (g.nv - grp + VS - 1) / VS;  // views of this group
    // float with the fast angle and the first-order sine: the pixel's sine
    // s = b / |p - S| comes from the reciprocal square root that |p - S| needs
    // anyway, and its angle in bins from the scaled asin polynomial
    const bool sine_path = fast && g.at_fast;
    const AsinScaled asn((float)inv_dg);
    for (int t0 = 0; t0 < nvg; t0 += 64) {
      const T hl = (t0 + lane < nvg) ? ht[grp + VS * (t0 + lane)] : T(0);
      const int cl = min((int)floor(T(2) * hl) + 1, NC);  // the candidate count of each lane's view
      const int tend = min(nvg, t0 + 64);
      for (int t = t0; t < tend; ++t) {
        const int v = grp + VS * t;
        const T H = lane_value(hl, t - t0);
        const int cnt = __builtin_amdgcn_readlane(cl, t - t0);
        const T cb = vt.p0[v], sb = vt.p1[v];
        if constexpr (sizeof(T) == 4) {
          if (sine_path) {
            const T a = fma(-px, cb, fma(-py, sb, D));
            const T bb = fma(px, sb, -py * cb);
            const T r2 = fma(a, a, bb * bb);
            const T rs = fast_rsq(r2);
            const T up = clampv(asn.eval(bb * rs, off), ulo, uhi);
            const T k0f = ceil(up - H);
            const T c1 = r2 * rs * T(g.du);
            const T dc1 = (up - k0f) * c1;
            const auto *yw = reinterpret_cast<const typename Pair<T>::v2 *>(ypad) + (roff + (unsigned)(int)k0f);
            acc = cnt == NC       ? at_fan_bins_lin<T, NC, NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 1 ? at_fan_bins_lin<T, NC - 1, NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 2 ? at_fan_bins_lin<T, (NC > 2 ? NC - 2 : 0), NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 3 ? at_fan_bins_lin<T, (NC > 3 ? NC - 3 : 0), NC>(yw, dc1, c1, cnt, acc)
                                  : at_fan_bins_lin<T, 0, NC>(yw, dc1, c1, cnt, acc);
            roff += (unsigned)VS * ldY;
            continue;
          }
        }
        const T a = D - fma(px, cb, py * sb);
        const T bb = fma(px, sb, -py * cb);
        T up = fma(fan_angle<T>(bb, a, fast), inv_dg, off);
        up = clampv(up, ulo, uhi);
        const T k0f = ceil(up - H);
        const unsigned k0 = (unsigned)((int)g.padY + (int)k0f);
        const typename Pair<T>::v2 *yw = reinterpret_cast<const typename Pair<T>::v2 *>(ypad) + (roff - g.padY + k0);
        if constexpr (sizeof(T) == 4) {
          // delta_k = |p - S| sin(g_p - g_k) with g_p - g_k = (up - k) dg; the sine to
          // third order, whose relative truncation error x^4/120 is below 1e-9 for
          // the candidate angles of a fan with D >= 2 N:
          // delta = d (c1 + c3 d^2), c1 = |p - S| dg, c3 = -c1 dg^2 / 6, d = up - k
          const T dg = T(g.du);
          const T r2 = fma(a, a, bb * bb);
          const T c1 = r2 * fast_rsq(r2) * dg;
          const T d0 = up - k0f;
          if (g.at_fast) {
            // sin(x) = x over the window (relative error within 1e-6)
            const T dc1 = d0 * c1;
            acc = cnt == NC       ? at_fan_bins_lin<T, NC, NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 1 ? at_fan_bins_lin<T, NC - 1, NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 2 ? at_fan_bins_lin<T, (NC > 2 ? NC - 2 : 0), NC>(yw, dc1, c1, cnt, acc)
                  : cnt == NC - 3 ? at_fan_bins_lin<T, (NC > 3 ? NC - 3 : 0), NC>(yw, dc1, c1, cnt, acc)
                                  : at_fan_bins_lin<T, 0, NC>(yw, dc1, c1, cnt, acc);
          } else {
            const T c3 = c1 * dg * dg * T(-1.0 / 6.0);
            acc += cnt == NC       ? at_fan_bins<T, NC, NC>(yw, d0, c1, c3, cnt)
                   : cnt == NC - 1 ? at_fan_bins<T, NC - 1, NC>(yw, d0, c1, c3, cnt)
                   : cnt == NC - 2 ? at_fan_bins<T, (NC > 2 ? NC - 2 : 0), NC>(yw, d0, c1, c3, cnt)
                                   : at_fan_bins<T, 0, NC>(yw, d0, c1, c3, cnt);
          }
        } else {
          const typename Pair<T>::v2 *cs = reinterpret_cast<const typename Pair<T>::v2 *>(vt.gcos) + k0;
#pragma unroll
          for (int q = 0; q < NC; ++q) {
            if (q < cnt) {
              const auto gq = cs[q];
              const auto pq = yw[q];
              const T delta = fma(bb, gq.x, -a * gq.y);
              const T wt = fma(-fabs(delta), pq.y, T(1));
              acc = fma(hat_clamp(wt), pq.x, acc);
            }
          }
        }
        roff += (unsigned)VS * ldY;
      }
    }
    if (!valid) acc = T(0);
  }
  acc = gather_view_groups(acc);
  const bool own = valid && grp == 0;
  epilogue(e, own ? (long long)j * g.nx + i : 0, own, acc, xo, b);
}

template <typename T, bool FAN, int NC, int VU>
__global__ __launch_bounds__(kBlock) void k_fwd_adj(GeomDev g, ViewTab<T> vt, const T *__restrict__ ypad,
                                                    T *__restrict__ xo, Epi<T> e, const int *stop) {
  if (stop && *stop) return;
  fwd_adj_body<T, FAN, NC, VU>(g, vt, ypad, xo, e, Blk{blockIdx.x, gridDim.x});
}


// ---------------------------------------------------------------------------
// batched launches: every active slice of a batch in one grid; workgroup ->
// (slice, local workgroup) by a search over the per-slice prefix sums, then
// the same bodies as the single-slice kernels
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline Epi<T> make_epi(const SliceDev<T> &d, const EpiCfg &ec, int k) {
  Epi<T> e{};
  e.ctl = d.ctl;
  e.use_ctl = 1;
  e.in_sel = ec.in_sel;
  e.prev_sel = ec.prev_sel;
  e.norm_to_t = ec.norm_to_t;
  e.prev = Col<const T>{resolve(d, ec.prev_buf, k), 0, 0, nullptr};
  e.out_raw = Col<T>{resolve(d, ec.out_raw_buf, k), 0, 0, nullptr};
  e.partials = d.partials;
  return e;
}

template <typename T>
__global__ __launch_bounds__(256) void kb_pad_rows(BatchDev<T> bd, int in_sel) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_PADR, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  pad_rows_body(resolve(d, in_sel, k), d.xpad, d.g.nx, d.g.ny, d.g.pad, d.g.ldR, b);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_pad_cols(BatchDev<T> bd, int in_sel) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_PADC, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const int tiles_x = (d.g.ldT + 31) / 32;
  pad_cols_body(resolve(d, in_sel, k), d.xpad, d.g.nx, d.g.ny, d.g.pad, d.g.ldT, d.g.offT, (int)b.id % tiles_x,
                (int)b.id / tiles_x);
}

template <typename T>
__global__ __launch_bounds__(256) void kb_pad_sino(BatchDev<T> bd, int in_sel, int adj) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_PADS, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const T *y = resolve(d, in_sel, k);
  if (adj && d.g.kind == 1)
    pad_sino_w_body(y, d.rt.wpad, d.ypad, d.g.nv, d.g.nu, d.g.padY, d.g.ldY, b);
  else
    pad_sino_body(y, d.ypad, d.g.nv, d.g.nu, d.g.padY, d.g.ldY, b);
}

template <typename T, int SW>
__global__ __launch_bounds__(kBlock) void kb_fwd(BatchDev<T> bd, int out_sel, EpiCfg ec) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_RAY, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const GeomDev g = d.g;
  const RayTab<T> rt = d.rt;
  fwd_body<T, SW>(g, rt, d.xpad, resolve(d, out_sel, k), make_epi(d, ec, k), b);
}

template <typename T, bool FAN, int NC>
__global__ __launch_bounds__(kBlock) void kb_back_adj(BatchDev<T> bd, int out_sel, EpiCfg ec) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_RAYBT, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const GeomDev g = d.g;
  const RayTab<T> rt = d.rt;
  back_adj_body<T, FAN, NC>(g, rt, d.xpad, resolve(d, out_sel, k), make_epi(d, ec, k), b);
}

template <typename T, bool FAN, int VU>
__global__ __launch_bounds__(kBlock) void kb_back(BatchDev<T> bd, int out_sel, EpiCfg ec) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_PIX, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const GeomDev g = d.g;
  const ViewTab<T> vt = d.vt;
  back_body<T, FAN, VU>(g, vt, d.ypad, resolve(d, out_sel, k), make_epi(d, ec, k), b);
}

template <typename T, bool FAN, int NC, int VU>
__global__ __launch_bounds__(kBlock) void kb_fwd_adj(BatchDev<T> bd, int out_sel, EpiCfg ec) {
  Blk b;
  const SliceDev<T> &d = slice_of(bd, BF_PIX, blockIdx.x, b);
  if (skip(bd, d)) return;
  const int k = d.ctl.ip[CI_K];
  const GeomDev g = d.g;
  const ViewTab<T> vt = d.vt;
  fwd_adj_body<T, FAN, NC, VU>(g, vt, d.ypad, resolve(d, out_sel, k), make_epi(d, ec, k), b);
}

}  // namespace

int pixel_blocks(const GeomDev &g) {
  if (g.kind == 2) return ((g.nx + 31) / 32) * ((g.ny + 7) / 8) * g.nz;
  return ((g.nx + kPixTileX - 1) / kPixTileX) * ((g.ny + kPixTileY - 1) / kPixTileY);
}
// Grid of the ray-driven kernels: B^T takes workgroups of 64 bins x 4 views,
// A the same count of workgroups over consecutive rays (256 per workgroup;
// the grid covers at least ceil(m / 256), surplus workgroups have no valid ray).
int ray_blocks(const GeomDev &g) {
  if (g.kind == 2) return (int)((g.m + kBlock - 1) / kBlock);
  return ((g.nu + 63) / 64) * ((g.nv + 3) / 4);
}
int bt_blocks(const GeomDev &g) {
  if (g.kind != 1) return ray_blocks(g);  // parallel beam: 4 views of whole rays; cone: its own layout
  return ((g.nu + 63) / 64) * ((g.nv + 1) / 2);
}

template <typename T>
void launch_pad_image(const GeomDev &g, Col<const T> x, T *pad, bool cols, const int *stop, hipStream_t s) {
  const long long totR = (long long)g.ny * g.ldR;
  const int nbR = (int)std::min<long long>((totR + 255) / 256, 2048);
  hipLaunchKernelGGL(k_pad_rows<T>, dim3(nbR), dim3(256), 0, s, x, pad, g.nx, g.ny, g.pad, g.ldR, stop);
  if (cols) {
    dim3 grid((g.ldT + 31) / 32, (g.nx + 31) / 32);
    hipLaunchKernelGGL(k_pad_cols<T>, grid, dim3(256), 0, s, x, pad, g.nx, g.ny, g.pad, g.ldT, g.offT, stop);
  }
}

template <typename T>
void launch_pad_sino(const GeomDev &g, Col<const T> y, T *pad, const int *stop, hipStream_t s) {
  const long long tot = (long long)g.nv * g.ldY;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_sino<T>, dim3(nb), dim3(256), 0, s, y, pad, g.nv, g.nu, g.padY, g.ldY, stop);
}

template <typename T>
void launch_pad_sino_adj(const GeomDev &g, const RayTab<T> &rt, Col<const T> y, T *pad, const int *stop,
                         hipStream_t s) {
  if (g.kind != 1) {
    launch_pad_sino<T>(g, y, pad, stop, s);
    return;
  }
  const long long tot = (long long)g.nv * g.ldY;
  const int nb = (int)std::min<long long>((tot + 255) / 256, 4096);
  hipLaunchKernelGGL(k_pad_sino_w<T>, dim3(nb), dim3(256), 0, s, y, rt.wpad, pad, g.nv, g.nu, g.padY, g.ldY, stop);
}

template <typename T>
void launch_fwd(const GeomDev &g, const RayTab<T> &rt, const T *pad, Col<T> y, const Epi<T> &e, const int *stop,
                hipStream_t s) {
  if (g.fwd_seg == 2)
    hipLaunchKernelGGL((k_fwd<T, 128>), dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, rt, pad, y, e, stop);
  else
    hipLaunchKernelGGL((k_fwd<T, 64>), dim3(ray_blocks(g)), dim3(kBlock), 0, s, g, rt, pad, y, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, ray_blocks(g), NORM_T1, stop, s);
}

template <typename T, bool FAN>
static void back_adj_nc(const GeomDev &g, const RayTab<T> &rt, const T *pad, Col<T> y, const Epi<T> &e,
                        const int *stop, hipStream_t s) {
  const dim3 grid(bt_blocks(g)), blk(kBlock);
  switch (g.nc_bt) {
    case 2: hipLaunchKernelGGL((k_back_adj<T, FAN, 2>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    case 3: hipLaunchKernelGGL((k_back_adj<T, FAN, 3>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    case 4: hipLaunchKernelGGL((k_back_adj<T, FAN, 4>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    case 5: hipLaunchKernelGGL((k_back_adj<T, FAN, 5>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    case 6: hipLaunchKernelGGL((k_back_adj<T, FAN, 6>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    case 7: hipLaunchKernelGGL((k_back_adj<T, FAN, 7>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
    default: hipLaunchKernelGGL((k_back_adj<T, FAN, 8>), grid, blk, 0, s, g, rt, pad, y, e, stop); break;
  }
}

template <typename T>
void launch_back_adj(const GeomDev &g, const RayTab<T> &rt, const T *pad, Col<T> y, const Epi<T> &e,
                     const int *stop, hipStream_t s) {
  if (g.kind == 1)
    back_adj_nc<T, true>(g, rt, pad, y, e, stop, s);
  else
    back_adj_nc<T, false>(g, rt, pad, y, e, stop, s);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, bt_blocks(g), NORM_T1, stop, s);
}

template <typename T>
void launch_back(const GeomDev &g, const ViewTab<T> &vt, const T *ypad, T *x, const Epi<T> &e, const int *stop,
                 hipStream_t s) {
  if (g.kind == 1)
    hipLaunchKernelGGL((k_back<T, true, 4>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, ypad, x, e, stop);
  else if (g.b_vu == 8)
    hipLaunchKernelGGL((k_back<T, false, 8>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, ypad, x, e, stop);
  else
    hipLaunchKernelGGL((k_back<T, false, 4>), dim3(pixel_blocks(g)), dim3(kBlock), 0, s, g, vt, ypad, x, e, stop);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, pixel_blocks(g), NORM_T1, stop, s);
}

// views per step of the parallel-beam A^T actually launched: the tuned count
// for windows of up to four bins, one view otherwise
__host__ inline int at_views(int nc, int tuned) { return nc <= 4 ? tuned : 1; }

template <typename T, bool FAN>
static void fwd_adj_nc(const GeomDev &g, const ViewTab<T> &vt, const RayTab<T> &rt, const T *ypad, T *x,
                       const Epi<T> &e, const int *stop, hipStream_t s) {
  const dim3 grid(pixel_blocks(g)), blk(kBlock);
  const int vu = FAN ? 1 : at_views(g.nc_at, g.at_vu);
#define GKB_AT(NC, VU) hipLaunchKernelGGL((k_fwd_adj<T, FAN, NC, VU>), grid, blk, 0, s, g, vt, ypad, x, e, stop)
  switch (g.nc_at) {
    case 2:
      if (vu == 4) GKB_AT(2, 4);
      else if (vu == 2) GKB_AT(2, 2);
      else GKB_AT(2, 1);
      break;
    case 3:
      if (vu == 4) GKB_AT(3, 4);
      else if (vu == 2) GKB_AT(3, 2);
      else GKB_AT(3, 1);
      break;
    case 4:
      if (vu == 4) GKB_AT(4, 4);
      else if (vu == 2) GKB_AT(4, 2);
      else GKB_AT(4, 1);
      break;
    case 5: GKB_AT(5, 1); break;
    case 6: GKB_AT(6, 1); break;
    case 7: GKB_AT(7, 1); break;
    default: GKB_AT(8, 1); break;
  }
#undef GKB_AT
}

template <typename T>
void launch_fwd_adj(const GeomDev &g, const ViewTab<T> &vt, const RayTab<T> &rt, const T *ypad, T *x,
                    const Epi<T> &e, const int *stop, hipStream_t s) {
  if (g.kind == 1)
    fwd_adj_nc<T, true>(g, vt, rt, ypad, x, e, stop, s);
  else
    fwd_adj_nc<T, false>(g, vt, rt, ypad, x, e, stop, s);
  if (e.norm_to_t) launch_norm_finalize(e.ctl, e.partials, pixel_blocks(g), NORM_T1, stop, s);
}

// ---- batched launchers ----
template <typename T>
void launch_b_pad_image(const BatchDev<T> &bd, const BatchLaunch &bl, int in_sel, hipStream_t s) {
  if (bl.tot[BF_PADR] > 0)
    hipLaunchKernelGGL(kb_pad_rows<T>, dim3(bl.tot[BF_PADR]), dim3(256), 0, s, bd, in_sel);
  if (bl.tot[BF_PADC] > 0)
    hipLaunchKernelGGL(kb_pad_cols<T>, dim3(bl.tot[BF_PADC]), dim3(256), 0, s, bd, in_sel);
}

template <typename T>
void launch_b_pad_sino(const BatchDev<T> &bd, const BatchLaunch &bl, int in_sel, int adj, hipStream_t s) {
  if (bl.tot[BF_PADS] > 0)
    hipLaunchKernelGGL(kb_pad_sino<T>, dim3(bl.tot[BF_PADS]), dim3(256), 0, s, bd, in_sel, adj);
}

template <typename T>
void launch_b_fwd(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  if (bl.tot[BF_RAY] <= 0) return;
  if (bl.fan)
    hipLaunchKernelGGL((kb_fwd<T, 64>), dim3(bl.tot[BF_RAY]), dim3(kBlock), 0, s, bd, out_sel, ec);
  else
    hipLaunchKernelGGL((kb_fwd<T, 128>), dim3(bl.tot[BF_RAY]), dim3(kBlock), 0, s, bd, out_sel, ec);
  if (ec.norm_to_t) launch_b_norm_finalize(bd, bl, BF_RAY, NORM_T1, s);
}

template <typename T, bool FAN>
static void b_back_adj_nc(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  const dim3 grid(bl.tot[BF_RAYBT]), blk(kBlock);
  switch (bl.nc_bt) {
    case 2: hipLaunchKernelGGL((kb_back_adj<T, FAN, 2>), grid, blk, 0, s, bd, out_sel, ec); break;
    case 3: hipLaunchKernelGGL((kb_back_adj<T, FAN, 3>), grid, blk, 0, s, bd, out_sel, ec); break;
    case 4: hipLaunchKernelGGL((kb_back_adj<T, FAN, 4>), grid, blk, 0, s, bd, out_sel, ec); break;
    case 5: hipLaunchKernelGGL((kb_back_adj<T, FAN, 5>), grid, blk, 0, s, bd, out_sel, ec); break;
    case 6: hipLaunchKernelGGL((kb_back_adj<T, FAN, 6>), grid, blk, 0, s, bd, out_sel, ec); break;
    case 7: hipLaunchKernelGGL((kb_back_adj<T, FAN, 7>), grid, blk, 0, s, bd, out_sel, ec); break;
    default: hipLaunchKernelGGL((kb_back_adj<T, FAN, 8>), grid, blk, 0, s, bd, out_sel, ec); break;
  }
}

template <typename T>
void launch_b_back_adj(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  if (bl.tot[BF_RAYBT] <= 0) return;
  if (bl.fan)
    b_back_adj_nc<T, true>(bd, bl, out_sel, ec, s);
  else
    b_back_adj_nc<T, false>(bd, bl, out_sel, ec, s);
  if (ec.norm_to_t) launch_b_norm_finalize(bd, bl, BF_RAYBT, NORM_T1, s);
}

template <typename T>
void launch_b_back(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  if (bl.tot[BF_PIX] <= 0) return;
  if (bl.fan)
    hipLaunchKernelGGL((kb_back<T, true, 4>), dim3(bl.tot[BF_PIX]), dim3(kBlock), 0, s, bd, out_sel, ec);
  else if (bl.b_vu == 8)
    hipLaunchKernelGGL((kb_back<T, false, 8>), dim3(bl.tot[BF_PIX]), dim3(kBlock), 0, s, bd, out_sel, ec);
  else
    hipLaunchKernelGGL((kb_back<T, false, 4>), dim3(bl.tot[BF_PIX]), dim3(kBlock), 0, s, bd, out_sel, ec);
  if (ec.norm_to_t) launch_b_norm_finalize(bd, bl, BF_PIX, NORM_T1, s);
}

template <typename T, bool FAN>
static void b_fwd_adj_nc(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  const dim3 grid(bl.tot[BF_PIX]), blk(kBlock);
  const int vu = FAN ? 1 : at_views(bl.nc_at, bl.at_vu);
#define GKB_AT(NC, VU) hipLaunchKernelGGL((kb_fwd_adj<T, FAN, NC, VU>), grid, blk, 0, s, bd, out_sel, ec)
  switch (bl.nc_at) {
    case 2:
      if (vu == 4) GKB_AT(2, 4);
      else if (vu == 2) GKB_AT(2, 2);
      else GKB_AT(2, 1);
      break;
    case 3:
      if (vu == 4) GKB_AT(3, 4);
      else if (vu == 2) GKB_AT(3, 2);
      else GKB_AT(3, 1);
      break;
    case 4:
      if (vu == 4) GKB_AT(4, 4);
      else if (vu == 2) GKB_AT(4, 2);
      else GKB_AT(4, 1);
      break;
    case 5: GKB_AT(5, 1); break;
    case 6: GKB_AT(6, 1); break;
    case 7: GKB_AT(7, 1); break;
    default: GKB_AT(8, 1); break;
  }
#undef GKB_AT
}

template <typename T>
void launch_b_fwd_adj(const BatchDev<T> &bd, const BatchLaunch &bl, int out_sel, EpiCfg ec, hipStream_t s) {
  if (bl.tot[BF_PIX] <= 0) return;
  if (bl.fan)
    b_fwd_adj_nc<T, true>(bd, bl, out_sel, ec, s);
  else
    b_fwd_adj_nc<T, false>(bd, bl, out_sel, ec, s);
  if (ec.norm_to_t) launch_b_norm_finalize(bd, bl, BF_PIX, NORM_T1, s);
}

#define GKB_INST(T)                                                                                               \
  template void launch_pad_image<T>(const GeomDev &, Col<const T>, T *, bool, const int *, hipStream_t);         \
  template void launch_pad_sino<T>(const GeomDev &, Col<const T>, T *, const int *, hipStream_t);                \
  template void launch_pad_sino_adj<T>(const GeomDev &, const RayTab<T> &, Col<const T>, T *, const int *,       \
                                       hipStream_t);                                                             \
  template void launch_fwd<T>(const GeomDev &, const RayTab<T> &, const T *, Col<T>, const Epi<T> &,             \
                              const int *, hipStream_t);                                                         \
  template void launch_back_adj<T>(const GeomDev &, const RayTab<T> &, const T *, Col<T>, const Epi<T> &,        \
                                   const int *, hipStream_t);                                                    \
  template void launch_back<T>(const GeomDev &, const ViewTab<T> &, const T *, T *, const Epi<T> &, const int *, \
                               hipStream_t);                                                                     \
  template void launch_fwd_adj<T>(const GeomDev &, const ViewTab<T> &, const RayTab<T> &, const T *, T *,        \
                                  const Epi<T> &, const int *, hipStream_t);                             \
  template void launch_b_pad_image<T>(const BatchDev<T> &, const BatchLaunch &, int, hipStream_t);               \
  template void launch_b_pad_sino<T>(const BatchDev<T> &, const BatchLaunch &, int, int, hipStream_t);           \
  template void launch_b_fwd<T>(const BatchDev<T> &, const BatchLaunch &, int, EpiCfg, hipStream_t);             \
  template void launch_b_back_adj<T>(const BatchDev<T> &, const BatchLaunch &, int, EpiCfg, hipStream_t);        \
  template void launch_b_back<T>(const BatchDev<T> &, const BatchLaunch &, int, EpiCfg, hipStream_t);            \
  template void launch_b_fwd_adj<T>(const BatchDev<T> &, const BatchLaunch &, int, EpiCfg, hipStream_t);
GKB_INST(float)
GKB_INST(double)
#undef GKB_INST

}  // namespace gkb
