// Host emulation of the projector kernels' address arithmetic.
//
// For a geometry's tables, every (or every stride-th) wavefront, ray, pixel
// or voxel of the launches that gkb_forward, gkb_back, gkb_forward_adjoint and
// gkb_back_adjoint make is replayed on the host in the kernels' own
// arithmetic (the same fused multiply-adds, clamps and roundings in the
// kernel's floating-point type), and
//  * every element address the kernel would read is checked against its
//    buffer: the padded line (2D) or the padded volume or sinogram (cone);
//  * every candidate that carries a nonzero interpolation weight (found in
//    double from the operator's definition) is checked to lie inside the
//    window the kernel reads, and lines or planes the kernel skips are checked
//    to carry none;
//  * the dispatch orders of the ray-driven 2D kernels are checked to be
//    permutations of their launches' workgroups.
// The fan-angle and reciprocal approximations of the pixel-driven kernels
// are replaced by exact double values; windows that depend on them are
// checked with the coordinate moved by 1e-3 bins both ways.

#include <algorithm>
#include <cmath>
#include <vector>

#include "tables.h"

namespace gkb {

namespace {

template <typename T>
T clampT(T x, T lo, T hi) {
  return std::min(std::max(x, lo), hi);
}

void add_read(CheckStat &s, long long idx, long long lo, long long hi) {
  ++s.reads;
  if (idx < lo || idx >= hi) ++s.out_of_bounds;
}

// a candidate left out with a weight above the rounding bound of the
// kernel's coordinates (CheckStat::thr) is a violation
void add_miss(CheckStat &s, double w) {
  if (w > s.thr) ++s.uncovered;
  s.max_uncovered_weight = std::max(s.max_uncovered_weight, w);
}

bool is_permutation(const std::vector<int> &o, int n) {
  if ((int)o.size() != n) return false;
  std::vector<char> seen(n, 0);
  for (int v : o) {
    if (v < 0 || v >= n || seen[v]) return false;
    seen[v] = 1;
  }
  return true;
}

// ---------------------------------------------------------------- 2D ----
struct Geo2 {
  const gkb_geometry *gg;
  const HostTables &t;
  const GeomDev &g;
  bool fan;
  double midx, midy;
  std::vector<double> ang;
  Geo2(const gkb_geometry *g_, const HostTables &t_)
      : gg(g_), t(t_), g(t_.gd), fan(g_->kind == GKB_FAN2D), midx(0.5 * (g_->nx - 1)), midy(0.5 * (g_->ny - 1)),
        ang(view_angles(g_)) {}
  // detector coordinate (bins) of the point (x, y) in view v: B's interpolation variable
  double u_of(int v, double x, double y) const {
    const double c = std::cos(ang[v]), s = std::sin(ang[v]);
    if (!fan) return (x * c + y * s) / g.du + g.off;
    const double a = g.D - (x * c + y * s), b = x * s - y * c;
    return std::atan2(b, a) / g.du + g.off;
  }
  double wB(int v, int k, double x, double y) const { return std::max(0.0, 1.0 - std::fabs(u_of(v, x, y) - k)); }
  bool rowdom(long long r) const { return (t.meta[r] >> 30) & 1; }
  // Joseph's interpolation weight of ray r on pixel (i, j) (without 1/|d_dom|)
  double wA(long long r, int i, int j) const {
    if (rowdom(r)) return std::max(0.0, 1.0 - std::fabs(t.base[r] + (j - midy) * t.slope[r] - i));
    return std::max(0.0, 1.0 - std::fabs(t.base[r] + (i - midx) * t.slope[r] - j));
  }
  // pixel (i, j) at position pos of line L of a ray stepping along rows (rowdom) or columns
  void pix(bool rd, int L, int pos, int &i, int &j) const {
    i = rd ? pos : L;
    j = rd ? L : pos;
  }
};

// A: gather path of every valid ray; segment path of whole wavefronts (float)
template <typename T>
void check_fwd(const Geo2 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  const int nblk = ((g.nu + 63) / 64) * ((g.nv + 3) / 4);
  for (int wg = 0; wg < nblk; ++wg)
    for (int wave = 0; wave < 4; ++wave) {
      if ((wg * 4 + wave) % stride) continue;
      const long long r0 = (long long)wg * 256 + wave * 64;
      bool all_valid = true, any_rd = false, any_cd = false;
      for (int lane = 0; lane < 64; ++lane) {
        const long long r = r0 + lane;
        if (r >= g.m) {
          all_valid = false;
          continue;
        }
        (G.rowdom(r) ? any_rd : any_cd) = true;
      }
      const bool seg = sizeof(T) == 4 && g.fwd_seg && all_valid && !(any_rd && any_cd);
      if (seg) {
        int wlo = 1 << 20, whi = -1;
        int lo[64], hi[64];
        for (int lane = 0; lane < 64; ++lane) {
          const int meta = t.meta[r0 + lane];
          lo[lane] = meta & 0x7fff;
          hi[lane] = (meta >> 15) & 0x7fff;
          if (lo[lane] <= hi[lane]) {
            wlo = std::min(wlo, lo[lane]);
            whi = std::max(whi, hi[lane]);
          }
        }
        s.units += 64;
        if (wlo > whi) continue;
        const bool rd = any_rd;
        const int ld = rd ? g.ldR : g.ldT, len = rd ? g.nx : g.ny;
        const float mid = rd ? 0.5f * float(g.ny - 1) : 0.5f * float(g.nx - 1);
        const long long line0 = (rd ? 0LL : g.offT) + g.pad;
        const float clo = -1.5f, chi = float(len) + 0.5f;
        // the staged form takes whole blocks of kFwdStageLines lines from wlo,
        // its segment starting at the crossing of the lead lane (0 or 63,
        // whichever has the smaller crossing at the middle line); the lines
        // after the last block exchange taps between lanes, the segment
        // starting at the smaller of lanes 0 and 63
        const int nstaged = kFwdSegStage ? ((whi - wlo + 1) / kFwdStageLines) * kFwdStageLines : 0;
        const int lead = (float)t.base[r0] <= (float)t.base[r0 + 63] ? 0 : 63;
        for (int j = wlo; j <= whi; ++j) {
          int fi[64];
          float cc[64];
          for (int lane = 0; lane < 64; ++lane) {
            const long long r = r0 + lane;
            cc[lane] = clampT(std::fma(float(j) - mid, (float)t.slope[r], (float)t.base[r]), clo, chi);
            fi[lane] = (int)std::floor(cc[lane]);
          }
          const bool staged = j - wlo < nstaged;
          // segment width: 128 (parallel beam, staged form) or 64
          const int sw = staged && g.fwd_seg == 2 ? 128 : 64;
          const int s0 = staged ? fi[lead] : std::min(fi[0], fi[63]);
          const long long ls = line0 + (long long)j * ld;  // element 0 of the line
          bool gather = false;
          for (int e = 0; e < sw; ++e) add_read(s, ls + s0 + e, 0, g.pad_elems);
          for (int lane = 0; lane < 64; ++lane)
            if ((unsigned)(fi[lane] - s0) > unsigned(sw - 2)) gather = true;
          for (int lane = 0; lane < 64; ++lane) {
            if (gather) {
              add_read(s, ls + fi[lane], ls - g.pad, ls - g.pad + ld);
              add_read(s, ls + fi[lane] + 1, ls - g.pad, ls - g.pad + ld);
            }
            // a line outside the lane's own range must add nothing: both taps in the padding
            if (j < lo[lane] || j > hi[lane]) {
              const double w0 = (fi[lane] >= 0 && fi[lane] < len) ? 1.0 - (cc[lane] - fi[lane]) : 0.0;
              const double w1 = (fi[lane] + 1 >= 0 && fi[lane] + 1 < len) ? (cc[lane] - fi[lane]) : 0.0;
              if (w0 > 0.0 || w1 > 0.0) add_miss(s, std::max(w0, w1));
            }
          }
        }
        continue;
      }
      for (int lane = 0; lane < 64; ++lane) {
        const long long r = r0 + lane;
        if (r >= g.m) continue;
        ++s.units;
        const int meta = t.meta[r];
        const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
        const bool rd = (meta >> 30) & 1;
        const int ld = rd ? g.ldR : g.ldT, len = rd ? g.nx : g.ny, nl = rd ? g.ny : g.nx;
        const T mid = rd ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
        const T clo = T(-1.5), chi = T(len) + T(0.5);
        const T base = (T)t.base[r], slope = (T)t.slope[r];
        if (lo <= hi && (lo < 0 || hi >= nl)) ++s.out_of_bounds;
        for (int j = lo; j <= hi; ++j) {
          const T c = clampT(T(std::fma(T(lo) - mid + T(j - lo), slope, base)), clo, chi);
          const int fl = (int)std::floor(c);
          const long long ls = (rd ? 0LL : g.offT) + (long long)j * ld;
          add_read(s, ls + g.pad + fl, ls, ls + ld);
          add_read(s, ls + g.pad + fl + 1, ls, ls + ld);
        }
        // lines the ray skips carry no weight (double crossing)
        for (int j = 0; j < nl; ++j) {
          if (j >= lo && j <= hi) continue;
          const double c = t.base[r] + (j - (double)mid) * t.slope[r];
          if (c > -1.0 && c < len) add_miss(s, std::min(1.0, std::min(c + 1.0, len - c)));
        }
      }
    }
}

// B^T: windows of whole wavefronts, in the launch layout of back_adj_body
template <typename T>
void check_back_adj(const Geo2 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  const bool fan = G.fan;
  const int VPW = fan ? 2 : 4;
  const int tiles_u = (g.nu + 63) >> 6;
  const int nblk = fan ? tiles_u * ((g.nv + 1) / 2) : tiles_u * ((g.nv + 3) / 4);
  const int NC = std::min(std::max(g.nc_bt, 2), 8);
  for (int wg = 0; wg < nblk; ++wg)
    for (int wave = 0; wave < 4; ++wave) {
      if ((wg * 4 + wave) % stride) continue;
      const int half = fan ? (wave & 1) : -1;
      const int view = (wg / tiles_u) * VPW + (fan ? wave >> 1 : wave);
      int cmax = 0;
      for (int lane = 0; lane < 64; ++lane) {
        const int bin = (wg % tiles_u) * 64 + lane;
        if (view < g.nv && bin < g.nu)
          cmax = std::max(cmax, (int)std::floor(T(2) * (T)t.h[(long long)view * g.nu + bin]) + 1);
      }
      const int n = std::min(cmax, NC);
      for (int lane = 0; lane < 64; ++lane) {
        const int bin = (wg % tiles_u) * 64 + lane;
        if (!(view < g.nv && bin < g.nu)) continue;
        const long long r = (long long)view * g.nu + bin;
        ++s.units;
        const T hr = (T)t.h[r];
        const int meta = t.meta_bt[r];
        const int flo = meta & 0x7fff, fhi = (meta >> 15) & 0x7fff;
        int lo = flo, hi = fhi;
        if (half >= 0) {
          const int mdl = lo + std::max(hi - lo + 1, 0) / 2;
          if (half == 0)
            hi = mdl - 1;
          else
            lo = mdl;
        }
        const bool rd = (meta >> 30) & 1;
        const int ld = rd ? g.ldR : g.ldT, len = rd ? g.nx : g.ny, nl = rd ? g.ny : g.nx;
        const T mid = rd ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
        const T base = (T)t.base[r], slope = (T)t.slope[r];
        const T clo = -hr - T(0.5), chi = T(len - 1) + hr + T(0.5);
        for (int j = lo; j <= hi; ++j) {
          const T c = clampT(T(std::fma(T(lo) - mid + T(j - lo), slope, base)), clo, chi);
          const int i0 = (int)std::ceil(c - hr);
          const long long ls = (rd ? 0LL : g.offT) + (long long)j * ld;
          add_read(s, ls + g.pad + i0, ls, ls + ld);
          add_read(s, ls + g.pad + i0 + n - 1, ls, ls + ld);
          s.reads += n - 2;
          // every pixel of the line with a nonzero weight lies in the window
          const double cd = t.base[r] + (j - (double)mid) * t.slope[r];
          const int a = std::max(0, (int)std::floor(cd - t.h[r]) - 4), b = std::min(len - 1, (int)std::ceil(cd + t.h[r]) + 4);
          for (int pos = a; pos <= b; ++pos) {
            if (pos >= i0 && pos < i0 + n) continue;
            int pi, pj;
            G.pix(rd, j, pos, pi, pj);
            const double w = G.wB(view, bin, pi - G.midx, pj - G.midy);
            if (w > 0.0) add_miss(s, w);
          }
        }
        // lines outside the ray's range carry no weight
        if ((wg * 4 + wave) % (4 * stride) == 0 || stride == 1)
          for (int j = 0; j < nl; ++j) {
            if (j >= flo && j <= fhi) continue;
            const double cd = t.base[r] + (j - (double)mid) * t.slope[r];
            const int a = std::max(0, (int)std::floor(cd - t.h[r]) - 4);
            const int b = std::min(len - 1, (int)std::ceil(cd + t.h[r]) + 4);
            for (int pos = a; pos <= b; ++pos) {
              int pi, pj;
              G.pix(rd, j, pos, pi, pj);
              const double w = G.wB(view, bin, pi - G.midx, pj - G.midy);
              if (w > 0.0) add_miss(s, w);
            }
          }
      }
    }
}

// pixel (i, j) and view group of thread tid of pixel tile blk
void tile_pix(const GeomDev &g, int blk, int tid, int &i, int &j, int &grp) {
  const int tiles_x = (g.nx + kPixTileX - 1) / kPixTileX;
  const int tx = blk % tiles_x, ty = blk / tiles_x;
  constexpr int tpix = kPixTileX * kPixTileY;
  i = tx * kPixTileX + tid % kPixTileX;
  j = ty * kPixTileY + (tid % tpix) / kPixTileX;
  grp = tid / tpix;
}

// B: the pair each (pixel, view) reads
template <typename T>
void check_back(const Geo2 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const int nblk = ((g.nx + kPixTileX - 1) / kPixTileX) * ((g.ny + kPixTileY - 1) / kPixTileY);
  for (int blk = 0; blk < nblk; ++blk)
    for (int tid = 0; tid < kBlock; ++tid) {
      if ((blk * kBlock + tid) % stride) continue;
      int i, j, grp;
      tile_pix(g, blk, tid, i, j, grp);
      if (!(i < g.nx && j < g.ny)) continue;
      ++s.units;
      const T ulo = T(-2), uhi = T(g.nu + 1);
      for (int v = grp; v < g.nv; v += kViewGroups) {
        const T u = clampT((T)G.u_of(v, i - G.midx, j - G.midy), ulo, uhi);
        const int fl = (int)std::floor(u);
        const long long rs = (long long)v * g.ldY;
        add_read(s, rs + g.padY + fl, rs, rs + g.ldY);
        add_read(s, rs + g.padY + fl + 1, rs, rs + g.ldY);
      }
    }
}

// A^T: candidate windows per (pixel, view)
template <typename T>
void check_fwd_adj(const Geo2 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  const int NC = std::min(std::max(g.nc_at, 2), 8);
  const int nblk = ((g.nx + kPixTileX - 1) / kPixTileX) * ((g.ny + kPixTileY - 1) / kPixTileY);
  const T ulo = -T(g.uclamp_at), uhi = T(g.nu - 1) + T(g.uclamp_at);
  for (int blk = 0; blk < nblk; ++blk)
    for (int tid = 0; tid < kBlock; ++tid) {
      if ((blk * kBlock + tid) % stride) continue;
      int i, j, grp;
      tile_pix(g, blk, tid, i, j, grp);
      const bool valid = i < g.nx && j < g.ny;
      if (!valid && !G.fan) continue;
      ++s.units;
      const T px = T(i) - T(0.5) * T(g.nx - 1), py = T(j) - T(0.5) * T(g.ny - 1);
      for (int v = grp; v < g.nv; v += kViewGroups) {
        T H;
        int cnt;
        double ud;  // exact detector coordinate
        T u;
        if (!G.fan) {
          u = clampT(T(std::fma(px, (T)t.p0[v], std::fma(py, (T)t.p1[v], T(g.off)))), ulo, uhi);
          H = (T)t.p4[v];
          cnt = std::min((int)std::floor(T(2) * H) + 1, NC);
          ud = G.u_of(v, i - G.midx, j - G.midy);
        } else {
          H = (T)t.htile[(size_t)blk * g.nv + v];
          cnt = std::min((int)std::floor(T(2) * H) + 1, NC);
          ud = G.u_of(v, i - G.midx, j - G.midy);
          u = clampT((T)ud, ulo, uhi);
        }
        const long long rs = (long long)v * g.ldY;
        // parallel beam with several views per step reads every view's full
        // window of the geometry's candidate count
        const int nread = G.fan ? cnt : std::max(cnt, std::min(g.nc_at, NC));
        // reads (fan beam: the same indices in units of (w y, w) pairs)
        for (int sh = -1; sh <= 1; ++sh) {
          if (!G.fan && sh != 0) continue;
          const T us = G.fan ? clampT(T(u + T(sh) * T(1e-3)), ulo, uhi) : u;
          const int k0 = (int)std::ceil(us - H);
          add_read(s, rs + g.padY + k0, rs, rs + g.ldY);
          add_read(s, rs + g.padY + k0 + nread - 1, rs, rs + g.ldY);
          s.reads += nread - 2;
          if (!valid) continue;
          // every bin whose ray passes within a pixel of p lies in the window
          const int a = std::max(0, (int)std::floor(ud) - NC - 4), b = std::min(g.nu - 1, (int)std::ceil(ud) + NC + 4);
          for (int k = a; k <= b; ++k) {
            if (k >= k0 && k < k0 + cnt) continue;
            const double w = G.wA((long long)v * g.nu + k, i, j);
            if (w > 0.0) add_miss(s, w);
          }
        }
      }
    }
}

// ---------------------------------------------------------------- cone ----
struct Geo3 {
  const HostTables &t;
  const GeomDev &g;
  double midx, midy, midz;
  std::vector<double> cb, sb;
  Geo3(const gkb_geometry *gg, const HostTables &t_)
      : t(t_), g(t_.gd), midx(0.5 * (gg->nx - 1)), midy(0.5 * (gg->ny - 1)), midz(0.5 * (gg->nz - 1)) {
    const std::vector<double> a = view_angles(gg);
    for (double x : a) {
      cb.push_back(std::cos(x));
      sb.push_back(std::sin(x));
    }
  }
  // B's bilinear weight of voxel (x, y, z) (centred coordinates) on detector pixel (k, r) of view v
  double wB(int v, int k, int r, double x, double y, double z) const {
    const double depth = g.D - (x * cb[v] + y * sb[v]);
    const double u = (y * cb[v] - x * sb[v]) * g.Su / depth + g.off;
    const double w = z * g.Sw / depth + g.offw;
    return std::max(0.0, 1.0 - std::fabs(u - k)) * std::max(0.0, 1.0 - std::fabs(w - r));
  }
  // rows l whose voxel at (x, y) can project within two detector rows of r in view v
  void rows_near(int v, int r, double x, double y, int &la, int &lb) const {
    const double depth = g.D - (x * cb[v] + y * sb[v]);
    const double zc = (r - g.offw) * depth / g.Sw, zh = depth / g.Sw;
    la = std::max(0, (int)std::floor(midz + zc - 2.0 * zh) - 1);
    lb = std::min(g.nz - 1, (int)std::ceil(midz + zc + 2.0 * zh) + 1);
  }
  // Joseph-3D weight of ray (v, r, k) on voxel (i, j, l): bilinear in the voxel's plane along the ray's dominant axis
  double wA(int v, int r, int k, int i, int j, int l) const {
    const size_t vk = (size_t)v * g.nu + k;
    const bool yd = (t.cmeta[vk] >> 30) & 1;
    const double mid = yd ? midy : midx;
    const int tpl = yd ? j : i, o1 = yd ? i : j;
    const double tf = tpl - mid;
    const double c1 = t.cbase1[vk] + tf * t.cslope1[vk];
    const double vv = (r - g.offw) * g.dw;
    const double c2 = vv * t.clmid[vk] + midz + tf * vv * t.clslope[vk];
    return std::max(0.0, 1.0 - std::fabs(c1 - o1)) * std::max(0.0, 1.0 - std::fabs(c2 - l));
  }
};

// A: plane range trimmed by the ray's height; skipped planes carry no weight
template <typename T>
void check_cone_fwd(const Geo3 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  for (long long rr = 0; rr < g.m; rr += stride) {
    const int k = (int)(rr % g.nu);
    const long long vr = rr / g.nu;
    const int r = (int)(vr % g.nw), v = (int)(vr / g.nw);
    const size_t vk = (size_t)v * g.nu + k;
    ++s.units;
    const int meta = t.cmeta[vk];
    int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
    const bool yd = (meta >> 30) & 1;
    const T vv = (T(r) - T(g.offw)) * T(g.dw);
    const T midz = T(0.5) * T(g.nz - 1);
    const T base2 = T(std::fma(vv, (T)t.clmid[vk], midz)), slope2 = vv * (T)t.clslope[vk];
    const T mid = yd ? T(0.5) * T(g.ny - 1) : T(0.5) * T(g.nx - 1);
    if (slope2 != T(0)) {
      T ta = (T(-1) - base2) / slope2, tb = (T(g.nz) - base2) / slope2;
      if (ta > tb) std::swap(ta, tb);
      lo = std::max(lo, (int)std::fmin(std::fmax(std::ceil(ta + mid) - T(1), T(-1)), T(32767)));
      hi = std::min(hi, (int)std::fmin(std::fmax(std::floor(tb + mid) + T(1), T(-1)), T(32767)));
    } else if (!(base2 > T(-1) && base2 < T(g.nz))) {
      hi = lo - 1;
    }
    const int nax = yd ? g.ny : g.nx, n1 = yd ? g.nx : g.ny;
    const int ld = yd ? g.ldV : g.ldX;
    const long long plane = yd ? g.planeY : g.planeX, vol0 = yd ? g.offYD : 0;
    const T c1lo = T(-1.5), c1hi = T(n1) + T(0.5), c2lo = T(-1.5), c2hi = T(g.nz) + T(0.5);
    const T base1 = (T)t.cbase1[vk], slope1 = (T)t.cslope1[vk];
    for (int tp = lo; tp <= hi; ++tp) {
      const T tf = T(lo) - mid + T(tp - lo);
      const T p1 = clampT(T(std::fma(tf, slope1, base1)), c1lo, c1hi);
      const T p2 = clampT(T(std::fma(tf, slope2, base2)), c2lo, c2hi);
      const long long o = vol0 + (long long)tp * plane + (long long)(g.P3 * ld + g.P3) +
                          (long long)((int)std::floor(p2) * ld + (int)std::floor(p1));
      add_read(s, o, 0, g.vol_pad_elems);
      add_read(s, o + 1 + ld, 0, g.vol_pad_elems);
      s.reads += 2;
    }
    // planes outside [lo, hi]: the sample's in-plane or height coordinate is outside (-1, n)
    for (int tp = 0; tp < nax; ++tp) {
      if (tp >= lo && tp <= hi) continue;
      const double tf = tp - (yd ? G.midy : G.midx);
      const double c1 = t.cbase1[vk] + tf * t.cslope1[vk];
      const double vvd = (r - g.offw) * g.dw;
      const double c2 = vvd * t.clmid[vk] + G.midz + tf * vvd * t.clslope[vk];
      if (c1 > -1.0 && c1 < n1 && c2 > -1.0 && c2 < g.nz)
        add_miss(s, std::min(std::min(c1 + 1.0, n1 - c1), 1.0) * std::min(std::min(c2 + 1.0, g.nz - c2), 1.0));
    }
  }
}

// B: the two pairs each (voxel, view) reads from the padded sinogram
template <typename T>
void check_cone_back(const Geo3 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  const T ulo = T(-2), uhi = T(g.nu), wlo = T(-2), whi = T(g.nw);
  for (long long p = 0; p < g.n; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), l = (int)(p / ((long long)g.nx * g.ny));
    ++s.units;
    const T x = T(i) - T(0.5) * T(g.nx - 1), y = T(j) - T(0.5) * T(g.ny - 1), z = T(l) - T(0.5) * T(g.nz - 1);
    for (int v = 0; v < g.nv; ++v) {
      const T cbv = (T)t.p0[v], sbv = (T)t.p1[v];
      const T depth = T(g.D) - T(std::fma(x, cbv, y * sbv));
      const T unum = T(std::fma(y, cbv, -(x * sbv)));
      const T inv = T(1) / depth;
      const T u = clampT(T(std::fma(unum, T(g.Su) * inv, T(g.off))), ulo, uhi);
      const T w = clampT(T(std::fma(z, T(g.Sw) * inv, T(g.offw))), wlo, whi);
      const long long o = (long long)v * g.sliceY + (long long)(g.PY3 * g.ldSu + g.PY3) +
                          (long long)((int)std::floor(w) * g.ldSu + (int)std::floor(u));
      add_read(s, o, 0, g.sino_pad_elems);
      add_read(s, o + g.ldSu + 1, 0, g.sino_pad_elems);
      s.reads += 2;
    }
  }
}

// B^T per-voxel loops (windows too large for the uniform form) of ray rr
template <typename T>
void check_cone_bt_generic(const Geo3 &G, long long rr, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  ++s.units;
  const int k = (int)(rr % g.nu);
  const long long vr = rr / g.nu;
  const int r = (int)(vr % g.nw), v = (int)(vr / g.nw);
  const size_t vk = (size_t)v * g.nu + k;
  const int meta = t.cmeta_bt[vk];
  const int lo = meta & 0x7fff, hi = (meta >> 15) & 0x7fff;
  const bool yd = (meta >> 30) & 1;
  const T base1 = (T)t.cbase1[vk], slope1 = (T)t.cslope1[vk], h1 = (T)t.ch1[vk];
  const T cbv = (T)t.p0[v], sbv = (T)t.p1[v], D = T(g.D);
  const T midx = T(0.5) * T(g.nx - 1), midy = T(0.5) * T(g.ny - 1), midz = T(0.5) * T(g.nz - 1);
  const T mid = yd ? midy : midx, mid1 = yd ? midx : midy;
  const int n1 = yd ? g.nx : g.ny, nax = yd ? g.ny : g.nx;
  const int ld = yd ? g.ldV : g.ldX;
  const long long plane = yd ? g.planeY : g.planeX;
  const long long vol0 = (yd ? g.offYD : 0LL) + (g.P3 * ld + g.P3);
  const T Su = T(g.Su), Sw = T(g.Sw), offu = T(g.off), offw = T(g.offw);
  const T kf = T(k), rf = T(r), inv_sw = T(1) / Sw, eps = T(1e-3);
  for (int tp = 0; tp < nax; ++tp) {
    const bool visited = tp >= lo && tp <= hi;
    const T tf = T(tp) - mid;
    const T c1 = T(std::fma(tf, slope1, base1));
    const int j0 = std::max((int)std::ceil(c1 - h1), 0), j1 = std::min((int)std::floor(c1 + h1), n1 - 1);
    const double c1d = t.cbase1[vk] + (tp - (yd ? G.midy : G.midx)) * t.cslope1[vk];
    const int a = std::max(0, (int)std::floor(c1d - t.ch1[vk]) - 3);
    const int b = std::min(n1 - 1, (int)std::ceil(c1d + t.ch1[vk]) + 3);
    for (int o = a; o <= b; ++o) {
      const bool col_in = visited && o >= j0 && o <= j1;
      int l0 = 1, l1 = 0;
      if (col_in) {
        const T oo = T(o) - mid1;
        const T x = yd ? oo : tf, y = yd ? tf : oo;
        const T depth = D - T(std::fma(x, cbv, y * sbv));
        const T unum = T(std::fma(y, cbv, -(x * sbv)));
        const T inv = T(1) / depth;
        const T u = T(std::fma(unum, Su * inv, offu));
        if (T(1) - std::fabs(u - kf) > T(0)) {
          const T zh = depth * inv_sw, zc = (rf - offw) * zh + midz;
          l0 = std::max((int)std::ceil(zc - zh - eps), 0);
          l1 = std::min((int)std::floor(zc + zh + eps), g.nz - 1);
          if (l0 <= l1) {
            add_read(s, vol0 + (long long)tp * plane + (long long)l0 * ld + o, 0, g.vol_pad_elems);
            add_read(s, vol0 + (long long)tp * plane + (long long)l1 * ld + o, 0, g.vol_pad_elems);
          }
        }
      }
      const double x = yd ? o - G.midx : tp - G.midx, y = yd ? tp - G.midy : o - G.midy;
      int la, lb;
      G.rows_near(v, r, x, y, la, lb);
      for (int l = la; l <= lb; ++l) {
        if (col_in && l >= l0 && l <= l1) continue;
        const double w = G.wB(v, k, r, x, y, l - G.midz);
        if (w > 0.0) add_miss(s, w);
      }
    }
  }
}

// B^T: the uniform windows of whole wavefronts (the per-voxel loops where
// the windows would be too large read within explicit bounds)
template <typename T>
void check_cone_back_adj(const Geo3 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  const long long nwave = (g.m + 63) / 64;
  for (long long wv = 0; wv < nwave; wv += stride) {
    int nj = 0, nl = 0;
    for (int lane = 0; lane < 64; ++lane) {
      const long long rr = wv * 64 + lane;
      if (rr >= g.m) continue;
      const int k = (int)(rr % g.nu);
      const long long vr = rr / g.nu;
      const int r = (int)(vr % g.nw), v = (int)(vr / g.nw);
      const size_t vk = (size_t)v * g.nu + k;
      const T h1 = (T)t.ch1[vk];
      nj = std::max(nj, (int)std::floor(T(2) * h1) + 1);
      const bool yd = (t.cmeta_bt[vk] >> 30) & 1;
      (void)yd;
    }
    nj = std::max(nj, 2);
    for (int lane = 0; lane < 64; ++lane) {
      const long long rr = wv * 64 + lane;
      if (rr >= g.m) continue;
      const int k = (int)(rr % g.nu);
      const long long vr = rr / g.nu;
      const int r = (int)(vr % g.nw), v = (int)(vr / g.nw);
      const size_t vk = (size_t)v * g.nu + k;
      const bool yd = (t.cmeta_bt[vk] >> 30) & 1;
      const T ddo = std::fabs(yd ? (T)t.p0[v] : (T)t.p1[v]);
      const T rho = std::fabs(T(r) - T(g.offw));
      const int nl_ray =
          (int)std::floor(T(std::fma(T(2), T(g.dmax3), rho * ddo * T(nj - 1))) / T(g.Sw) + T(2e-3)) + 1;
      nl = std::max(nl, nl_ray);
    }
    const bool fits = nl <= 4 && nl <= g.nz + 2 * g.P3 && nj <= 5 && nj <= std::min(g.nx, g.ny) + 2 * g.P3;
    if (!fits) {
      for (int lane = 0; lane < 64; ++lane)
        if (wv * 64 + lane < g.m) check_cone_bt_generic<T>(G, wv * 64 + lane, s);
      continue;
    }
    const int NJ = nj;
    for (int lane = 0; lane < 64; ++lane) {
      const long long rr = wv * 64 + lane;
      if (rr >= g.m) continue;
      ++s.units;
      const int k = (int)(rr % g.nu);
      const long long vr = rr / g.nu;
      const int r = (int)(vr % g.nw), v = (int)(vr / g.nw);
      const size_t vk = (size_t)v * g.nu + k;
      const int meta = t.cmeta_bt[vk];
      const int flo = meta & 0x7fff, fhi = (meta >> 15) & 0x7fff;
      int lo = flo, hi = fhi;
      const bool yd = (meta >> 30) & 1;
      const T base1 = (T)t.cbase1[vk], slope1 = (T)t.cslope1[vk], h1 = (T)t.ch1[vk];
      const T cbv = (T)t.p0[v], sbv = (T)t.p1[v], D = T(g.D);
      const T midx = T(0.5) * T(g.nx - 1), midy = T(0.5) * T(g.ny - 1), midz = T(0.5) * T(g.nz - 1);
      const T mid = yd ? midy : midx, mid1 = yd ? midx : midy;
      const int n1 = yd ? g.nx : g.ny, nax = yd ? g.ny : g.nx;
      const int ld = yd ? g.ldV : g.ldX;
      const long long plane = yd ? g.planeY : g.planeX;
      const long long vol0 = (yd ? g.offYD : 0LL) + (g.P3 * ld + g.P3);
      const T Sw = T(g.Sw), inv_sw = T(1) / Sw;
      const T rhov = T(r) - T(g.offw);
      const T eps = T(1e-3);
      const T ddo = yd ? -cbv : -sbv, dtt = yd ? -sbv : -cbv;
      {
        const T vv = rhov * T(g.dw);
        const T base2 = T(std::fma(vv, (T)t.clmid[vk], midz)), slope2 = vv * (T)t.clslope[vk];
        const T zm = T(std::fma(T(g.dmax3), inv_sw, std::fabs(rhov) * inv_sw * (h1 + T(1)))) + T(1);
        if (slope2 != T(0)) {
          T ta = (T(-1) - zm - base2) / slope2, tb = (T(g.nz) + zm - base2) / slope2;
          if (ta > tb) std::swap(ta, tb);
          lo = std::max(lo, (int)std::fmin(std::fmax(std::ceil(ta + mid) - T(1), T(-1)), T(32767)));
          hi = std::min(hi, (int)std::fmin(std::fmax(std::floor(tb + mid) + T(1), T(-1)), T(32767)));
        } else if (!(base2 > T(-1) - zm && base2 < T(g.nz) + zm)) {
          hi = lo - 1;
        }
      }
      const T rm = (rhov - T(1)) * inv_sw;
      const bool last_end = (rm >= T(0)) != (ddo >= T(0));
      const T cmin = (last_end ? rm * (T(NJ - 1) * ddo) : T(0)) + (midz - eps);
      const T jlo = T(-g.P3), jhi = T(n1 - 1 + g.P3 - (NJ - 1));
      const T llo = T(-g.P3), lhi = T(g.nz - 1 + g.P3 - (nl - 1));
      for (int tp = lo; tp <= hi; ++tp) {
        const T tf = T(tp) - mid;
        const T j0f = clampT(T(std::ceil(T(std::fma(tf, slope1, base1)) - h1)), jlo, jhi);
        const T o0 = j0f - mid1;
        const T dep0 = T(std::fma(o0, ddo, T(std::fma(tf, dtt, D))));
        const T l0f = clampT(T(std::ceil(T(std::fma(rm, dep0, cmin)))), llo, lhi);
        const int j0 = (int)j0f, l0 = (int)l0f;
        const long long base = vol0 + (long long)tp * plane;
        add_read(s, base + (long long)l0 * ld + j0, 0, g.vol_pad_elems);
        add_read(s, base + (long long)(l0 + nl - 1) * ld + j0 + NJ - 1, 0, g.vol_pad_elems);
        s.reads += (long long)nl * NJ - 2;
        // every voxel of the plane with a nonzero weight lies in the window
        const double c1 = t.cbase1[vk] + (tp - (yd ? G.midy : G.midx)) * t.cslope1[vk];
        const int a = std::max(0, (int)std::floor(c1 - t.ch1[vk]) - 3);
        const int b = std::min(n1 - 1, (int)std::ceil(c1 + t.ch1[vk]) + 3);
        for (int o = a; o <= b; ++o) {
          const double x = yd ? o - G.midx : tp - G.midx, y = yd ? tp - G.midy : o - G.midy;
          int la, lb;
          G.rows_near(v, r, x, y, la, lb);
          for (int l = la; l <= lb; ++l) {
            if (o >= j0 && o < j0 + NJ && l >= l0 && l < l0 + nl) continue;
            const double w = G.wB(v, k, r, x, y, l - G.midz);
            if (w > 0.0) add_miss(s, w);
          }
        }
      }
      // planes outside [lo, hi] carry no weight near the ray
      for (int tp = 0; tp < nax; ++tp) {
        if (tp >= lo && tp <= hi) continue;
        const double c1 = t.cbase1[vk] + (tp - (yd ? G.midy : G.midx)) * t.cslope1[vk];
        const int a = std::max(0, (int)std::floor(c1 - t.ch1[vk]) - 3);
        const int b = std::min(n1 - 1, (int)std::ceil(c1 + t.ch1[vk]) + 3);
        for (int o = a; o <= b; ++o) {
          const double x = yd ? o - G.midx : tp - G.midx, y = yd ? tp - G.midy : o - G.midy;
          int la, lb;
          G.rows_near(v, r, x, y, la, lb);
          for (int l = la; l <= lb; ++l) {
            const double w = G.wB(v, k, r, x, y, l - G.midz);
            if (w > 0.0) add_miss(s, w);
          }
        }
      }
    }
  }
}

// A^T: the candidate columns and rows of every (voxel, view)
template <typename T>
void check_cone_fwd_adj(const Geo3 &G, int stride, CheckStat &s) {
  const GeomDev &g = G.g;
  const HostTables &t = G.t;
  for (long long p = 0; p < g.n; p += stride) {
    const int i = (int)(p % g.nx), j = (int)((p / g.nx) % g.ny), l = (int)(p / ((long long)g.nx * g.ny));
    ++s.units;
    const T x = T(i) - T(0.5) * T(g.nx - 1), y = T(j) - T(0.5) * T(g.ny - 1), z = T(l) - T(0.5) * T(g.nz - 1);
    const T D = T(g.D), Su = T(g.Su), offu = T(g.off), offw = T(g.offw), du = T(g.du), dw = T(g.dw);
    const T hk_fac = T(g.hk_fac), eps = T(1e-3);
    for (int v = 0; v < g.nv; ++v) {
      const T cbv = (T)t.p0[v], sbv = (T)t.p1[v];
      const T depth = D - T(std::fma(x, cbv, y * sbv));
      const T unum = T(std::fma(y, cbv, -(x * sbv)));
      const T inv = T(1) / depth;
      const T u = T(std::fma(unum, Su * inv, offu));
      const T hk = T(std::fma(hk_fac, inv, T(1e-4)));
      const int k0 = std::max((int)std::ceil(u - hk), 0), k1 = std::min((int)std::floor(u + hk), g.nu - 1);
      const T dxs = x - D * cbv, dys = y - D * sbv;
      const int a = std::max(0, k0 - 4), b = std::min(g.nu - 1, k1 + 4);
      for (int k = a; k <= b; ++k) {
        const size_t vk = (size_t)v * g.nu + k;
        const T pkx = (T)t.cpk[2 * vk], pky = (T)t.cpk[2 * vk + 1];
        const T lam = (pky != T(0) ? dys : dxs) * pkx;
        const T ldw = lam * dw;
        const T rh = T(1) / ldw, rc = T(std::fma(z, rh, offw));
        const int r0 = std::max((int)std::ceil(rc - rh - eps), 0), r1 = std::min((int)std::floor(rc + rh + eps), g.nw - 1);
        const bool kin = k >= k0 && k <= k1;
        if (kin) s.reads += std::max(r1 - r0 + 1, 0);
        const int ra = std::max(0, r0 - 3), rb = std::min(g.nw - 1, r1 + 3);
        for (int r = ra; r <= rb; ++r) {
          if (kin && r >= r0 && r <= r1) continue;
          const double w = G.wA(v, r, k, i, j, l);
          if (w > 0.0) add_miss(s, w);
        }
        (void)du;
      }
    }
  }
}

// Coordinates |c| <= L = max(nx, ny, nz, n_det_u, n_det_v) + 16 formed in the
// kernel's type move a window edge by a few units in their last place: in
// float 8 L 2^-24, and the weights of the hats (slopes at most about 1.5 per
// pixel or bin) left out there are of that size.  Double: 1e-9.
double rounding_bound(const gkb_geometry *g, bool f32) {
  const int L = std::max({g->nx, g->ny, std::max(g->nz, 1), g->n_det_u, std::max(g->n_det_v, 1)}) + 16;
  return f32 ? 8.0 * L * 5.9604644775390625e-08 : 1e-9;
}

}  // namespace

bool check_tables_2d(const gkb_geometry *g, const HostTables &t, bool f32, int stride, CheckStat stats[4]) {
  Geo2 G(g, t);
  for (int i = 0; i < 4; ++i) stats[i].thr = rounding_bound(g, f32);
  if (f32) {
    check_fwd<float>(G, stride, stats[0]);
    check_back<float>(G, stride, stats[1]);
    check_fwd_adj<float>(G, stride, stats[2]);
    check_back_adj<float>(G, stride, stats[3]);
  } else {
    check_fwd<double>(G, stride, stats[0]);
    check_back<double>(G, stride, stats[1]);
    check_fwd_adj<double>(G, stride, stats[2]);
    check_back_adj<double>(G, stride, stats[3]);
  }
  const GeomDev &gd = t.gd;
  const int tiles_u = (gd.nu + 63) / 64;
  const int nfwd = tiles_u * ((gd.nv + 3) / 4);
  const int nbt = gd.kind == GKB_FAN2D ? tiles_u * ((gd.nv + 1) / 2) : nfwd;
  return is_permutation(t.order_fwd, nfwd) && is_permutation(t.order_bt, nbt) && (long long)nfwd * 256 >= gd.m;
}

void check_tables_cone(const gkb_geometry *g, const HostTables &t, bool f32, int stride, CheckStat stats[4]) {
  Geo3 G(g, t);
  for (int i = 0; i < 4; ++i) stats[i].thr = rounding_bound(g, f32);
  if (f32) {
    check_cone_fwd<float>(G, stride, stats[0]);
    check_cone_back<float>(G, stride, stats[1]);
    check_cone_fwd_adj<float>(G, stride, stats[2]);
    check_cone_back_adj<float>(G, stride, stats[3]);
  } else {
    check_cone_fwd<double>(G, stride, stats[0]);
    check_cone_back<double>(G, stride, stats[1]);
    check_cone_fwd_adj<double>(G, stride, stats[2]);
    check_cone_back_adj<double>(G, stride, stats[3]);
  }
}

}  // namespace gkb
