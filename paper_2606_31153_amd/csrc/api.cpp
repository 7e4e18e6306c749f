// Host side of libgkb: the C ABI declared in include/gkb.h, geometry tables,
// workspaces, kernel tracing and the AB-/BA-/matched GKB drivers.
//
// The drivers follow the Golub-Kahan bidiagonalisation of Sec. 3 (Algs.
// "GKB", "AB-GKB", "BA-GKB") read as the Paige-Saunders recurrence:
// iteration k forms s_{k+1}, t_{k+1} from M q_k, then q_{k+1}, alpha_{k+1}
// from M^T s_{k+1} with one-sided reorthogonalisation, and finally solves the
// projected problem (eq. proj GKB) for u_k and applies the discrepancy
// principle (eq. DP) to ||A x_k - b||.  Every quantity that changes from one
// iteration to the next lives in device memory (the iteration counter
// included), so one iteration is a fixed sequence of kernel launches; the
// host only reads the stop flag, a few iterations behind the device.

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/gkb.h"
#include "internal.h"
#include "tables.h"

using namespace gkb;

namespace {

thread_local std::string g_err;

gkb_status fail(gkb_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

inline size_t al256_bytes(size_t b) { return (b + 255) & ~size_t(255); }

#define HIPC(expr)                                                                          \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess) return fail(GKB_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// --------------------------------------------------------------------------
// device buffer
// --------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) bytes = b;
    return e;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

// --------------------------------------------------------------------------
// geometry tables
// --------------------------------------------------------------------------

}  // namespace

namespace gkb {

// views per step of the parallel-beam A^T and B when a geometry is not tuned
constexpr int kDefaultAtViews = 4, kDefaultBViews = 8;

std::vector<double> view_angles(const gkb_geometry *g) {
  std::vector<double> a(g->n_views);
  for (int v = 0; v < g->n_views; ++v) a[v] = g->angles ? g->angles[v] : v * (g->angle_span / g->n_views);
  return a;
}

// Lines [lo, hi] of a ray whose crossing coordinate on line L is
// c(L) = c_mid + (L - mid) * slope: the lines with c in [cmin, cmax].
void line_range(double c_mid, double slope, double mid, int nlines, double cmin, double cmax, int &lo, int &hi) {
  double Llo, Lhi;
  if (std::fabs(slope) < 1e-300) {
    if (c_mid < cmin || c_mid > cmax) {
      lo = 1;
      hi = 0;
      return;
    }
    Llo = 0;
    Lhi = nlines - 1;
  } else {
    double a = mid + (cmin - c_mid) / slope, b = mid + (cmax - c_mid) / slope;
    if (a > b) std::swap(a, b);
    Llo = std::ceil(a - 1e-9);
    Lhi = std::floor(b + 1e-9);
  }
  lo = (int)std::max(0.0, Llo);
  hi = (int)std::min((double)nlines - 1, Lhi);
  if (lo > hi) {
    lo = 1;
    hi = 0;
  }
}

// Fan-beam A^T: a pixel p gets a nonzero weight from the bins k with
// |g_p - g_k| < asin(|d_dom,k| / |p - S|) (Joseph's weight as a function of the
// fan angle); the kernel bounds |d_dom,k| by the pixel's own ray's plus the fan
// spread of the candidates, and asin(z) by z (1 + z^2).  Per 32x2 tile of
// pixel centres and per view, the largest such half-width (in bins) over the
// tile follows from the tile's nearest point to the source (largest 1/|p - S|)
// and the largest max(|cos|, |sin|) of the directions from the source to the
// tile (1 if they cross an axis direction, else at a corner).  The kernel
// takes a window of floor(2H) + 1 bins from ceil(u_p - H) for every pixel of
// the tile.
void fan_tile_halfwidths(const gkb_geometry *g, const std::vector<double> &ang, HostTables &t) {
  const GeomDev &gd = t.gd;
  const int nx = g->nx, ny = g->ny, nv = g->n_views;
  const int tx_n = (nx + kPixTileX - 1) / kPixTileX, ty_n = (ny + kPixTileY - 1) / kPixTileY;
  const double midx = 0.5 * (nx - 1), midy = 0.5 * (ny - 1);
  const double quarter = 0.5 * M_PI;
  t.htile.assign((size_t)tx_n * ty_n * nv, 0.0);
  for (int v = 0; v < nv; ++v) {
    const double Sx = g->src_dist * std::cos(ang[v]), Sy = g->src_dist * std::sin(ang[v]);
    for (int ty = 0; ty < ty_n; ++ty)
      for (int tx = 0; tx < tx_n; ++tx) {
        // rectangle of the tile's pixel centres
        const double x0 = tx * kPixTileX - midx, x1 = std::min(tx * kPixTileX + kPixTileX - 1, nx - 1) - midx;
        const double y0 = ty * kPixTileY - midy, y1 = std::min(ty * kPixTileY + kPixTileY - 1, ny - 1) - midy;
        const double dx = std::max({x0 - Sx, 0.0, Sx - x1}), dy = std::max({y0 - Sy, 0.0, Sy - y1});
        const double rinv = 1.0 / std::sqrt(dx * dx + dy * dy);
        // directions from the source to the corners, as angles about the
        // direction to the tile's centre (the tile subtends less than pi)
        const double cx = 0.5 * (x0 + x1) - Sx, cy = 0.5 * (y0 + y1) - Sy;
        const double phic = std::atan2(cy, cx);
        double lo = 0.0, hi = 0.0, ddm = 0.0;
        const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
        for (double px : xs)
          for (double py : ys) {
            const double ex = px - Sx, ey = py - Sy;
            const double dphi = std::atan2(cx * ey - cy * ex, cx * ex + cy * ey);
            lo = std::min(lo, dphi);
            hi = std::max(hi, dphi);
            ddm = std::max(ddm, std::max(std::fabs(ex), std::fabs(ey)) / std::sqrt(ex * ex + ey * ey));
          }
        if (std::ceil((phic + lo) / quarter) <= (phic + hi) / quarter) ddm = 1.0;
        const double z = std::min(ddm + gd.dd_spread, 1.0) * rinv;
        t.htile[((size_t)ty * tx_n + tx) * nv + v] = gd.hmax_fan * z * (1.0 + z * z) + 1e-3;
      }
  }
}

// Ray geometry in pixel index coordinates (crossing at the middle line and
// its slope per line), filled for every ray of a 2D geometry.
void ray_dispatch_orders(HostTables &t, int nu, int nv, bool fan);

void build_tables(const gkb_geometry *g, HostTables &t) {
  const int nx = g->nx, ny = g->ny, nv = g->n_views, nu = g->n_det_u;
  const long long m = (long long)nv * nu;
  const double du = g->det_pitch_u;
  const double off = 0.5 * (nu - 1);
  const bool fan = g->kind == GKB_FAN2D;
  const std::vector<double> ang = view_angles(g);
  t.base.resize(m);
  t.slope.resize(m);
  t.w.resize(m);
  t.h.resize(m);
  t.meta.resize(m);
  t.meta_bt.resize(m);
  if (fan) {
    t.t0.resize(m);
    t.dt.resize(m);
    t.dperp.resize(m);
    t.dpar.resize(m);
  }
  t.p0.resize(nv);
  t.p1.resize(nv);
  t.p2.resize(nv);
  t.p3.resize(nv);
  t.p4.resize(nv);
  const double midy = 0.5 * (ny - 1), midx = 0.5 * (nx - 1);
  const double tan_dg = std::tan(du);
  double hmax_bt = 0.0, hmax_at = 0.0;
  for (int v = 0; v < nv; ++v) {
    const double th = ang[v];
    const double c = std::cos(th), s = std::sin(th);
    if (!fan) {
      const double dd = std::max(std::fabs(c), std::fabs(s));
      t.p0[v] = c / du;
      t.p1[v] = s / du;
      t.p2[v] = 1.0 / dd;
      t.p3[v] = du / dd;
      t.p4[v] = dd / du;
      hmax_at = std::max(hmax_at, dd / du);
    } else {
      t.p0[v] = c;
      t.p1[v] = s;
      t.p2[v] = t.p3[v] = t.p4[v] = 0.0;
    }
    const double Sx = g->src_dist * c, Sy = g->src_dist * s;
    for (int k = 0; k < nu; ++k) {
      const long long r = (long long)v * nu + k;
      double cmid, slope, w, h;
      bool rowdom;
      if (!fan) {
        const double sk = (k - off) * du;
        rowdom = std::fabs(c) >= std::fabs(s);
        if (rowdom) {
          cmid = sk / c + midx;
          slope = -s / c;
          w = 1.0 / std::fabs(c);
        } else {
          cmid = sk / s + midy;
          slope = -c / s;
          w = 1.0 / std::fabs(s);
        }
        h = du * w;
      } else {
        const double gam = (k - off) * du;
        const double dx = -std::cos(th + gam), dy = -std::sin(th + gam);
        rowdom = std::fabs(dy) >= std::fabs(dx);
        double t0, dt, dperp, dpar;
        if (rowdom) {
          cmid = Sx - Sy * dx / dy + midx;
          slope = dx / dy;
          w = 1.0 / std::fabs(dy);
          t0 = -Sy / dy;
          dt = 1.0 / dy;
          dperp = -dy;
          dpar = dx;
        } else {
          cmid = Sy - Sx * dy / dx + midy;
          slope = dy / dx;
          w = 1.0 / std::fabs(dx);
          t0 = -Sx / dx;
          dt = 1.0 / dx;
          dperp = dx;
          dpar = dy;
        }
        t.t0[r] = t0;
        t.dt[r] = dt;
        t.dperp[r] = dperp;
        t.dpar[r] = dpar;
        // B^T candidates on a line: |delta| < tan(dg) * along, |delta| = |dperp| |d|
        const int nl = rowdom ? ny : nx;
        const double mid = rowdom ? midy : midx;
        const double al = std::max(std::fabs(t0 + (0 - mid) * dt), std::fabs(t0 + (nl - 1 - mid) * dt)) + 4.0;
        h = tan_dg * al / (std::fabs(dperp) - tan_dg) * 1.0001 + 1e-3;
      }
      const int nl = rowdom ? ny : nx, len = rowdom ? nx : ny;
      const double mid = rowdom ? midy : midx;
      int lo, hi;
      line_range(cmid, slope, mid, nl, -1.0, (double)len, lo, hi);
      t.meta[r] = lo | (hi << 15) | ((rowdom ? 1 : 0) << 30);
      line_range(cmid, slope, mid, nl, -h, len - 1 + h, lo, hi);
      t.meta_bt[r] = lo | (hi << 15) | ((rowdom ? 1 : 0) << 30);
      if (fan && lo <= hi) {
        const double a0 = t.t0[r] + (lo - mid) * t.dt[r], a1 = t.t0[r] + (hi - mid) * t.dt[r];
        t.min_along = std::min(t.min_along, std::min(std::fabs(a0), std::fabs(a1)));
      }
      if (!rowdom) t.has_coldom = true;
      t.base[r] = cmid;
      t.slope[r] = slope;
      t.w[r] = w;
      t.h[r] = h;
      hmax_bt = std::max(hmax_bt, h);
    }
  }
  GeomDev &gd = t.gd;
  gd.kind = g->kind;
  gd.nx = nx;
  gd.ny = ny;
  gd.nv = nv;
  gd.nu = nu;
  gd.n = (long long)nx * ny;
  gd.m = m;
  gd.du = du;
  gd.D = g->src_dist;
  gd.off = off;
  gd.inv_du = 1.0 / du;
  gd.tan_dg = tan_dg;
  gd.hmax_fan = (1.0 / du) * (1.0 + 1e-5);
  if (fan) {
    // A^T candidates: within asin(|d_dom| / |p - S|) of the pixel's fan angle
    const double rc = std::sqrt(midx * midx + midy * midy);
    const double z = 1.0 / (g->src_dist - rc);
    hmax_at = gd.hmax_fan * z * (1.0 + z * z) + 1e-3;
    gd.dd_spread = (hmax_at + 2.0) * du;
    // |tan| of the largest pixel fan angle (pixel centres within rc of the centre)
    const double tmax = rc / std::sqrt(g->src_dist * g->src_dist - rc * rc);
    gd.fast_atan = tmax <= 0.5 ? 1 : 0;
    // B^T in float: a candidate's source distance differs from the crossing's
    // by e = dpar d / along, where the candidate window (floor(2h) + 1 pixels
    // from ceil(c - h)) gives |d| <= 2h + 1, and the angle to a candidate with
    // a nonzero weight has |tan| <= tan(dg): 1/(1 + e) to second order and
    // atan(z) = z are exact to e^3 + dg^2 / 3 relative
    const double emax = (2.0 * hmax_bt + 1.0) / t.min_along;
    gd.bt_fast = (emax * emax * emax + du * du / 3.0 <= 1e-6) ? 1 : 0;
    // A^T in float: delta_k = |p - S| sin(g_p - g_k) with |g_p - g_k| <= (h + 1) dg
    // over the candidate window; sin(x) = x is exact to x^2 / 6 relative
    const double xmax = (hmax_at + 1.0) * du;
    gd.at_fast = (xmax * xmax / 6.0 <= 1e-6) ? 1 : 0;
    // A: adjacent rays are D dg apart at the centre; below 0.9 pixels the 64
    // rays of a wavefront usually cross a line within 64 pixels (the kernel
    // checks every line)
    gd.fwd_seg = (g->src_dist * du <= 0.9) ? 1 : 0;
  } else if (kFwdSegStage) {
    // parallel beam: adjacent rays cross a line at most sqrt(2) du apart, so
    // the 64 rays of a wavefront fit a 128-element segment while 63 sqrt(2) du
    // stays below 126 (the staged form; the kernel checks every line)
    gd.fwd_seg = (63.0 * std::sqrt(2.0) * du <= 124.0) ? 2 : 0;
  }
  gd.at_vu = kDefaultAtViews;
  gd.b_vu = kDefaultBViews;
  gd.nc_bt = (int)std::floor(2.0 * hmax_bt) + 1;
  gd.nc_at = (int)std::floor(2.0 * hmax_at) + 1;
  gd.pad = gd.nc_bt + (int)std::ceil(hmax_bt) + 2;
  gd.ldR = nx + 2 * gd.pad;
  gd.ldT = ny + 2 * gd.pad;
  gd.offT = (long long)ny * gd.ldR;
  // 128 elements of slack: A's segment loads read up to 126 past the end of a padded line
  gd.pad_elems = gd.offT + (long long)nx * gd.ldT + 128;
  // A's segment path addresses the padded image with 32-bit element offsets
  if (gd.pad_elems >= (1LL << 31)) gd.fwd_seg = 0;
  gd.uclamp_at = hmax_at + 1.0;
  gd.padY = std::max(4, gd.nc_at + (int)std::ceil(2.0 * hmax_at) + 3);
  gd.ldY = nu + 2 * gd.padY;
  gd.ypad_elems = (long long)nv * gd.ldY;
  if (fan) {
    t.gcs.assign(2 * (size_t)gd.ldY, 0.0);
    for (int k = 0; k < gd.ldY; ++k) t.gcs[2 * k] = 1.0;
    for (int k = 0; k < nu; ++k) {
      const double gam = (k - off) * du;
      t.gcs[2 * (gd.padY + k)] = std::cos(gam);
      t.gcs[2 * (gd.padY + k) + 1] = std::sin(gam);
    }
    t.wpad.assign(gd.ypad_elems, 0.0);
    for (int v = 0; v < nv; ++v)
      for (int k = 0; k < nu; ++k) t.wpad[(long long)v * gd.ldY + gd.padY + k] = t.w[(long long)v * nu + k];
    fan_tile_halfwidths(g, ang, t);
  }
  ray_dispatch_orders(t, nu, nv, fan);
}

// Dispatch orders of the ray-driven 2D kernels.  A workgroup lasts as long
// as its longest ray (its wavefronts loop until their last lane is done and
// meet at the closing reduction), and a launch holds more workgroups than the
// GPU runs at once, so the workgroups are issued longest first (the
// longest-processing-time rule): the tail of the launch is then made of short
// ones.  A: workgroup w holds rays 256 w .. 256 w + 255 (ceil(nu / 64) *
// ceil(nv / 4) workgroups); B^T: workgroup w holds bins 64 (w mod T) .. + 63
// of V views from V (w div T), T = ceil(nu / 64): V = 4 (parallel beam) or
// V = 2 with each ray in two halves (fan beam; the key, the longest ray,
// orders them as the longest half would).  Ties keep their index order.
void ray_dispatch_orders(HostTables &t, int nu, int nv, bool fan) {
  const long long m = (long long)nu * nv;
  const int tiles_u = (nu + 63) / 64;
  auto lines = [](int meta) { return std::max(0, ((meta >> 15) & 0x7fff) - (meta & 0x7fff) + 1); };
  std::vector<int> key;
  auto order_by = [&](std::vector<int> &order) {
    const int nblk = (int)key.size();
    order.resize(nblk);
    for (int w = 0; w < nblk; ++w) order[w] = w;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key[a] > key[b]; });
  };
  key.assign(tiles_u * ((nv + 3) / 4), 0);
  for (int w = 0; w < (int)key.size(); ++w) {
    int k = 0;
    for (long long r = (long long)w * 256; r < std::min(m, (long long)w * 256 + 256); ++r) k = std::max(k, lines(t.meta[r]));
    key[w] = k;
  }
  order_by(t.order_fwd);
  const int vpw = fan ? 2 : 4;
  key.assign(tiles_u * ((nv + vpw - 1) / vpw), 0);
  for (int w = 0; w < (int)key.size(); ++w) {
    const int v0 = (w / tiles_u) * vpw, b0 = (w % tiles_u) * 64;
    int k = 0;
    for (int v = v0; v < std::min(nv, v0 + vpw); ++v)
      for (int b = b0; b < std::min(nu, b0 + 64); ++b) k = std::max(k, lines(t.meta_bt[(long long)v * nu + b]));
    key[w] = k;
  }
  order_by(t.order_bt);
}

// Cone beam: per (view, column) the ray's dominant axis and its crossings
// (see ConeTab), formed in double; the direction is built from the detector
// point exactly as P - S with P = S + SDD c + u_k e_u.
void build_cone_tables(const gkb_geometry *g, HostTables &t) {
  const int nx = g->nx, ny = g->ny, nz = g->nz, nv = g->n_views, nu = g->n_det_u, nw = g->n_det_v;
  const double du = g->det_pitch_u, dw = g->det_pitch_v, D = g->src_dist, SDD = g->src_det_dist;
  const double offu = 0.5 * (nu - 1), offw = 0.5 * (nw - 1);
  const double midx = 0.5 * (nx - 1), midy = 0.5 * (ny - 1);
  const std::vector<double> ang = view_angles(g);
  const size_t nvk = (size_t)nv * nu;
  t.cbase1.resize(nvk);
  t.cslope1.resize(nvk);
  t.clmid.resize(nvk);
  t.clslope.resize(nvk);
  t.cdxy2.resize(nvk);
  t.ch1.resize(nvk);
  t.cpk.resize(2 * nvk);
  t.cmeta.resize(nvk);
  t.cmeta_bt.resize(nvk);
  t.p0.resize(nv);
  t.p1.resize(nv);
  t.p2.assign(nv, 0.0);
  t.p3.assign(nv, 0.0);
  t.p4.assign(nv, 0.0);
  double min_ddom = 1e300;
  for (int v = 0; v < nv; ++v) {
    const double cb = std::cos(ang[v]), sb = std::sin(ang[v]);
    t.p0[v] = cb;
    t.p1[v] = sb;
    const double Sx = D * cb, Sy = D * sb;
    for (int k = 0; k < nu; ++k) {
      const size_t vk = (size_t)v * nu + k;
      const double uu = (k - offu) * du;
      const double dx = (Sx + SDD * (-cb) + uu * (-sb)) - Sx;
      const double dy = (Sy + SDD * (-sb) + uu * cb) - Sy;
      const bool ydom = std::fabs(dy) > std::fabs(dx);
      const double Sax = ydom ? Sy : Sx, So = ydom ? Sx : Sy, dax = ydom ? dy : dx, dob = ydom ? dx : dy;
      const int nax = ydom ? ny : nx, n1 = ydom ? nx : ny;
      const double midax = ydom ? midy : midx, mid1 = ydom ? midx : midy;
      min_ddom = std::min(min_ddom, std::fabs(dax));
      const double slope1 = dob / dax;
      const double base1 = So + (0.0 - Sax) / dax * dob + mid1;
      t.cslope1[vk] = slope1;
      t.cbase1[vk] = base1;
      t.clmid[vk] = -Sax / dax;
      t.clslope[vk] = 1.0 / dax;
      t.cdxy2[vk] = dx * dx + dy * dy;
      t.cpk[2 * vk] = 1.0 / dax;
      t.cpk[2 * vk + 1] = ydom ? 1.0 : 0.0;
      // B^T half-width: the in-plane interval whose voxels project within one
      // column of k, evaluated exactly at the first and last plane (it grows
      // monotonically with the depth along the ray)
      double h = 0.0;
      for (int e = 0; e < 2; ++e) {
        const double a = (e ? nax - 1 : 0) - midax;
        const double oc = base1 + a * slope1 - mid1;
        for (int sg = -1; sg <= 1; sg += 2) {
          const double U = (k + sg - offu) * du / SDD;
          const double den = ydom ? (-sb + U * cb) : (cb + U * sb);
          if (std::fabs(den) < 1e-12) {
            h = std::max(h, (double)n1 + 2.0);
            continue;
          }
          const double o = ydom ? (U * (D - a * sb) - a * cb) / den : (U * (D - a * cb) + a * sb) / den;
          h = std::max(h, std::fabs(o - oc));
        }
      }
      h = std::min(h * 1.0001 + 1e-3, (double)n1 + 2.0);
      t.ch1[vk] = h;
      int lo, hi;
      line_range(base1, slope1, midax, nax, -1.0, (double)n1, lo, hi);
      t.cmeta[vk] = lo | (hi << 15) | ((ydom ? 1 : 0) << 30);
      line_range(base1, slope1, midax, nax, -h, n1 - 1 + h, lo, hi);
      t.cmeta_bt[vk] = lo | (hi << 15) | ((ydom ? 1 : 0) << 30);
      if (ydom)
        t.has_ydom = true;
      else
        t.has_xdom = true;
    }
  }
  t.min_ddom = min_ddom;
  GeomDev &gd = t.gd;
  gd.kind = GKB_CONE3D;
  gd.nx = nx;
  gd.ny = ny;
  gd.nz = nz;
  gd.nv = nv;
  gd.nu = nu;
  gd.nw = nw;
  gd.n = (long long)nx * ny * nz;
  gd.m = (long long)nv * nw * nu;
  gd.du = du;
  gd.dw = dw;
  gd.D = D;
  gd.SDD = SDD;
  gd.off = offu;
  gd.offw = offw;
  gd.inv_du = 1.0 / du;
  gd.Su = SDD / du;
  gd.Sw = SDD / dw;
  gd.hk_fac = std::sqrt(SDD * SDD + (offu * du) * (offu * du)) / du * (1.0 + 1e-6);
  gd.nc_bt = 2;
  gd.nc_at = 2;
  gd.P3 = 2;
  gd.dmax3 = D + std::hypot(midx + gd.P3 + 1.0, midy + gd.P3 + 1.0);
  gd.ldX = ny + 2 * gd.P3;
  gd.ldV = nx + 2 * gd.P3;
  gd.planeX = (long long)(nz + 2 * gd.P3) * gd.ldX;
  gd.planeY = (long long)(nz + 2 * gd.P3) * gd.ldV;
  gd.offYD = (long long)nx * gd.planeX;
  gd.vol_pad_elems = gd.offYD + (long long)ny * gd.planeY;
  gd.PY3 = 2;
  gd.ldSu = nu + 2 * gd.PY3;
  gd.sliceY = (long long)(nw + 2 * gd.PY3) * gd.ldSu;
  gd.sino_pad_elems = (long long)nv * gd.sliceY;
  gd.pad_elems = gd.vol_pad_elems;
  gd.ypad_elems = std::max(gd.sino_pad_elems, gd.m);
}

}  // namespace gkb

namespace {

struct DevTables {
  DevBuf buf;
  RayTab<float> rt32{};
  ViewTab<float> vt32{};
  RayTab<double> rt64{};
  ViewTab<double> vt64{};
  ConeTab<float> ct32{};
  ConeTab<double> ct64{};
  bool has_coldom = false;
  bool has_xdom = false, has_ydom = false;
  GeomDev gd{};
};

template <typename T>
hipError_t upload_cone_tables(const HostTables &h, DevTables &d) {
  const size_t nvk = h.cbase1.size();
  const int nv = h.gd.nv;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t aT = al(sizeof(T) * nvk), aI = al(sizeof(int) * nvk), aV = al(sizeof(T) * nv);
  const size_t total = 6 * aT + 2 * aT + 2 * aI + 2 * aV;
  hipError_t e = d.buf.ensure(total);
  if (e != hipSuccess) return e;
  char *p = d.buf.as<char>();
  std::vector<T> tmp;
  auto put = [&](const std::vector<double> &src, size_t stride) -> const T * {
    T *dst = reinterpret_cast<T *>(p);
    p += stride;
    tmp.assign(src.size(), T(0));
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
    (void)hipMemcpy(dst, tmp.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return dst;
  };
  auto put_i = [&](const std::vector<int> &src) -> const int * {
    int *dst = reinterpret_cast<int *>(p);
    p += aI;
    (void)hipMemcpy(dst, src.data(), sizeof(int) * src.size(), hipMemcpyHostToDevice);
    return dst;
  };
  ConeTab<T> ct{};
  ViewTab<T> vt{};
  ct.base1 = put(h.cbase1, aT);
  ct.slope1 = put(h.cslope1, aT);
  ct.lmid = put(h.clmid, aT);
  ct.lslope = put(h.clslope, aT);
  ct.dxy2 = put(h.cdxy2, aT);
  ct.h1 = put(h.ch1, aT);
  ct.pk = put(h.cpk, 2 * aT);
  ct.meta = put_i(h.cmeta);
  ct.meta_bt = put_i(h.cmeta_bt);
  vt.p0 = put(h.p0, aV);
  vt.p1 = put(h.p1, aV);
  if constexpr (sizeof(T) == 4) {
    d.ct32 = ct;
    d.vt32 = vt;
  } else {
    d.ct64 = ct;
    d.vt64 = vt;
  }
  d.has_xdom = h.has_xdom;
  d.has_ydom = h.has_ydom;
  d.gd = h.gd;
  return hipGetLastError();
}

template <typename T>
hipError_t upload_tables(const HostTables &h, DevTables &d) {
  const long long m = h.gd.m;
  const int nv = h.gd.nv;
  const bool fan = h.gd.kind == GKB_FAN2D;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t rayT = al(sizeof(T) * m), rayI = al(sizeof(int) * m), viewT = al(sizeof(T) * nv),
               binT = al(sizeof(T) * 2 * h.gd.ldY), wpT = al(sizeof(T) * (fan ? h.gd.ypad_elems : 1)),
               tileT = al(sizeof(T) * std::max<size_t>(h.htile.size(), 1));
  const size_t total = 8 * rayT + 4 * rayI + 5 * viewT + binT + wpT + tileT;
  hipError_t e = d.buf.ensure(total);
  if (e != hipSuccess) return e;
  char *p = d.buf.as<char>();
  std::vector<T> tmp;
  auto put = [&](const std::vector<double> &src, size_t stride) -> const T * {
    T *dst = reinterpret_cast<T *>(p);
    p += stride;
    if (src.empty()) return dst;
    tmp.assign(src.size(), T(0));
    for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
    (void)hipMemcpy(dst, tmp.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return dst;
  };
  auto put_i = [&](const std::vector<int> &src) -> const int * {
    int *dst = reinterpret_cast<int *>(p);
    p += rayI;
    (void)hipMemcpy(dst, src.data(), sizeof(int) * src.size(), hipMemcpyHostToDevice);
    return dst;
  };
  RayTab<T> rt{};
  ViewTab<T> vt{};
  rt.base = put(h.base, rayT);
  rt.slope = put(h.slope, rayT);
  rt.w = put(h.w, rayT);
  rt.h = put(h.h, rayT);
  rt.t0 = put(h.t0, rayT);
  rt.dt = put(h.dt, rayT);
  rt.dperp = put(h.dperp, rayT);
  rt.dpar = put(h.dpar, rayT);
  rt.meta = put_i(h.meta);
  rt.meta_bt = put_i(h.meta_bt);
  rt.order_fwd = put_i(h.order_fwd);
  rt.order_bt = put_i(h.order_bt);
  vt.p0 = put(h.p0, viewT);
  vt.p1 = put(h.p1, viewT);
  vt.p2 = put(h.p2, viewT);
  vt.p3 = put(h.p3, viewT);
  vt.p4 = put(h.p4, viewT);
  vt.gcos = put(h.gcs, binT);
  rt.wpad = put(h.wpad, wpT);
  vt.htile = put(h.htile, tileT);
  if constexpr (sizeof(T) == 4) {
    d.rt32 = rt;
    d.vt32 = vt;
  } else {
    d.rt64 = rt;
    d.vt64 = vt;
  }
  d.has_coldom = h.has_coldom;
  d.gd = h.gd;
  return hipGetLastError();
}

std::string geom_key(const gkb_geometry *g, int dtype) {
  std::string k;
  char buf[256];
  snprintf(buf, sizeof buf, "%d|%d|%d|%d|%d|%d|%d|%d|%.17g|%.17g|%.17g|%.17g|%.17g|%d|", g->kind, g->nx, g->ny,
           g->nz, g->n_views, g->n_det_u, g->n_det_v, dtype, g->angle_span, g->det_pitch_u, g->det_pitch_v,
           g->src_dist, g->src_det_dist, g->angles ? 1 : 0);
  k = buf;
  if (g->angles) {
    k.append(reinterpret_cast<const char *>(g->angles), sizeof(double) * g->n_views);
  }
  return k;
}

// --------------------------------------------------------------------------
// tracing
// --------------------------------------------------------------------------
struct TraceStat {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  int count = 0;
  double ms = 0.0;
};

}  // namespace

// --------------------------------------------------------------------------
// context
// --------------------------------------------------------------------------
struct gkb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::map<std::string, std::unique_ptr<DevTables>> tables;
  // host-side geometry of gkb_back_noalloc: layout scalars and the view
  // constants staged as they are copied into the device scratch array
  struct NoallocGeom {
    GeomDev gd{};
    size_t off_p1 = 0, off_y = 0;          // byte offsets of p1 and the padded sinogram
    std::vector<unsigned char> staged;     // [p0 | p1] in the dtype, off_y bytes
  };
  std::map<std::string, std::unique_ptr<NoallocGeom>> noalloc_geoms;
  // scratch for standalone projector calls and reductions
  DevBuf xpad, ypad, partials;
  DevBuf ywpad;  // fan-beam A^T input as (w y, w) pairs, apart from ypad so that neither layout overwrites the other's pads
  // solve workspace
  DevBuf Q, yk, rdbl, s, w, tmp_n, tmp_m, ctl_d, ctl_i;
  DevBuf gm_y, gm_h;  // GMRES and hybrid GKB: the A-images Y; GMRES: the Hessenberg columns
  DevBuf hy_w;        // enlarged-subspace TSVD: Jacobi workspace (W, V)
  DevBuf gram;        // Gram matrix of the Krylov basis (delayed second Gram-Schmidt round)
  int *host_flag = nullptr;      // host-mapped
  int *host_flag_dev = nullptr;  // its device address
  // batched solves: vectors, control blocks, slice descriptors, launch maps
  DevBuf bws, bwd, bwi, bsd, bmap, brep;
  int *bflags = nullptr, *bflags_dev = nullptr;  // host-mapped stop mirrors, one per slice
  int bflags_n = 0;
  int *bpin = nullptr;  // pinned staging of launch maps: two slots
  size_t bpin_slot = 0;
  hipEvent_t bpin_ev[2] = {nullptr, nullptr};
  // learned filter: activations, masks, filter output, training buffers
  DevBuf na0, na1, na2, nga, ngb, nmask, nout, ngout, nxh, nr, npart, nsums, nred, ny;
  // batched solves: 1 = every iteration's launches captured in a hipGraph
  // (re-captured when the set of active slices changes) and replayed
  int batch_graph = 0;
  hipStream_t cap_stream = nullptr;  // capture stream (created on first use)
  // tracing
  bool trace = false;
  std::string trace_only;  // non-empty: record only this kernel name
  std::map<std::string, TraceStat> stats;
  std::vector<hipEvent_t> event_pool;

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void flush_trace() {
    for (auto &kv : stats) {
      for (auto &pr : kv.second.pending) {
        float ms = 0.f;
        (void)hipEventSynchronize(pr.second);
        (void)hipEventElapsedTime(&ms, pr.first, pr.second);
        kv.second.ms += ms;
        kv.second.count += 1;
        event_pool.push_back(pr.first);
        event_pool.push_back(pr.second);
      }
      kv.second.pending.clear();
    }
  }
};

namespace {

struct TraceScope {
  gkb_ctx *c;
  const char *name;
  hipEvent_t a = nullptr;
  TraceScope(gkb_ctx *ctx, const char *n) : c(ctx), name(n) {
    if (c->trace && (c->trace_only.empty() || c->trace_only == n)) {
      a = c->get_event();
      (void)hipEventRecord(a, c->stream);
    }
  }
  ~TraceScope() {
    if (a) {
      hipEvent_t b = c->get_event();
      (void)hipEventRecord(b, c->stream);
      c->stats[name].pending.emplace_back(a, b);
    }
  }
};

gkb_status validate_geom(const gkb_geometry *g, int dtype) {
  if (!g) return fail(GKB_EINVAL, "geometry is NULL");
  if (dtype != GKB_F32 && dtype != GKB_F64) return fail(GKB_EINVAL, "dtype must be GKB_F32 or GKB_F64");
  if (g->kind == GKB_CONE3D) {
    if (g->nx < 1 || g->ny < 1 || g->nz < 1 || g->nx > 16384 || g->ny > 16384 || g->nz > 16384)
      return fail(GKB_EINVAL, "nx, ny, nz must be in [1, 16384]");
    if (g->n_views < 1) return fail(GKB_EINVAL, "n_views must be >= 1");
    if (g->n_det_u < 1 || g->n_det_v < 1) return fail(GKB_EINVAL, "n_det_u and n_det_v must be >= 1");
    if (!(g->det_pitch_u > 0.0) || !std::isfinite(g->det_pitch_u) || !(g->det_pitch_v > 0.0) ||
        !std::isfinite(g->det_pitch_v))
      return fail(GKB_EINVAL, "detector pitches must be > 0");
    if (!g->angles && !std::isfinite(g->angle_span)) return fail(GKB_EINVAL, "angle_span must be finite");
    if (g->angles)
      for (int v = 0; v < g->n_views; ++v)
        if (!std::isfinite(g->angles[v])) return fail(GKB_EINVAL, "angles must be finite");
    const double half_diag = 0.5 * std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny);
    if (!(g->src_dist > half_diag + 2.0) || !std::isfinite(g->src_dist))
      return fail(GKB_EINVAL, "cone beam: src_dist must exceed the volume's half-diagonal + 2");
    if (!(g->src_det_dist > 0.0) || !std::isfinite(g->src_det_dist))
      return fail(GKB_EINVAL, "cone beam: src_det_dist must be > 0");
    return GKB_OK;
  }
  if (g->kind != GKB_PAR2D && g->kind != GKB_FAN2D) return fail(GKB_EINVAL, "unknown geometry kind");
  if (g->nx < 1 || g->ny < 1 || g->nx > 16384 || g->ny > 16384)
    return fail(GKB_EINVAL, "nx, ny must be in [1, 16384]");
  if (g->nz != 1 && g->nz != 0) return fail(GKB_EINVAL, "nz must be 1 for 2D geometry");
  if (g->n_views < 1) return fail(GKB_EINVAL, "n_views must be >= 1");
  if (g->n_det_u < 1 || (g->n_det_v != 1 && g->n_det_v != 0))
    return fail(GKB_EINVAL, "n_det_u must be >= 1 and n_det_v 1 for 2D geometry");
  if (!(g->det_pitch_u > 0.0) || !std::isfinite(g->det_pitch_u)) return fail(GKB_EINVAL, "det_pitch_u must be > 0");
  if (!g->angles && !std::isfinite(g->angle_span)) return fail(GKB_EINVAL, "angle_span must be finite");
  if (g->angles)
    for (int v = 0; v < g->n_views; ++v)
      if (!std::isfinite(g->angles[v])) return fail(GKB_EINVAL, "angles must be finite");
  if (g->kind == GKB_FAN2D) {
    const double half_diag = 0.5 * std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny);
    if (!(g->src_dist > half_diag + 2.0))
      return fail(GKB_EINVAL, "fan beam: src_dist must exceed the image half-diagonal + 2");
    if (!(g->det_pitch_u * g->n_det_u < 3.0)) return fail(GKB_EINVAL, "fan beam: fan angle must be < 3 rad");
  }
  return GKB_OK;
}

gkb_status get_tables(gkb_ctx *c, const gkb_geometry *g, int dtype, DevTables **out) {
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  const std::string key = geom_key(g, dtype);
  auto it = c->tables.find(key);
  if (it != c->tables.end()) {
    *out = it->second.get();
    return GKB_OK;
  }
  HostTables h;
  if (g->kind == GKB_CONE3D) {
    build_cone_tables(g, h);
    if (!(h.min_ddom > 0.5 * (g->n_det_v - 1) * g->det_pitch_v))
      return fail(GKB_EUNSUPPORTED, "cone beam: some ray would step along z (detector too tall for the "
                                    "source-detector distance)");
    if (h.gd.vol_pad_elems >= (1LL << 32) || h.gd.sino_pad_elems >= (1LL << 32))
      return fail(GKB_EUNSUPPORTED, "volume or sinogram too large for 32-bit offsets");
    auto d = std::make_unique<DevTables>();
    hipError_t e = (dtype == GKB_F32) ? upload_cone_tables<float>(h, *d) : upload_cone_tables<double>(h, *d);
    if (e == hipErrorOutOfMemory) return fail(GKB_ENOMEM, "out of device memory for geometry tables");
    if (e != hipSuccess) return fail(GKB_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
    *out = d.get();
    c->tables.emplace(key, std::move(d));
    return GKB_OK;
  }
  build_tables(g, h);
  if (h.gd.nc_bt > 8 || h.gd.nc_at > 8)
    return fail(GKB_EUNSUPPORTED, "detector pitch too fine relative to the pixel pitch (more than 8 "
                                  "interpolation candidates per line)");
  if (h.gd.pad_elems >= (1LL << 31) || h.gd.ypad_elems >= (1LL << 31))
    return fail(GKB_EUNSUPPORTED, "image or sinogram too large for 32-bit offsets");
  auto d = std::make_unique<DevTables>();
  hipError_t e = (dtype == GKB_F32) ? upload_tables<float>(h, *d) : upload_tables<double>(h, *d);
  if (e == hipErrorOutOfMemory) return fail(GKB_ENOMEM, "out of device memory for geometry tables");
  if (e != hipSuccess) return fail(GKB_EDEVICE, std::string("table upload: ") + hipGetErrorString(e));
  *out = d.get();
  c->tables.emplace(key, std::move(d));
  return GKB_OK;
}

template <typename T>
const RayTab<T> &rt_of(const DevTables &d);
template <>
const RayTab<float> &rt_of<float>(const DevTables &d) {
  return d.rt32;
}
template <>
const RayTab<double> &rt_of<double>(const DevTables &d) {
  return d.rt64;
}
template <typename T>
const ViewTab<T> &vt_of(const DevTables &d);
template <>
const ViewTab<float> &vt_of<float>(const DevTables &d) {
  return d.vt32;
}
template <>
const ViewTab<double> &vt_of<double>(const DevTables &d) {
  return d.vt64;
}

template <typename T>
const ConeTab<T> &ct_of(const DevTables &d);
template <>
const ConeTab<float> &ct_of<float>(const DevTables &d) {
  return d.ct32;
}
template <>
const ConeTab<double> &ct_of<double>(const DevTables &d) {
  return d.ct64;
}

template <typename T>
Col<T> col(T *p) {
  return Col<T>{p, 0, 0, nullptr};
}
template <typename T>
Col<T> colk(T *base, long long ld, int off, const int *kptr) {
  return Col<T>{base, ld, off, kptr};
}

template <typename T>
Epi<T> plain_epi() {
  Epi<T> e{};
  e.use_ctl = 0;
  e.in_sel = IN_ONE;
  e.prev_sel = PREV_NONE;
  e.norm_to_t = 0;
  e.prev = Col<const T>{nullptr, 0, 0, nullptr};
  e.out_raw = Col<T>{nullptr, 0, 0, nullptr};
  return e;
}

gkb_status ensure_scratch(gkb_ctx *c, const GeomDev &g, size_t elem, long long nblocks_times_cols) {
  HIPC(c->xpad.ensure(elem * (size_t)g.pad_elems));
  HIPC(c->ypad.ensure(2 * elem * (size_t)g.ypad_elems));
  if (g.kind == GKB_FAN2D) HIPC(c->ywpad.ensure(2 * elem * (size_t)g.ypad_elems));
  HIPC(c->partials.ensure(sizeof(double) * std::max<long long>(nblocks_times_cols, 1024)));
  return GKB_OK;
}

// ----- standalone projector application -----
enum Op { OP_A = 0, OP_B = 1, OP_AT = 2, OP_BT = 3 };

template <typename T>
gkb_status apply_op(gkb_ctx *c, const DevTables &d, int op, const void *in, void *out) {
  const GeomDev &g = d.gd;
  const long long nb = std::max<long long>({(long long)ray_blocks(g), (long long)bt_blocks(g), (long long)pixel_blocks(g), 1LL});
  gkb_status st = ensure_scratch(c, g, sizeof(T), nb);
  if (st != GKB_OK) return st;
  Epi<T> e = plain_epi<T>();
  const T *xi = static_cast<const T *>(in);
  T *xo = static_cast<T *>(out);
  T *xpad = c->xpad.as<T>();
  T *ypad = c->ypad.as<T>();
  if (g.kind == GKB_CONE3D) {
    hipStream_t st = c->stream;
    switch (op) {
      case OP_A: {
        launch_cone_pad_volume<T>(g, col<const T>(xi), xpad, d.has_xdom, d.has_ydom, nullptr, st);
        TraceScope ts(c, "fwd");
        launch_cone_fwd<T>(g, ct_of<T>(d), xpad, col<T>(xo), e, nullptr, st);
        break;
      }
      case OP_BT: {
        launch_cone_pad_volume<T>(g, col<const T>(xi), xpad, d.has_xdom, d.has_ydom, nullptr, st);
        TraceScope ts(c, "back_adj");
        launch_cone_back_adj<T>(g, ct_of<T>(d), vt_of<T>(d), xpad, col<T>(xo), e, nullptr, st);
        break;
      }
      case OP_B: {
        launch_cone_pad_sino<T>(g, col<const T>(xi), ypad, nullptr, st);
        TraceScope ts(c, "back");
        launch_cone_back<T>(g, vt_of<T>(d), ypad, xo, e, nullptr, st);
        break;
      }
      case OP_AT: {
        launch_cone_weight_sino<T>(g, ct_of<T>(d), col<const T>(xi), ypad, nullptr, st);
        TraceScope ts(c, "fwd_adj");
        launch_cone_fwd_adj<T>(g, ct_of<T>(d), vt_of<T>(d), ypad, xo, e, nullptr, st);
        break;
      }
    }
    HIPC(hipGetLastError());
    return GKB_OK;
  }
  switch (op) {
    case OP_A: {
      launch_pad_image<T>(g, col<const T>(xi), xpad, d.has_coldom, nullptr, c->stream);
      TraceScope ts(c, "fwd");
      launch_fwd<T>(g, rt_of<T>(d), xpad, col<T>(xo), e, nullptr, c->stream);
      break;
    }
    case OP_BT: {
      launch_pad_image<T>(g, col<const T>(xi), xpad, d.has_coldom, nullptr, c->stream);
      TraceScope ts(c, "back_adj");
      launch_back_adj<T>(g, rt_of<T>(d), xpad, col<T>(xo), e, nullptr, c->stream);
      break;
    }
    case OP_B: {
      launch_pad_sino<T>(g, col<const T>(xi), ypad, nullptr, c->stream);
      TraceScope ts(c, "back");
      launch_back<T>(g, vt_of<T>(d), ypad, xo, e, nullptr, c->stream);
      break;
    }
    case OP_AT: {
      launch_pad_sino_adj<T>(g, rt_of<T>(d), col<const T>(xi), ypad, nullptr, c->stream);
      TraceScope ts(c, "fwd_adj");
      launch_fwd_adj<T>(g, vt_of<T>(d), rt_of<T>(d), ypad, xo, e, nullptr, c->stream);
      break;
    }
  }
  HIPC(hipGetLastError());
  return GKB_OK;
}

gkb_status projector_call(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *in, void *out, int op) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!in || !out) return fail(GKB_EINVAL, "data pointer is NULL");
  DevTables *d = nullptr;
  gkb_status st = get_tables(c, g, dtype, &d);
  if (st != GKB_OK) return st;
  HIPC(hipSetDevice(c->device));
  return dtype == GKB_F32 ? apply_op<float>(c, *d, op, in, out) : apply_op<double>(c, *d, op, in, out);
}

// ----- autotuning of the launch choices -----
// Parallel beam: A^T with 1, 2 and 4 views per step and B with 4 and 8 are
// timed (HIP events, mean of five launches after one warm-up) on a constant
// sinogram of the geometry, and the fastest of each is kept in the
// geometry's tables, where every later call, solve and batch takes it from.
// The choices change the order of loads, not of any sum.
template <typename T>
gkb_status autotune_impl(gkb_ctx *c, DevTables &d, gkb_tuning *out) {
  GeomDev &g = d.gd;
  gkb_tuning t{};
  for (double &v : t.at_us) v = 0.0;
  for (double &v : t.b_us) v = 0.0;
  if (g.kind == GKB_PAR2D) {
    const long long nb = std::max<long long>({(long long)ray_blocks(g), (long long)bt_blocks(g), (long long)pixel_blocks(g), 1LL});
    gkb_status st = ensure_scratch(c, g, sizeof(T), nb);
    if (st != GKB_OK) return st;
    HIPC(c->tmp_m.ensure(sizeof(T) * (size_t)g.m));
    HIPC(c->tmp_n.ensure(sizeof(T) * (size_t)g.n));
    T *y = c->tmp_m.as<T>(), *x = c->tmp_n.as<T>(), *ypad = c->ypad.as<T>();
    HIPC(hipMemsetAsync(y, 0x3c, sizeof(T) * (size_t)g.m, c->stream));
    launch_pad_sino<T>(g, col<const T>(y), ypad, nullptr, c->stream);
    hipEvent_t e0 = c->get_event(), e1 = c->get_event();
    auto time_it = [&](auto launch) -> double {
      launch();
      (void)hipEventRecord(e0, c->stream);
      for (int r = 0; r < 5; ++r) launch();
      (void)hipEventRecord(e1, c->stream);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      return 1e3 * ms / 5.0;
    };
    const Epi<T> e = plain_epi<T>();
    const int at_cand[3] = {1, 2, 4}, b_cand[2] = {4, 8};
    int best_at = g.at_vu, best_b = g.b_vu;
    double bt = 1e300, bb = 1e300;
    for (int i = 0; i < 3; ++i) {
      g.at_vu = at_cand[i];
      t.at_us[i] = time_it([&]() { launch_fwd_adj<T>(g, vt_of<T>(d), rt_of<T>(d), ypad, x, e, nullptr, c->stream); });
      if (t.at_us[i] < bt) {
        bt = t.at_us[i];
        best_at = at_cand[i];
      }
    }
    for (int i = 0; i < 2; ++i) {
      g.b_vu = b_cand[i];
      t.b_us[i] = time_it([&]() { launch_back<T>(g, vt_of<T>(d), ypad, x, e, nullptr, c->stream); });
      if (t.b_us[i] < bb) {
        bb = t.b_us[i];
        best_b = b_cand[i];
      }
    }
    c->event_pool.push_back(e0);
    c->event_pool.push_back(e1);
    HIPC(hipGetLastError());
    g.at_vu = best_at;
    g.b_vu = best_b;
  }
  t.at_views_per_step = g.at_vu;
  t.b_views_per_step = g.b_vu;
  if (out) *out = t;
  return GKB_OK;
}

gkb_status autotune(gkb_ctx *c, const gkb_geometry *geom, int dtype, gkb_tuning *out) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  DevTables *d = nullptr;
  gkb_status st = get_tables(c, geom, dtype, &d);
  if (st != GKB_OK) return st;
  HIPC(hipSetDevice(c->device));
  return dtype == GKB_F32 ? autotune_impl<float>(c, *d, out) : autotune_impl<double>(c, *d, out);
}

gkb_status set_tuning(gkb_ctx *c, const gkb_geometry *geom, int dtype, const gkb_tuning *t) {
  if (!c || !t) return fail(GKB_EINVAL, "NULL argument");
  if (t->at_views_per_step != 1 && t->at_views_per_step != 2 && t->at_views_per_step != 4)
    return fail(GKB_EINVAL, "A^T views per step must be 1, 2 or 4");
  if (t->b_views_per_step != 4 && t->b_views_per_step != 8) return fail(GKB_EINVAL, "B views per step must be 4 or 8");
  DevTables *d = nullptr;
  gkb_status st = get_tables(c, geom, dtype, &d);
  if (st != GKB_OK) return st;
  d->gd.at_vu = t->at_views_per_step;
  d->gd.b_vu = t->b_views_per_step;
  return GKB_OK;
}

// ----- allocation-free back projection -----
// gkb_back_noalloc runs the same padding and B kernels as gkb_back, with their
// scratch (the per-view constants and the padded sinogram) in the file-scope
// device array `scratch` instead of context buffers, so that the call
// allocates no device memory.  Every GPU the library runs on holds one copy of
// the array until the process ends; host code reaches it only through the
// per-device address resolved in gkb_create.  Calls that overlap on one GPU
// (from any context or stream) share the array and race.
constexpr size_t kNoallocBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

// The calling thread's current device must be `device`.
gkb_status resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(GKB_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return GKB_OK;
  void *ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(GKB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return GKB_OK;
}

template <typename T>
gkb_status back_noalloc_impl(gkb_ctx *c, const gkb_geometry *g, int dtype, const T *y, T *x) {
  const std::string key = geom_key(g, dtype);
  auto it = c->noalloc_geoms.find(key);
  if (it == c->noalloc_geoms.end()) {
    HostTables h;
    build_tables(g, h);
    if (h.gd.nc_bt > 8 || h.gd.nc_at > 8)
      return fail(GKB_EUNSUPPORTED, "detector pitch too fine relative to the pixel pitch (more than 8 "
                                    "interpolation candidates per line)");
    if (h.gd.ypad_elems >= (1LL << 31)) return fail(GKB_EUNSUPPORTED, "sinogram too large for 32-bit offsets");
    auto na = std::make_unique<gkb_ctx::NoallocGeom>();
    na->gd = h.gd;
    const size_t vb = al256_bytes(sizeof(T) * (size_t)h.gd.nv);
    na->off_p1 = vb;
    na->off_y = 2 * vb;
    na->staged.assign(na->off_y, 0);
    T *p0 = reinterpret_cast<T *>(na->staged.data());
    T *p1 = reinterpret_cast<T *>(na->staged.data() + na->off_p1);
    for (int v = 0; v < h.gd.nv; ++v) {
      p0[v] = (T)h.p0[v];
      p1[v] = (T)h.p1[v];
    }
    it = c->noalloc_geoms.emplace(key, std::move(na)).first;
  }
  const gkb_ctx::NoallocGeom &na = *it->second;
  const GeomDev &gd = na.gd;
  const size_t need = na.off_y + sizeof(T) * (size_t)gd.ypad_elems;
  if (need > kNoallocBytes)
    return fail(GKB_EINVAL, "gkb_back_noalloc: the geometry needs " + std::to_string(need) +
                                " bytes of scratch, more than the fixed " + std::to_string(kNoallocBytes) +
                                " (views x (detector bins + padding) too large)");
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    base = g_scratch_ptr[c->device];
  }
  if (!base) return fail(GKB_EDEVICE, "gkb_back_noalloc: scratch address not resolved for this device");
  unsigned char *sb = static_cast<unsigned char *>(base);
  HIPC(hipMemcpyAsync(sb, na.staged.data(), na.off_y, hipMemcpyHostToDevice, c->stream));
  ViewTab<T> vt{};
  vt.p0 = reinterpret_cast<const T *>(sb);
  vt.p1 = reinterpret_cast<const T *>(sb + na.off_p1);
  T *ypad = reinterpret_cast<T *>(sb + na.off_y);
  // every element of the padded sinogram is written here (the pads as zeros)
  launch_pad_sino<T>(gd, col<const T>(y), ypad, nullptr, c->stream);
  launch_back<T>(gd, vt, ypad, x, plain_epi<T>(), nullptr, c->stream);
  HIPC(hipGetLastError());
  return GKB_OK;
}

gkb_status back_noalloc(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *y, void *x) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!y || !x) return fail(GKB_EINVAL, "data pointer is NULL");
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  if (g->kind == GKB_CONE3D) return fail(GKB_EUNSUPPORTED, "gkb_back_noalloc: 2D geometries only");
  HIPC(hipSetDevice(c->device));
  return dtype == GKB_F32
             ? back_noalloc_impl<float>(c, g, dtype, static_cast<const float *>(y), static_cast<float *>(x))
             : back_noalloc_impl<double>(c, g, dtype, static_cast<const double *>(y), static_cast<double *>(x));
}

// --------------------------------------------------------------------------
// learned sinogram filter: network object, filter chains, training
// --------------------------------------------------------------------------
}  // namespace

struct gkb_net {
  int device = 0;
  DevBuf W, m, v, grad, prep;  // master weights, Adam state, gradient, derived layouts
  NetW nw{};
  int step = 0;
};

namespace {

constexpr long long kOffW2 = (long long)kNetC * kNetK, kOffW3 = kOffW2 + (long long)kNetC * kNetC * kNetK,
                    kOffW4 = kOffW3 + (long long)kNetC * kNetC * kNetK;

gkb_status net_prepare(gkb_net *net, hipStream_t st) {
  launch_net_prep(net->W.as<float>(), net->nw, st);
  HIPC(hipGetLastError());
  return GKB_OK;
}

// rows (views x detector rows) and columns of a geometry's sinogram
void net_shape(const gkb_geometry *g, long long &rows, int &L) {
  rows = (long long)g->n_views * (g->kind == GKB_CONE3D ? g->n_det_v : 1);
  L = g->n_det_u;
}

// positions per chunk of the filter chains (two activation buffers of
// 32 floats per position)
constexpr long long kNetChunk = 1LL << 23;

gkb_status net_scratch(gkb_ctx *c, long long rows, int L) {
  const long long per = std::min(rows, std::max(1LL, kNetChunk / L)) * L;
  HIPC(c->na0.ensure(sizeof(float) * kNetC * (size_t)per));
  HIPC(c->na1.ensure(sizeof(float) * kNetC * (size_t)per));
  HIPC(c->nmask.ensure(sizeof(unsigned) * 3 * (size_t)(rows * L)));
  HIPC(c->nout.ensure(sizeof(float) * (size_t)(rows * L)));
  return GKB_OK;
}

enum NetOp { NET_MASKS = 0, NET_F = 1, NET_FT = 2 };

// NET_MASKS: out = N(y) and the frozen masks of y; NET_F: out = F y;
// NET_FT: out = F^T y (the masks as last computed).  Rows in chunks.
void net_chain(gkb_ctx *c, const gkb_net *net, int op, Col<const float> y, float *out, long long rows, int L,
               const int *stop, hipStream_t st) {
  const long long m = rows * L;
  const long long crow = std::max(1LL, kNetChunk / L);
  float *a0 = c->na0.as<float>(), *a1 = c->na1.as<float>();
  unsigned *masks = c->nmask.as<unsigned>();
  const NetW &w = net->nw;
  for (long long r0 = 0; r0 < rows; r0 += crow) {
    const long long nr = std::min(crow, rows - r0);
    const long long off = r0 * L;
    Col<const float> yin{y.base + off, y.ld, y.off, y.kptr};
    unsigned *m0 = masks + off, *m1 = masks + m + off, *m2 = masks + 2 * m + off;
    if (op == NET_MASKS) {
      launch_net_c1(yin, a0, m0, w.w1, L, nr, 1, stop, st);
      launch_net_c32(a0, a1, m1, w.w2b, L, nr, 3, 1, stop, st);
      launch_net_c32(a1, a0, m2, w.w3b, L, nr, 3, 1, stop, st);
      launch_net_c4(a0, out + off, w.w4, L, nr, stop, st);
    } else if (op == NET_F) {
      launch_net_c1(yin, a0, m0, w.w1, L, nr, 2, stop, st);
      launch_net_c32(a0, a1, m1, w.w2b, L, nr, 3, 2, stop, st);
      launch_net_c32(a1, a0, m2, w.w3b, L, nr, 3, 2, stop, st);
      launch_net_c4(a0, out + off, w.w4, L, nr, stop, st);
    } else {
      launch_net_c1(yin, a0, m2, w.w4t, L, nr, 2, stop, st);
      launch_net_c32(a0, a1, m1, w.w3t, L, nr, 3, 2, stop, st);
      launch_net_c32(a1, a0, m0, w.w2t, L, nr, 3, 2, stop, st);
      launch_net_c4(a0, out + off, w.w1t, L, nr, stop, st);
    }
  }
}

// He initialisation N(0, 2 / fan_in) from a counter-based generator:
// SplitMix64 (Steele, Lea and Flood 2014) for uniform 53-bit numbers,
// Box-Muller for the normal deviates.
void he_init(unsigned long long seed, std::vector<float> &w) {
  auto mix = [](uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  };
  auto unif = [&](uint64_t i) { return ((mix(seed * 0x100000001B3ULL + i) >> 11) + 0.5) * (1.0 / 9007199254740992.0); };
  const double pi = 3.14159265358979323846;
  w.resize(kNetParams);
  for (int i = 0; i < kNetParams; ++i) {
    const double fan_in = (i < kOffW2) ? kNetK : (double)kNetC * kNetK;
    const double u1 = unif(2 * (uint64_t)i), u2 = unif(2 * (uint64_t)i + 1);
    const double g = std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * pi * u2);
    w[i] = (float)(g * std::sqrt(2.0 / fan_in));
  }
}

// gradient of the mean training loss over a batch of S sinograms b [S][m]
// and targets x [S][n] (2D geometry); optional Adam step
gkb_status net_grad_impl(gkb_ctx *c, gkb_net *net, const gkb_geometry *g, int S, const float *b, const float *x,
                         int objective, double *loss_out) {
  DevTables *d = nullptr;
  gkb_status stt = get_tables(c, g, GKB_F32, &d);
  if (stt != GKB_OK) return stt;
  const GeomDev &gd = d->gd;
  hipStream_t st = c->stream;
  const long long mS = gd.m, n = gd.n, rows = (long long)S * gd.nv, M = rows * gd.nu;
  const int L = gd.nu;
  const size_t act = sizeof(float) * kNetC * (size_t)M;
  HIPC(c->na0.ensure(act));
  HIPC(c->na1.ensure(act));
  HIPC(c->na2.ensure(act));
  HIPC(c->nga.ensure(act));
  HIPC(c->ngb.ensure(act));
  HIPC(c->nmask.ensure(sizeof(unsigned) * 3 * (size_t)M));
  HIPC(c->nout.ensure(sizeof(float) * (size_t)M));
  HIPC(c->ngout.ensure(sizeof(float) * (size_t)M));
  HIPC(c->nxh.ensure(sizeof(float) * (size_t)n));
  HIPC(c->nr.ensure(sizeof(float) * (size_t)n));
  HIPC(c->npart.ensure(sizeof(float) * (size_t)net_wgrad_blocks() * kNetC * kNetC * kNetK));
  HIPC(c->nsums.ensure(sizeof(double) * 2 * (size_t)S));
  HIPC(c->nred.ensure(sizeof(double) * 2 * 1024));
  const long long nb = std::max<long long>({(long long)ray_blocks(gd), (long long)bt_blocks(gd), (long long)pixel_blocks(gd), 1LL});
  stt = ensure_scratch(c, gd, sizeof(float), nb);
  if (stt != GKB_OK) return stt;
  float *a1 = c->na0.as<float>(), *a2 = c->na1.as<float>(), *a3 = c->na2.as<float>();
  float *ga = c->nga.as<float>(), *gb = c->ngb.as<float>(), *out = c->nout.as<float>(), *gout = c->ngout.as<float>();
  unsigned *mk = c->nmask.as<unsigned>();
  unsigned *m0 = mk, *m1 = mk + M, *m2 = mk + 2 * M;
  float *part = c->npart.as<float>(), *grad = net->grad.as<float>();
  const NetW &w = net->nw;
  // input of the trained map: b (learned filtered back projection), or the
  // noise-free data A x through the filter frozen at b (operator objective)
  const float *in = b;
  if (objective == 0) {
    // forward with the training rounding (bfloat16 operands in layers 2, 3)
    launch_net_c1(Col<const float>{b, 0, 0, nullptr}, a1, m0, w.w1, L, rows, 1, nullptr, st);
    launch_net_c32(a1, a2, m1, w.w2b, L, rows, 1, 1, nullptr, st);
    launch_net_c32(a2, a3, m2, w.w3b, L, rows, 1, 1, nullptr, st);
    launch_net_c4(a3, out, w.w4, L, rows, nullptr, st);
  } else {
    HIPC(c->ny.ensure(sizeof(float) * (size_t)M));
    float *y = c->ny.as<float>();
    // masks of b in the precision the solve uses
    launch_net_c1(Col<const float>{b, 0, 0, nullptr}, a1, m0, w.w1, L, rows, 1, nullptr, st);
    launch_net_c32(a1, a2, m1, w.w2b, L, rows, 3, 1, nullptr, st);
    launch_net_c32(a2, a3, m2, w.w3b, L, rows, 3, 1, nullptr, st);
    for (int si = 0; si < S; ++si) {
      launch_pad_image<float>(gd, col<const float>(x + si * n), c->xpad.as<float>(), d->has_coldom, nullptr, st);
      launch_fwd<float>(gd, rt_of<float>(*d), c->xpad.as<float>(), col<float>(y + si * mS), plain_epi<float>(),
                        nullptr, st);
    }
    launch_net_c1(Col<const float>{y, 0, 0, nullptr}, a1, m0, w.w1, L, rows, 2, nullptr, st);
    launch_net_c32(a1, a2, m1, w.w2b, L, rows, 1, 2, nullptr, st);
    launch_net_c32(a2, a3, m2, w.w3b, L, rows, 1, 2, nullptr, st);
    launch_net_c4(a3, out, w.w4, L, rows, nullptr, st);
    in = y;
  }
  // per sample: xhat = B N(b_s); r = xhat - x_s; gout_s = B^T r * 2 / (||x_s||^2 S)
  const Epi<float> pe = plain_epi<float>();
  for (int si = 0; si < S; ++si) {
    launch_pad_sino<float>(gd, col<const float>(out + si * mS), c->ypad.as<float>(), nullptr, st);
    launch_back<float>(gd, vt_of<float>(*d), c->ypad.as<float>(), c->nxh.as<float>(), pe, nullptr, st);
    launch_net_resid(c->nxh.as<float>(), x + si * n, c->nr.as<float>(), n, c->nred.as<double>(),
                     c->nsums.as<double>() + 2 * si, st);
    launch_net_scale(c->nr.as<float>(), n, c->nsums.as<double>() + 2 * si, S, st);
    launch_pad_image<float>(gd, col<const float>(c->nr.as<float>()), c->xpad.as<float>(), d->has_coldom, nullptr,
                            st);
    launch_back_adj<float>(gd, rt_of<float>(*d), c->xpad.as<float>(), col<float>(gout + si * mS), pe, nullptr, st);
  }
  // backward
  const int np = net_wgrad_blocks();
  launch_net_wgrad_edge(a3, gout, part, L, rows, -1, st);
  launch_net_reduce(part, np, kNetC * kNetK, grad + kOffW4, 1.0, st);
  launch_net_c1(Col<const float>{gout, 0, 0, nullptr}, ga, m2, w.w4t, L, rows, 2, nullptr, st);
  launch_net_wgrad32(ga, a2, part, L, rows, st);
  launch_net_reduce(part, np, kNetC * kNetC * kNetK, grad + kOffW3, 1.0, st);
  launch_net_c32(ga, gb, m1, w.w3t, L, rows, 1, 2, nullptr, st);
  launch_net_wgrad32(gb, a1, part, L, rows, st);
  launch_net_reduce(part, np, kNetC * kNetC * kNetK, grad + kOffW2, 1.0, st);
  launch_net_c32(gb, ga, m0, w.w2t, L, rows, 1, 2, nullptr, st);
  launch_net_wgrad_edge(ga, in, part, L, rows, 1, st);
  launch_net_reduce(part, np, kNetC * kNetK, grad, 1.0, st);
  HIPC(hipGetLastError());
  std::vector<double> sums(2 * (size_t)S);
  HIPC(hipMemcpyAsync(sums.data(), c->nsums.p, sizeof(double) * sums.size(), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  double loss = 0.0;
  for (int si = 0; si < S; ++si) loss += sums[2 * si] / sums[2 * si + 1];
  loss /= S;
  if (!std::isfinite(loss)) return fail(GKB_ENONFINITE, "non-finite training loss");
  if (loss_out) *loss_out = loss;
  return GKB_OK;
}

gkb_status net_check(gkb_ctx *c, const gkb_net *net) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!net) return fail(GKB_EINVAL, "network is NULL");
  if (net->device != c->device) return fail(GKB_EINVAL, "network and context are on different devices");
  return GKB_OK;
}

// --------------------------------------------------------------------------
// GKB driver
// --------------------------------------------------------------------------
enum Mode { MODE_AB = 0, MODE_BA = 1, MODE_GKB = 2 };

template <typename T>
struct Solver {
  gkb_ctx *c;
  const DevTables &d;
  const GeomDev &g;
  int mode;
  int K;
  long long n, m, dimq, dims;
  long long ldq;  // column stride of Q (a multiple of 4)
  T *Q = nullptr, *yk = nullptr, *s = nullptr, *w = nullptr, *tn = nullptr, *tm = nullptr;
  T *xpad = nullptr, *ypad = nullptr, *ywpad = nullptr;
  // Padded inputs written by the producers.  A kernel that makes a vector the
  // next projector reads also writes its padded copy (PadOut), and the tags
  // name the vector whose copy each padded buffer holds, so the consumer
  // skips its padding kernel.  2D solves without the learned filter only.
  enum Tag : int { TAG_NONE = 0, TAG_Q, TAG_YK, TAG_S, TAG_TM, TAG_BQ, TAG_ATS };
  int tag_x = TAG_NONE, tag_y = TAG_NONE, tag_yw = TAG_NONE;
  Ctl ctl{};
  double *partials = nullptr;
  hipStream_t st;
  const int *stop = nullptr;
  const int *kp = nullptr;
  // learned filter inside B (BA-GKB, FP32): M = B F A, M^T = A^T F^T B^T
  const gkb_net *net = nullptr;
  long long nrows = 0;
  int nL = 0;

  Solver(gkb_ctx *ctx, const DevTables &dt, int md, int kmax) : c(ctx), d(dt), g(dt.gd), mode(md), K(kmax) {
    n = g.n;
    m = g.m;
    dimq = (mode == MODE_AB) ? m : n;
    ldq = (dimq + 3) / 4 * 4;
    dims = (mode == MODE_BA) ? n : m;
    st = c->stream;
  }

  gkb_status alloc() {
    HIPC(c->Q.ensure(sizeof(T) * (size_t)ldq * (K + 1)));
    HIPC(c->yk.ensure(sizeof(T) * (size_t)m));
    HIPC(c->rdbl.ensure(sizeof(double) * 2 * (size_t)((m + 3) / 4 * 4)));
    HIPC(c->s.ensure(sizeof(T) * (size_t)dims));
    HIPC(c->w.ensure(sizeof(T) * (size_t)dimq));
    HIPC(c->tmp_n.ensure(sizeof(T) * (size_t)n));
    HIPC(c->tmp_m.ensure(sizeof(T) * (size_t)m));
    const size_t nd = CD_COUNT + 11 * (size_t)(K + 2);
    HIPC(c->ctl_d.ensure(sizeof(double) * nd));
    HIPC(c->ctl_i.ensure(sizeof(int) * CI_COUNT));
    HIPC(c->gram.ensure(sizeof(double) * (size_t)(K + 1) * (size_t)(K + 1)));
    const long long vb = std::max<long long>(
        {(long long)vec_blocks(dimq), (long long)vec_blocks(m), (long long)vec_blocks(dims)});
    const long long pb = std::max<long long>(
        {(long long)ray_blocks(g), (long long)bt_blocks(g), (long long)pixel_blocks(g), 2 * vb * (K + 2),
         (long long)upd_blocks(dimq)});
    gkb_status stt = ensure_scratch(c, g, sizeof(T), pb);
    if (stt != GKB_OK) return stt;
    if (!c->host_flag) {
      HIPC(hipHostMalloc((void **)&c->host_flag, sizeof(int) * 4, hipHostMallocMapped));
      HIPC(hipHostGetDevicePointer((void **)&c->host_flag_dev, c->host_flag, 0));
    }
    Q = c->Q.as<T>();
    yk = c->yk.as<T>();
    s = c->s.as<T>();
    w = c->w.as<T>();
    tn = c->tmp_n.as<T>();
    tm = c->tmp_m.as<T>();
    xpad = c->xpad.as<T>();
    ypad = c->ypad.as<T>();
    ywpad = (g.kind == GKB_FAN2D) ? c->ywpad.as<T>() : ypad;
    double *dp = c->ctl_d.as<double>();
    ctl.ip = c->ctl_i.as<int>();
    ctl.dp = dp;
    dp += CD_COUNT;
    double **arrs[] = {&ctl.alpha, &ctl.t, &ctl.rho, &ctl.pres, &ctl.u,   &ctl.Rd,
                       &ctl.Rth,   &ctl.Rphi, &ctl.c, &ctl.rre,  &ctl.lamh};
    for (double **a : arrs) {
      *a = dp;
      dp += K + 2;
    }
    ctl.aw = c->rdbl.as<double>();
    ctl.r = ctl.aw + (m + 3) / 4 * 4;  // 32-byte aligned quads
    ctl.gram = c->gram.as<double>();
    ctl.K = K;
    ctl.host_stop = c->host_flag_dev;
    partials = c->partials.as<double>();
    stop = ctl.ip + CI_STOP;
    kp = ctl.ip + CI_K;
    return GKB_OK;
  }

  Epi<T> epi() const {
    Epi<T> e = plain_epi<T>();
    e.ctl = ctl;
    e.use_ctl = 1;
    e.partials = partials;
    return e;
  }

  // column i (0-based, shifted by the device counter k) of Q
  Col<const T> qcol(int off) const { return colk<const T>(Q, ldq, off, kp); }

  // ----- the four projectors with device-addressed operands -----
  bool cone() const { return g.kind == GKB_CONE3D; }
  bool fusing() const { return !cone() && !filtered(); }
  // padded copies in the layouts A / B^T (image), B (sinogram) and A^T read
  PadOut<T> pad_image_out() const {
    PadOut<T> p{};
    p.dst = xpad;
    p.kind = PADK_IMAGE;
    p.n1 = g.nx;
    p.lead = g.ldR;
    p.off0 = g.pad;
    p.ldT = g.ldT;
    p.offT = d.has_coldom ? g.offT : -1;
    return p;
  }
  PadOut<T> pad_sino_out() const {
    PadOut<T> p{};
    p.dst = ypad;
    p.kind = PADK_SINO;
    p.n1 = g.nu;
    p.lead = g.ldY;
    p.off0 = g.padY;
    return p;
  }
  PadOut<T> pad_adj_out() const {
    if (g.kind != GKB_FAN2D) return pad_sino_out();
    PadOut<T> p = pad_sino_out();
    p.dst = ywpad;
    p.kind = PADK_SINO_W;
    p.w = rt_of<T>(d).w;
    return p;
  }
  // the four projectors; `tag` names the input (TAG_NONE: unknown), and the
  // padding kernel is skipped when the padded buffer already holds it
  // stp: the stop flag the launches test (nullptr: run unconditionally)
  void A(Col<const T> in, Col<T> out, const Epi<T> &e, const int *stp, int tag) {
    if (cone()) {
      launch_cone_pad_volume<T>(g, in, xpad, d.has_xdom, d.has_ydom, stp, st);
      TraceScope ts(c, "fwd");
      launch_cone_fwd<T>(g, ct_of<T>(d), xpad, out, e, stp, st);
      return;
    }
    if (tag == TAG_NONE || tag_x != tag) launch_pad_image<T>(g, in, xpad, d.has_coldom, stp, st);
    tag_x = tag;
    TraceScope ts(c, "fwd");
    launch_fwd<T>(g, rt_of<T>(d), xpad, out, e, stp, st);
  }
  void A(Col<const T> in, Col<T> out, const Epi<T> &e, int tag = TAG_NONE) { A(in, out, e, stop, tag); }
  void Bt(Col<const T> in, Col<T> out, const Epi<T> &e, int tag = TAG_NONE) {
    if (cone()) {
      launch_cone_pad_volume<T>(g, in, xpad, d.has_xdom, d.has_ydom, stop, st);
      TraceScope ts(c, "back_adj");
      launch_cone_back_adj<T>(g, ct_of<T>(d), vt_of<T>(d), xpad, out, e, stop, st);
      return;
    }
    if (tag == TAG_NONE || tag_x != tag) launch_pad_image<T>(g, in, xpad, d.has_coldom, stop, st);
    tag_x = tag;
    TraceScope ts(c, "back_adj");
    launch_back_adj<T>(g, rt_of<T>(d), xpad, out, e, stop, st);
  }
  // stp: the stop flag the launches test (nullptr: run unconditionally)
  void B(Col<const T> in, T *out, const Epi<T> &e, const int *stp, int tag = TAG_NONE) {
    if (cone()) {
      launch_cone_pad_sino<T>(g, in, ypad, stp, st);
      TraceScope ts(c, "back");
      launch_cone_back<T>(g, vt_of<T>(d), ypad, out, e, stp, st);
      return;
    }
    if (tag == TAG_NONE || tag_y != tag) launch_pad_sino<T>(g, in, ypad, stp, st);
    tag_y = tag;
    TraceScope ts(c, "back");
    launch_back<T>(g, vt_of<T>(d), ypad, out, e, stp, st);
  }
  void B(Col<const T> in, T *out, const Epi<T> &e, int tag = TAG_NONE) { B(in, out, e, stop, tag); }
  void At(Col<const T> in, T *out, const Epi<T> &e, int tag = TAG_NONE) {
    if (cone()) {
      launch_cone_weight_sino<T>(g, ct_of<T>(d), in, ypad, stop, st);
      TraceScope ts(c, "fwd_adj");
      launch_cone_fwd_adj<T>(g, ct_of<T>(d), vt_of<T>(d), ypad, out, e, stop, st);
      return;
    }
    int &tg = (g.kind == GKB_FAN2D) ? tag_yw : tag_y;
    if (tag == TAG_NONE || tg != tag) launch_pad_sino_adj<T>(g, rt_of<T>(d), in, ywpad, stop, st);
    tg = tag;
    TraceScope ts(c, "fwd_adj");
    launch_fwd_adj<T>(g, vt_of<T>(d), rt_of<T>(d), ywpad, out, e, stop, st);
  }
  // after a launch whose epilogue wrote the padded copy of the vector `tag`
  void wrote_image(int tag) { tag_x = tag; }
  void wrote_sino(int tag) { tag_y = tag; }
  void wrote_adj(int tag) { (g.kind == GKB_FAN2D ? tag_yw : tag_y) = tag; }
  void forget_pads() { tag_x = tag_y = tag_yw = TAG_NONE; }

  // s~ <- M q_k - alpha_k/t_k s~ (s stored unnormalised, s_k = s~/t_k); t_{k+1}; Y_k
  void apply_M() {
    Epi<T> e = epi();
    e.prev_sel = PREV_NEG_ALPHA_OVER_T;
    e.prev = col<const T>(s);
    e.norm_to_t = 1;
    const bool fu = fusing();
    Epi<T> pe = plain_epi<T>();
    if (mode == MODE_BA) {  // Y_k = A q_k ; s~ = B Y_k - ...  (B F Y_k with the filter)
      if (fu) pe.pout = pad_sino_out();
      A(qcol(-1), col<T>(yk), pe, TAG_Q);
      if (fu) wrote_sino(TAG_YK);
      if (filtered()) {
        filter(NET_F, col<const T>(yk));
        B(col<const T>(c->nout.as<T>()), s, e);
      } else {
        if (fu) e.pout = pad_image_out();
        B(col<const T>(yk), s, e, TAG_YK);
        if (fu) wrote_image(TAG_S);
      }
    } else if (mode == MODE_AB) {  // Y_k = A B q_k ; s~ = Y_k - ...
      if (fu) pe.pout = pad_image_out();
      B(qcol(-1), tn, pe, TAG_Q);
      if (fu) wrote_image(TAG_BQ);
      e.out_raw = col<T>(yk);
      if (fu) e.pout = pad_adj_out();
      A(col<const T>(tn), col<T>(s), e, TAG_BQ);
      if (fu) wrote_adj(TAG_S);
    } else {  // matched: Y_k = A q_k ; s~ = Y_k - ...
      e.out_raw = col<T>(yk);
      if (fu) e.pout = pad_adj_out();
      A(qcol(-1), col<T>(s), e, TAG_Q);
      if (fu) wrote_adj(TAG_S);
    }
  }

  bool filtered() const { return std::is_same<T, float>::value && net != nullptr; }
  // filter chain into the context's filter output buffer (FP32 path only)
  void filter(int op, Col<const T> in) {
    if constexpr (std::is_same<T, float>::value) {
      TraceScope ts(c, op == NET_FT ? "filter_t" : "filter");
      net_chain(c, net, op, in, c->nout.as<float>(), nrows, nL, stop, st);
    }
  }

  // w <- M^T s_{k+1} - t_{k+1} q_k   (k = 0: w <- M^T s_1)
  void apply_Mt(bool first) {
    Epi<T> e0 = epi();
    e0.in_sel = IN_INV_TNEXT;  // s_{k+1} = s~ / t_{k+1}
    Epi<T> e1 = epi();
    if (!first) {
      e1.prev_sel = PREV_NEG_TNEXT;
      e1.prev = qcol(-1);
    }
    const bool fu = fusing();
    if (mode == MODE_BA) {  // A^T (B^T s)  (A^T F^T B^T s with the filter)
      if (fu) e0.pout = pad_adj_out();
      Bt(col<const T>(s), col<T>(tm), e0, TAG_S);
      if (fu) wrote_adj(TAG_TM);
      if (filtered()) {
        filter(NET_FT, col<const T>(tm));
        At(col<const T>(c->nout.as<T>()), w, e1);
      } else {
        At(col<const T>(tm), w, e1, TAG_TM);
      }
    } else if (mode == MODE_AB) {  // B^T (A^T s)
      if (fu) e0.pout = pad_image_out();
      At(col<const T>(s), tn, e0, TAG_S);
      if (fu) wrote_image(TAG_ATS);
      Bt(col<const T>(tn), col<T>(w), e1, TAG_ATS);
    } else {  // A^T s
      Epi<T> e = e1;
      e.in_sel = IN_INV_TNEXT;
      At(col<const T>(s), w, e, TAG_S);
    }
  }

  void iteration(bool reorth, int k) {
    apply_M();
    apply_Mt(false);
    reorth_and_normalize_impl(reorth);
    {
      TraceScope ts(c, "small_solve");
      launch_small_solve(ctl, st);
    }
    {
      TraceScope ts(c, "residual");
      launch_resid<T>(ctl, yk, m, partials, st);
    }
  }

  // reorthogonalise w against the columns q_1..q_k of Q (the kernels read k
  // from the control block), then alpha_{k+1} and q_{k+1}
  void reorth_and_normalize_impl(bool reorth) {
    TraceScope ts(c, "reorth");
    if (reorth) {
      // two classical rounds, the second from the Gram matrix (one read of Q
      // for the inner products, one for the update)
      launch_dcgs_dots<T>(ctl, Q, ldq, w, dimq, partials, st, q_streams());
      launch_dcgs_coef(ctl, st);
      update_normalize(1);
    } else {
      // no reorthogonalisation: only the norm alpha_{k+1} = ||w|| (no columns)
      update_normalize(0);
    }
  }

  // RRE(x_k) = ||x_k - x_true|| / ||x_true|| (eq. RE) after iteration k: x_k
  // is assembled from Q and u_k as the returned solution is (AB: B Q_k u_k).
  // The kernels are not gated by the stop flag, so the stopping iterate's
  // error is recorded; iterations queued after a stop recompute the same
  // value.  The B call pads its own input, so later consumers re-pad.
  void rre_step(const T *x_true) {
    if (mode == MODE_AB) {
      launch_solution<T>(ctl, Q, ldq, dimq, tm, st);
      B(col<const T>(tm), tn, plain_epi<T>(), nullptr);
    } else {
      launch_solution<T>(ctl, Q, ldq, dimq, tn, st);
    }
    launch_rre<T>(ctl, tn, x_true, n, partials, st);
  }

  // q_{k+1} = w / alpha_{k+1}, with the padded copy the next iteration's first
  // projector reads (A: image; AB's B: sinogram)
  void normalize() {
    if (!fusing()) {
      launch_normalize<T>(ctl, w, Q, ldq, dimq, st);
      return;
    }
    launch_normalize<T>(ctl, w, Q, ldq, dimq, st, mode == MODE_AB ? pad_sino_out() : pad_image_out());
    if (mode == MODE_AB)
      wrote_sino(TAG_Q);
    else
      wrote_image(TAG_Q);
  }

  // the stored basis (K + 1 columns of ldq) larger than the last-level cache:
  // its reorthogonalisation passes stream it with nontemporal loads, which
  // keeps the projectors' data in that cache (a basis that fits is read with
  // ordinary loads, so that the update pass finds what the inner products
  // brought in)
  bool q_streams() const { return (long long)(ctl.K + 1) * ldq * (long long)sizeof(T) > kLlcBytes; }
  // the same for the stored A-images Y (GMRES and hybrid solves: K columns of
  // ldy), which the residual reads in full every iteration
  bool y_streams() const { return (long long)ctl.K * ldy * (long long)sizeof(T) > kLlcBytes; }

  // w -= Q c over the reorthogonalisation columns (reorth_cols = 0: none),
  // then q_{k+1} = w / alpha_{k+1} with alpha_{k+1} summed from the update's
  // partials inside the normalisation
  void update_normalize(int reorth_cols) {
    if (!fusing()) {
      launch_update_normalize<T>(ctl, Q, ldq, w, dimq, partials, st, reorth_cols, PadOut<T>{}, q_streams());
      return;
    }
    launch_update_normalize<T>(ctl, Q, ldq, w, dimq, partials, st, reorth_cols,
                               mode == MODE_AB ? pad_sino_out() : pad_image_out(), q_streams());
    if (mode == MODE_AB)
      wrote_sino(TAG_Q);
    else
      wrote_image(TAG_Q);
  }

  // ----- AB-/BA-GMRES (Algs. "AB-GMRES", "BA-GMRES") on the same buffers -----
  // Q holds the Arnoldi basis (dimension m for AB, n for BA), w the vector
  // being orthogonalised, Y the A-images of the basis (AB: A B q_i, the raw
  // product before orthogonalisation; BA: A q_i), ldy a multiple of 4.
  T *Y = nullptr;
  long long ldy = 0;

  gkb_status gm_alloc() {
    ldy = (m + 3) / 4 * 4;
    HIPC(c->gm_y.ensure(sizeof(T) * (size_t)ldy * K));
    ctl.ldh = K + 2;
    HIPC(c->gm_h.ensure(sizeof(double) * (size_t)ctl.ldh * (K + 2)));
    Y = c->gm_y.as<T>();
    ctl.hm = c->gm_h.as<double>();
    return GKB_OK;
  }

  // w = M q_k and the A-image Y[:, k-1]
  void gm_apply_M() {
    const bool fu = fusing();
    Col<T> ycol = colk<T>(Y, ldy, -1, kp);
    Epi<T> pe = plain_epi<T>();
    if (mode == MODE_AB) {  // w = A (B q_k); Y_k = w before orthogonalisation
      if (fu) pe.pout = pad_image_out();
      B(qcol(-1), tn, pe, TAG_Q);
      if (fu) wrote_image(TAG_BQ);
      Epi<T> e = plain_epi<T>();
      e.out_raw = ycol;
      A(col<const T>(tn), col<T>(w), e, TAG_BQ);
    } else {  // Y_k = A q_k ; w = B Y_k
      if (fu) pe.pout = pad_sino_out();
      A(qcol(-1), ycol, pe, TAG_Q);
      if (fu) wrote_sino(TAG_YK);
      B(colk<const T>(Y, ldy, -1, kp), w, plain_epi<T>(), TAG_YK);
    }
  }

  // Arnoldi step: two classical Gram-Schmidt rounds of w against q_1..q_k
  // (the second's inner products from the Gram matrix), their coefficients
  // summed into column k of H; h_{k+1,k} = ||w|| into alpha[k+1]; q_{k+1}
  void gm_orthogonalise() {
    TraceScope ts(c, "reorth");
    launch_dcgs_dots<T>(ctl, Q, ldq, w, dimq, partials, st, q_streams());
    launch_dcgs_coef(ctl, st);
    launch_gm_hcol(ctl, st);  // h_{1..k,k}: both rounds' coefficients
    update_normalize(1);
  }

  void gm_iteration(int k, const T *b) {
    gm_apply_M();
    gm_orthogonalise();
    {
      TraceScope ts(c, "small_solve");
      launch_gm_solve(ctl, st);
    }
    {
      TraceScope ts(c, "residual");
      launch_gm_resid<T>(ctl, Y, ldy, b, m, partials, st, NORM_GMRHO, y_streams());
    }
  }

  // ----- hybrid regularisation: lambda_k on C_k each iteration -----
  // The residual recurrence of the plain solve assumes one lambda for all
  // iterations, so rho_k = ||Y_k u_k - b|| is formed from the A-images of
  // the basis (as for GMRES: BA: A q_i; AB: A B q_i).
  gkb_status hy_alloc() {
    ldy = (m + 3) / 4 * 4;
    HIPC(c->gm_y.ensure(sizeof(T) * (size_t)ldy * K));
    Y = c->gm_y.as<T>();
    return GKB_OK;
  }

  void hy_iteration(bool reorth, int k, const T *b) {
    T *keep = yk;
    yk = Y + (size_t)(k - 1) * (size_t)ldy;  // the A-image of q_k is column k - 1 of Y
    apply_M();
    yk = keep;
    apply_Mt(false);
    reorth_and_normalize_impl(reorth);
    {
      TraceScope ts(c, "small_solve");
      launch_hy_lambda(ctl, st);
      launch_hy_solve(ctl, st);
    }
    {
      TraceScope ts(c, "residual");
      launch_gm_resid<T>(ctl, Y, ldy, b, m, partials, st, NORM_RHO, y_streams());
    }
  }
};

template <typename T>
gkb_status solve_impl(gkb_ctx *c, const gkb_geometry *geom, int dtype, const void *bv, const gkb_solve_opts *o,
                      void *xv, gkb_solve_info *info, int mode, const gkb_hybrid_opts *hy = nullptr) {
  auto t_start = std::chrono::steady_clock::now();
  DevTables *d = nullptr;
  gkb_status stt = get_tables(c, geom, dtype, &d);
  if (stt != GKB_OK) return stt;
  Solver<T> S(c, *d, mode, o->k_max);
  stt = S.alloc();
  if (stt != GKB_OK) return stt;
  // hybrid regularisation (lambda_k on C_k) or the enlarged-subspace TSVD
  const bool hyb = hy && hy->lambda_rule != GKB_LAMBDA_FIXED;
  const int tsvd_rank = hy ? hy->tsvd_rank : 0;
  double *tsvd_w = nullptr;
  if (hyb) {
    stt = S.hy_alloc();
    if (stt != GKB_OK) return stt;
  }
  if (tsvd_rank > 0) {
    const size_t K = (size_t)o->k_max;
    HIPC(c->hy_w.ensure(sizeof(double) * ((K + 1) * K + K * K)));
    tsvd_w = c->hy_w.as<double>();
  }
  if (o->precond) {
    S.net = o->precond;
    net_shape(geom, S.nrows, S.nL);
    stt = net_scratch(c, S.nrows, S.nL);
    if (stt != GKB_OK) return stt;
  }
  const T *b = static_cast<const T *>(bv);
  T *x = static_cast<T *>(xv);
  hipStream_t st = c->stream;
  const GeomDev &g = d->gd;

  // control block
  int hip_[CI_COUNT] = {0};
  double hdp[CD_COUNT] = {0};
  hdp[CD_TAUE] = o->use_dp ? o->tau * o->noise_norm : 0.0;
  hdp[CD_LAMBDA] = o->lambda;
  hdp[CD_ETAEPS] = 100.0 * (sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16) * 2.0;
  hdp[CD_USEDP] = o->use_dp ? 1.0 : 0.0;
  hdp[CD_KMAX] = o->k_max;
  hdp[CD_RNS] = o->rns_eps;
  hdp[CD_REACH] = (o->precond && o->use_dp) ? 1.0 : 0.0;
  hdp[CD_HRULE] = hyb ? hy->lambda_rule : HY_FIXED;
  hdp[CD_HTARGET] = (hyb && hy->lambda_rule == GKB_LAMBDA_DP) ? hy->tau_proj * hy->eta_proj : 0.0;
  HIPC(hipMemcpyAsync(S.ctl.ip, hip_, sizeof hip_, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(S.ctl.dp, hdp, sizeof hdp, hipMemcpyHostToDevice, st));
  *c->host_flag = 0;

  // the padded buffers the producers write into keep zero pads from here on
  if (S.fusing()) {
    HIPC(hipMemsetAsync(S.xpad, 0, sizeof(T) * (size_t)g.pad_elems, st));
    HIPC(hipMemsetAsync(S.ypad, 0, sizeof(T) * (size_t)g.ypad_elems, st));
    if (g.kind == GKB_FAN2D) HIPC(hipMemsetAsync(S.ywpad, 0, 2 * sizeof(T) * (size_t)g.ypad_elems, st));
  }
  S.forget_pads();

  // start-up (k = 0): r_0 = -b, ||b||; s~_1 = rhs, t_1; q_1, alpha_1
  launch_resid_init<T>(S.ctl, b, g.m, S.partials, st);
  if (mode == MODE_BA) {
    Epi<T> e = S.epi();
    e.norm_to_t = 1;
    if (S.filtered()) {  // rhs B F b = B N(b); the masks of b are frozen here
      S.filter(NET_MASKS, col<const T>(b));
      S.B(col<const T>(c->nout.as<T>()), S.s, e);
    } else {
      S.B(col<const T>(b), S.s, e);
    }
  } else {
    launch_copy<T>(b, S.s, g.m, st);
    launch_norm_to<T>(S.ctl, S.s, g.m, NORM_T1, S.partials, st);
  }
  S.apply_Mt(true);
  launch_norm_to<T>(S.ctl, S.w, S.dimq, NORM_ALPHA1, S.partials, st);
  S.normalize();
  HIPC(hipGetLastError());
  double h3[3];
  HIPC(hipMemcpyAsync(&h3[0], S.ctl.t + 1, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(&h3[1], S.ctl.alpha + 1, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(&h3[2], S.ctl.dp + CD_BNORM, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const double t1 = h3[0], bnorm = h3[2];
  const double a1 = (t1 > 0.0) ? h3[1] : 0.0;  // M^T (s/t_1) is 0/0 when t_1 = 0
  if (!std::isfinite(bnorm) || !std::isfinite(t1) || !std::isfinite(a1))
    return fail(GKB_ENONFINITE, "non-finite value in b (or in the start-up vectors)");
  gkb_solve_info inf{};
  inf.t1 = t1;
  inf.alpha1 = a1;
  int k_stop = 0, reason = 0;
  if (!(t1 > 0.0) || !(a1 > 0.0)) {
    // rhs = 0 or M^T rhs = 0: x = 0 is the least-squares solution in the (empty) Krylov space
    HIPC(hipMemsetAsync(x, 0, sizeof(T) * (size_t)g.n, st));
    HIPC(hipStreamSynchronize(st));
    reason = GKB_STOP_BREAKDOWN;
    inf.residual = bnorm;
    inf.proj_residual = t1;
  } else {
    launch_set_int(S.ctl.ip + CI_K, 1, st);
    const int L = 4;
    std::vector<hipEvent_t> evs(L, nullptr);
    for (auto &e : evs) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const bool reorth = o->reorth != 0;
    const T *x_true = (o->x_true && o->rre_history) ? static_cast<const T *>(o->x_true) : nullptr;
    if (x_true) launch_norm_to<T>(S.ctl, x_true, g.n, NORM_XTRUE, S.partials, st);
    int launched = 0;
    for (int k = 1; k <= o->k_max; ++k) {
      if (hyb)
        S.hy_iteration(reorth, k, b);
      else
        S.iteration(reorth, k);
      if (x_true) S.rre_step(x_true);
      HIPC(hipEventRecord(evs[k % L], st));
      ++launched;
      if (k >= L) {
        HIPC(hipEventSynchronize(evs[(k - L + 1) % L]));
        if (*(volatile int *)c->host_flag) break;
      }
    }
    HIPC(hipGetLastError());
    // launches queued after the stop did not run: no padded copy is known
    S.forget_pads();
    // enlarged-subspace TSVD: u from the rank-r truncated SVD of C_K
    if (tsvd_rank > 0) launch_tsvd(S.ctl, tsvd_w, tsvd_w + (size_t)(o->k_max + 1) * o->k_max, tsvd_rank, st);
    // solution x = Q_k u_k (BA, matched) or B (Q_k u_k) (AB)
    if (mode == MODE_AB) {
      launch_solution<T>(S.ctl, S.Q, S.ldq, S.dimq, S.tm, st);
      S.B(col<const T>(S.tm), x, plain_epi<T>(), nullptr);
    } else {
      launch_solution<T>(S.ctl, S.Q, S.ldq, S.dimq, x, st);
    }
    if (tsvd_rank > 0) {  // ||A x - b|| of the truncated solution
      S.A(col<const T>(x), col<T>(S.tm), plain_epi<T>(), nullptr, Solver<T>::TAG_NONE);
      launch_final_residual<T>(S.ctl, S.tm, b, g.m, S.partials, st);
    }
    HIPC(hipGetLastError());
    int hi[CI_COUNT];
    HIPC(hipMemcpyAsync(hi, S.ctl.ip, sizeof hi, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (auto &e : evs) (void)hipEventDestroy(e);
    k_stop = hi[CI_KSTOP];
    reason = hi[CI_REASON];
    std::vector<double> rho(o->k_max + 2), pres(o->k_max + 2);
    HIPC(hipMemcpy(rho.data(), S.ctl.rho, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(pres.data(), S.ctl.pres, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    inf.residual = rho[k_stop];
    inf.proj_residual = pres[k_stop];
    if (o->residual_history)
      for (int k = 1; k <= k_stop; ++k) o->residual_history[k - 1] = rho[k];
    if (x_true) {
      std::vector<double> rre(o->k_max + 2);
      HIPC(hipMemcpy(rre.data(), S.ctl.rre, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
      for (int k = 1; k <= k_stop; ++k) o->rre_history[k - 1] = rre[k];
    }
    if (hyb && hy->lambda_history) {
      std::vector<double> lh(o->k_max + 2);
      HIPC(hipMemcpy(lh.data(), S.ctl.lamh, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
      for (int k = 1; k <= o->k_max; ++k) hy->lambda_history[k - 1] = (k <= k_stop) ? lh[k] : 0.0;
    }
    if (tsvd_rank > 0) {
      // ||A x - b|| of the returned x, and ||C_K u - t_1 e_1|| of its u
      const int K = k_stop;
      std::vector<double> al(K + 2), tt(K + 2), uu(K + 2);
      HIPC(hipMemcpy(&inf.residual, S.ctl.dp + CD_FINALRES, sizeof(double), hipMemcpyDeviceToHost));
      HIPC(hipMemcpy(al.data(), S.ctl.alpha, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      HIPC(hipMemcpy(tt.data(), S.ctl.t, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      HIPC(hipMemcpy(uu.data(), S.ctl.u, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      double pr = 0.0;
      for (int i = 1; i <= K + 1; ++i) {
        double r = (i <= K ? al[i] * uu[i] : 0.0) + (i >= 2 ? tt[i] * uu[i - 1] : 0.0);
        if (i == 1) r -= tt[1];
        pr += r * r;
      }
      inf.proj_residual = std::sqrt(pr);
    }
    (void)launched;
  }
  if (o->alpha_history || o->t_history) {
    std::vector<double> al(o->k_max + 2), tt(o->k_max + 2);
    HIPC(hipMemcpy(al.data(), S.ctl.alpha, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(tt.data(), S.ctl.t, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    al[1] = inf.alpha1;  // 0 (not 0/0) when t_1 = 0
    for (int k = 1; k <= o->k_max + 1; ++k) {
      if (o->alpha_history) o->alpha_history[k - 1] = (k <= k_stop + 1) ? al[k] : 0.0;
      if (o->t_history) o->t_history[k - 1] = (k <= k_stop + 1) ? tt[k] : 0.0;
    }
  }
  inf.k_stop = k_stop;
  inf.reason = reason;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (info) *info = inf;
  return GKB_OK;
}

// AB-GMRES / BA-GMRES from x_0 = 0: the Arnoldi iteration on M = AB or BA
// with the stopping rules of the GKB solves on rho_k = ||A x_k - b||.
template <typename T>
gkb_status gm_solve_impl(gkb_ctx *c, const gkb_geometry *geom, int dtype, const void *bv, const gkb_solve_opts *o,
                         void *xv, gkb_solve_info *info, int mode) {
  auto t_start = std::chrono::steady_clock::now();
  DevTables *d = nullptr;
  gkb_status stt = get_tables(c, geom, dtype, &d);
  if (stt != GKB_OK) return stt;
  Solver<T> S(c, *d, mode, o->k_max);
  stt = S.alloc();
  if (stt != GKB_OK) return stt;
  stt = S.gm_alloc();
  if (stt != GKB_OK) return stt;
  const T *b = static_cast<const T *>(bv);
  T *x = static_cast<T *>(xv);
  hipStream_t st = c->stream;
  const GeomDev &g = d->gd;

  int hip_[CI_COUNT] = {0};
  double hdp[CD_COUNT] = {0};
  hdp[CD_TAUE] = o->use_dp ? o->tau * o->noise_norm : 0.0;
  hdp[CD_ETAEPS] = 100.0 * (sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16) * 2.0;
  hdp[CD_USEDP] = o->use_dp ? 1.0 : 0.0;
  hdp[CD_KMAX] = o->k_max;
  hdp[CD_RNS] = o->rns_eps;
  HIPC(hipMemcpyAsync(S.ctl.ip, hip_, sizeof hip_, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(S.ctl.dp, hdp, sizeof hdp, hipMemcpyHostToDevice, st));
  *c->host_flag = 0;
  if (S.fusing()) {
    HIPC(hipMemsetAsync(S.xpad, 0, sizeof(T) * (size_t)g.pad_elems, st));
    HIPC(hipMemsetAsync(S.ypad, 0, sizeof(T) * (size_t)g.ypad_elems, st));
    if (g.kind == GKB_FAN2D) HIPC(hipMemsetAsync(S.ywpad, 0, 2 * sizeof(T) * (size_t)g.ypad_elems, st));
  }
  S.forget_pads();

  // start-up (k = 0): ||b||; r_0 = b (AB) or B b (BA); alpha[1] = ||r_0||; q_1
  launch_resid_init<T>(S.ctl, b, g.m, S.partials, st);
  if (mode == MODE_BA)
    S.B(col<const T>(b), S.w, plain_epi<T>());
  else
    launch_copy<T>(b, S.w, g.m, st);
  launch_norm_to<T>(S.ctl, S.w, S.dimq, NORM_ALPHA1, S.partials, st);
  S.normalize();
  HIPC(hipGetLastError());
  double h2[2];
  HIPC(hipMemcpyAsync(&h2[0], S.ctl.alpha + 1, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipMemcpyAsync(&h2[1], S.ctl.dp + CD_BNORM, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  const double beta = h2[0], bnorm = h2[1];
  if (!std::isfinite(bnorm) || !std::isfinite(beta))
    return fail(GKB_ENONFINITE, "non-finite value in b (or in the start-up vector)");
  gkb_solve_info inf{};
  inf.t1 = beta;
  int k_stop = 0, reason = 0;
  std::vector<double> al(o->k_max + 2, 0.0);
  if (!(beta > 0.0)) {
    HIPC(hipMemsetAsync(x, 0, sizeof(T) * (size_t)g.n, st));
    HIPC(hipStreamSynchronize(st));
    reason = GKB_STOP_BREAKDOWN;
    inf.residual = bnorm;
  } else {
    launch_set_int(S.ctl.ip + CI_K, 1, st);
    const int L = 4;
    std::vector<hipEvent_t> evs(L, nullptr);
    for (auto &e : evs) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const T *x_true = (o->x_true && o->rre_history) ? static_cast<const T *>(o->x_true) : nullptr;
    if (x_true) launch_norm_to<T>(S.ctl, x_true, g.n, NORM_XTRUE, S.partials, st);
    for (int k = 1; k <= o->k_max; ++k) {
      S.gm_iteration(k, b);
      if (x_true) S.rre_step(x_true);
      HIPC(hipEventRecord(evs[k % L], st));
      if (k >= L) {
        HIPC(hipEventSynchronize(evs[(k - L + 1) % L]));
        if (*(volatile int *)c->host_flag) break;
      }
    }
    HIPC(hipGetLastError());
    S.forget_pads();
    if (mode == MODE_AB) {
      launch_solution<T>(S.ctl, S.Q, S.ldq, S.dimq, S.tm, st);
      S.B(col<const T>(S.tm), x, plain_epi<T>(), nullptr);
    } else {
      launch_solution<T>(S.ctl, S.Q, S.ldq, S.dimq, x, st);
    }
    HIPC(hipGetLastError());
    int hi[CI_COUNT];
    HIPC(hipMemcpyAsync(hi, S.ctl.ip, sizeof hi, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (auto &e : evs) (void)hipEventDestroy(e);
    k_stop = hi[CI_KSTOP];
    reason = hi[CI_REASON];
    std::vector<double> rho(o->k_max + 2), pres(o->k_max + 2);
    HIPC(hipMemcpy(rho.data(), S.ctl.rho, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(pres.data(), S.ctl.pres, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    HIPC(hipMemcpy(al.data(), S.ctl.alpha, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
    inf.residual = rho[k_stop];
    inf.proj_residual = pres[k_stop];
    inf.alpha1 = al[2];
    if (o->residual_history)
      for (int k = 1; k <= k_stop; ++k) o->residual_history[k - 1] = rho[k];
    if (x_true) {
      std::vector<double> rre(o->k_max + 2);
      HIPC(hipMemcpy(rre.data(), S.ctl.rre, sizeof(double) * (o->k_max + 2), hipMemcpyDeviceToHost));
      for (int k = 1; k <= k_stop; ++k) o->rre_history[k - 1] = rre[k];
    }
  }
  al[1] = beta;
  // alpha_history: ||r_0||, then h_{k+1,k} for k = 1..k_stop; t_history: zeros
  for (int k = 1; k <= o->k_max + 1; ++k) {
    if (o->alpha_history) o->alpha_history[k - 1] = (k <= k_stop + 1) ? al[k] : 0.0;
    if (o->t_history) o->t_history[k - 1] = 0.0;
  }
  inf.k_stop = k_stop;
  inf.reason = reason;
  inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  if (info) *info = inf;
  return GKB_OK;
}

gkb_status validate_opts(const gkb_solve_opts *o) {
  if (o->k_max < 1 || o->k_max > 4096) return fail(GKB_EINVAL, "k_max must be in [1, 4096]");
  if (!(o->lambda >= 0.0) || !std::isfinite(o->lambda)) return fail(GKB_EINVAL, "lambda must be finite and >= 0");
  if (o->use_dp && (!(o->tau > 0.0) || !std::isfinite(o->tau)))
    return fail(GKB_EINVAL, "tau must be > 0 when the discrepancy principle is on");
  if (o->use_dp && (!(o->noise_norm >= 0.0) || !std::isfinite(o->noise_norm)))
    return fail(GKB_EINVAL, "noise_norm must be finite and >= 0");
  if (!(o->rns_eps >= 0.0) || !std::isfinite(o->rns_eps)) return fail(GKB_EINVAL, "rns_eps must be finite and >= 0");
  if ((o->x_true == nullptr) != (o->rre_history == nullptr))
    return fail(GKB_EINVAL, "x_true and rre_history are given together");
  return GKB_OK;
}

gkb_status gm_entry(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o, void *x,
                    gkb_solve_info *info, int mode) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!o) return fail(GKB_EINVAL, "options are NULL");
  if (!b || !x) return fail(GKB_EINVAL, "data pointer is NULL");
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  st = validate_opts(o);
  if (st != GKB_OK) return st;
  if (o->k_max > kGmMaxK) return fail(GKB_EINVAL, "GMRES: k_max must be <= 1024");
  if (o->lambda != 0.0) return fail(GKB_EUNSUPPORTED, "GMRES has no Tikhonov term (lambda must be 0)");
  if (o->precond) return fail(GKB_EUNSUPPORTED, "the learned filter is for BA-GKB only");
  HIPC(hipSetDevice(c->device));
  return dtype == GKB_F32 ? gm_solve_impl<float>(c, g, dtype, b, o, x, info, mode)
                          : gm_solve_impl<double>(c, g, dtype, b, o, x, info, mode);
}

gkb_status hy_entry(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                    const gkb_hybrid_opts *h, void *x, gkb_solve_info *info, int mode) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!o || !h) return fail(GKB_EINVAL, "options are NULL");
  if (!b || !x) return fail(GKB_EINVAL, "data pointer is NULL");
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  st = validate_opts(o);
  if (st != GKB_OK) return st;
  if (o->precond) return fail(GKB_EUNSUPPORTED, "hybrid solves take no learned filter");
  if (o->k_max > kHyMaxK) return fail(GKB_EINVAL, "hybrid and TSVD solves: k_max must be <= 1024");
  if (o->lambda != 0.0) return fail(GKB_EINVAL, "hybrid and TSVD solves choose lambda themselves (lambda must be 0)");
  if (h->lambda_rule < GKB_LAMBDA_FIXED || h->lambda_rule > GKB_LAMBDA_GCV)
    return fail(GKB_EINVAL, "lambda_rule must be GKB_LAMBDA_FIXED, GKB_LAMBDA_DP or GKB_LAMBDA_GCV");
  if ((h->lambda_rule == GKB_LAMBDA_FIXED) == (h->tsvd_rank == 0))
    return fail(GKB_EINVAL, "give either a lambda rule or a TSVD rank");
  if (h->tsvd_rank < 0 || h->tsvd_rank > o->k_max) return fail(GKB_EINVAL, "tsvd_rank must be in [1, k_max]");
  if (h->lambda_rule == GKB_LAMBDA_DP &&
      (!(h->tau_proj >= 0.0) || !std::isfinite(h->tau_proj) || !(h->eta_proj >= 0.0) || !std::isfinite(h->eta_proj)))
    return fail(GKB_EINVAL, "tau_proj and eta_proj must be finite and >= 0");
  HIPC(hipSetDevice(c->device));
  return dtype == GKB_F32 ? solve_impl<float>(c, g, dtype, b, o, x, info, mode, h)
                          : solve_impl<double>(c, g, dtype, b, o, x, info, mode, h);
}

gkb_status solve_entry(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                       void *x, gkb_solve_info *info, int mode) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (!o) return fail(GKB_EINVAL, "options are NULL");
  if (!b || !x) return fail(GKB_EINVAL, "data pointer is NULL");
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  st = validate_opts(o);
  if (st != GKB_OK) return st;
  HIPC(hipSetDevice(c->device));
  if (o->precond) {
    if (mode != MODE_BA) return fail(GKB_EUNSUPPORTED, "the learned filter sits inside B: BA-GKB only");
    if (dtype != GKB_F32) return fail(GKB_EUNSUPPORTED, "the learned filter runs in FP32 (GKB_F32)");
    st = net_check(c, o->precond);
    if (st != GKB_OK) return st;
    // learned solve; plain BA-GKB is the fallback when the learned one does
    // not reach the discrepancy level, breaks down early or meets a
    // non-finite value.  With the discrepancy principle on, the attempt also
    // ends once its residual, at its mean decrease over the last five
    // iterations, would still be above the level at k_max: a residual that
    // levels off above the level then costs the iterations up to that point
    // instead of k_max before the fallback.
    gkb_solve_info li{};
    st = solve_impl<float>(c, g, dtype, b, o, x, &li, mode);
    // with the discrepancy principle on, the learned solution is kept only if
    // it meets the discrepancy level, whatever stopped the iteration (a
    // residual-stagnation stop above the level falls back as well)
    const bool dp_missed = o->use_dp && !(li.residual <= o->tau * o->noise_norm);
    const bool bad = st == GKB_ENONFINITE ||
                     (st == GKB_OK && (li.reason == GKB_STOP_DP_NOT_REACHED || dp_missed || !(li.t1 > 0.0) ||
                                       (li.reason == GKB_STOP_BREAKDOWN && li.k_stop < 3)));
    if (!bad) {
      if (st == GKB_OK && info) *info = li;
      return st;
    }
    gkb_solve_opts po = *o;
    po.precond = nullptr;
    gkb_solve_info pi{};
    st = solve_impl<float>(c, g, dtype, b, &po, x, &pi, mode);
    if (st != GKB_OK) return st;
    pi.reason = GKB_STOP_FALLBACK;
    pi.seconds += li.seconds;
    if (info) *info = pi;
    return GKB_OK;
  }
  return dtype == GKB_F32 ? solve_impl<float>(c, g, dtype, b, o, x, info, mode)
                          : solve_impl<double>(c, g, dtype, b, o, x, info, mode);
}

// --------------------------------------------------------------------------
// batched multi-slice driver: every launch covers all active slices
// --------------------------------------------------------------------------
inline size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

struct SliceHost {
  const DevTables *d;
  long long n, m, dimq, dims, ldq;
  int K;
  int cnt[BF_COUNT];
  // byte offsets into the vector workspace
  size_t oQ, oyk, os, ow, otn, otm, oxp, oyp;
  // element offsets into the double workspace (control arrays, residual
  // vectors Aw and r, partials)
  size_t oarr, ores, opart, ogram;
};

// Launch map of the slices in `active` (slice ids): the active list followed
// by the per-family prefix sums.
void build_map(const std::vector<SliceHost> &sh, const std::vector<int> &active, std::vector<int> &buf,
               BatchLaunch &bl) {
  const int na = (int)active.size();
  buf.assign(na + BF_COUNT * (na + 1), 0);
  for (int a = 0; a < na; ++a) buf[a] = active[a];
  for (int f = 0; f < BF_COUNT; ++f) {
    int *pre = buf.data() + na + f * (na + 1);
    pre[0] = 0;
    for (int a = 0; a < na; ++a) pre[a + 1] = pre[a] + sh[active[a]].cnt[f];
    bl.tot[f] = pre[na];
  }
  bl.na = na;
}

// Stages a launch map through one of two pinned slots and copies it to the
// device map buffer, ordered on the stream after every earlier launch.
gkb_status upload_map(gkb_ctx *c, const std::vector<int> &buf) {
  const int j = (int)(c->bpin_slot++ & 1);
  const size_t slot_ints = c->bmap.bytes / sizeof(int);
  if (buf.size() > slot_ints) return fail(GKB_EINVAL, "internal: launch map larger than its buffer");
  if (c->bpin_ev[j]) HIPC(hipEventSynchronize(c->bpin_ev[j]));
  int *h = c->bpin + (size_t)j * slot_ints;
  std::memcpy(h, buf.data(), sizeof(int) * buf.size());
  HIPC(hipMemcpyAsync(c->bmap.p, h, sizeof(int) * buf.size(), hipMemcpyHostToDevice, c->stream));
  if (!c->bpin_ev[j]) HIPC(hipEventCreateWithFlags(&c->bpin_ev[j], hipEventDisableTiming));
  HIPC(hipEventRecord(c->bpin_ev[j], c->stream));
  return GKB_OK;
}

template <typename T>
gkb_status batch_impl(gkb_ctx *c, int mode, int ns, const gkb_geometry *geoms, int dtype, const void *const *bv,
                      const gkb_solve_opts *opts, void *const *xv, gkb_solve_info *info) {
  auto t_start = std::chrono::steady_clock::now();
  hipStream_t st = c->stream;
  std::vector<SliceHost> sh(ns);
  BatchLaunch bl{};
  bl.nc_bt = 2;
  bl.nc_at = 2;
  bl.kmax = 1;
  size_t bytesT = 0, ndbl = (size_t)ns * CD_COUNT;
  double best_pv = 0.0;
  for (int s = 0; s < ns; ++s) {
    DevTables *d = nullptr;
    gkb_status stt = get_tables(c, &geoms[s], dtype, &d);
    if (stt != GKB_OK) return stt;
    const GeomDev &g = d->gd;
    if (s == 0) bl.fan = g.kind == GKB_FAN2D;
    if ((g.kind == GKB_FAN2D) != (bl.fan != 0))
      return fail(GKB_EINVAL, "all slices of a batch must share the geometry kind");
    SliceHost &h = sh[s];
    h.d = d;
    h.n = g.n;
    h.m = g.m;
    h.K = opts[s].k_max;
    h.dimq = mode == MODE_AB ? g.m : g.n;
    h.dims = mode == MODE_BA ? g.n : g.m;
    h.ldq = (h.dimq + 3) / 4 * 4;
    bl.nc_bt = std::max(bl.nc_bt, g.nc_bt);
    bl.nc_at = std::max(bl.nc_at, g.nc_at);
    if (s == 0 || (double)g.n * g.nv > best_pv) {  // the tuned choices of the slice with the most pixel-views
      best_pv = (double)g.n * g.nv;
      bl.at_vu = g.at_vu;
      bl.b_vu = g.b_vu;
    }
    bl.kmax = std::max(bl.kmax, h.K);
    h.cnt[BF_RAY] = ray_blocks(g);
    h.cnt[BF_RAYBT] = bt_blocks(g);
    h.cnt[BF_PIX] = pixel_blocks(g);
    h.cnt[BF_VQ] = vec_blocks(h.dimq);
    h.cnt[BF_VQU] = upd_blocks(h.dimq);
    h.cnt[BF_VQD] = dots_blocks(h.dimq);
    h.cnt[BF_VM] = vec_blocks(g.m);
    h.cnt[BF_PADR] = (int)std::min<long long>(((long long)g.ny * g.ldR + 255) / 256, 2048);
    h.cnt[BF_PADC] = d->has_coldom ? ((g.ldT + 31) / 32) * ((g.nx + 31) / 32) : 0;
    h.cnt[BF_PADS] = (int)std::min<long long>(((long long)g.nv * g.ldY + 255) / 256, 4096);
    auto take = [&](size_t elems) {
      const size_t o = bytesT;
      bytesT += al256(sizeof(T) * elems);
      return o;
    };
    h.oQ = take((size_t)h.ldq * (h.K + 1));
    h.oyk = take((size_t)g.m);
    h.os = take((size_t)h.dims);
    h.ow = take((size_t)h.dimq);
    h.otn = take((size_t)g.n);
    h.otm = take((size_t)g.m);
    h.oxp = take((size_t)g.pad_elems);
    h.oyp = take(2 * (size_t)g.ypad_elems);
    h.oarr = ndbl;
    ndbl += 9 * (size_t)(h.K + 2);
    ndbl = (ndbl + 31) / 32 * 32;
    h.ores = ndbl;
    ndbl += 2 * (size_t)((g.m + 3) / 4 * 4);
    h.ogram = ndbl;
    ndbl += (size_t)(h.K + 1) * (size_t)(h.K + 1);
    ndbl = (ndbl + 31) / 32 * 32;
    h.opart = ndbl;
    ndbl += (size_t)std::max<long long>(
        {(long long)h.cnt[BF_RAY], (long long)h.cnt[BF_RAYBT], (long long)h.cnt[BF_PIX], 2LL * h.cnt[BF_VQD] * (h.K + 2),
         (long long)h.cnt[BF_VQU],
         (long long)h.cnt[BF_VM] * (h.K + 2), 1024LL});
    ndbl = (ndbl + 31) / 32 * 32;
  }
  // workspaces
  HIPC(c->bws.ensure(bytesT));
  HIPC(c->bwd.ensure(sizeof(double) * ndbl));
  HIPC(c->bwi.ensure(sizeof(int) * (size_t)ns * CI_COUNT));
  HIPC(c->bsd.ensure(sizeof(SliceDev<T>) * (size_t)ns));
  const size_t slot_ints = (size_t)ns + BF_COUNT * (size_t)(ns + 1);
  if (c->bmap.bytes < sizeof(int) * slot_ints) {
    HIPC(hipStreamSynchronize(st));
    HIPC(c->bmap.ensure(sizeof(int) * slot_ints));
    if (c->bpin) HIPC(hipHostFree(c->bpin));
    c->bpin = nullptr;
    HIPC(hipHostMalloc((void **)&c->bpin, 2 * c->bmap.bytes, hipHostMallocDefault));
  }
  HIPC(c->brep.ensure(sizeof(double) * 4 * (size_t)ns));
  if (c->bflags_n < ns) {
    HIPC(hipStreamSynchronize(st));
    if (c->bflags) HIPC(hipHostFree(c->bflags));
    c->bflags = nullptr;
    HIPC(hipHostMalloc((void **)&c->bflags, sizeof(int) * ns, hipHostMallocMapped));
    HIPC(hipHostGetDevicePointer((void **)&c->bflags_dev, c->bflags, 0));
    c->bflags_n = ns;
  }
  char *wsT = c->bws.as<char>();
  double *wsD = c->bwd.as<double>();
  int *wsI = c->bwi.as<int>();

  // slice descriptors and control headers
  std::vector<SliceDev<T>> hsd(ns);
  std::vector<double> hdp((size_t)ns * CD_COUNT, 0.0);
  std::vector<int> hip_((size_t)ns * CI_COUNT, 0);
  for (int s = 0; s < ns; ++s) {
    const SliceHost &h = sh[s];
    const gkb_solve_opts &o = opts[s];
    SliceDev<T> &d = hsd[s];
    d.g = h.d->gd;
    d.rt = rt_of<T>(*h.d);
    d.vt = vt_of<T>(*h.d);
    Ctl &ctl = d.ctl;
    ctl.ip = wsI + (size_t)s * CI_COUNT;
    ctl.dp = wsD + (size_t)s * CD_COUNT;
    double *dp = wsD + h.oarr;
    double **arrs[] = {&ctl.alpha, &ctl.t, &ctl.rho, &ctl.pres, &ctl.u, &ctl.Rd, &ctl.Rth, &ctl.Rphi, &ctl.c};
    for (double **a : arrs) {
      *a = dp;
      dp += h.K + 2;
    }
    ctl.rre = nullptr;  // no reconstruction-error histories in batched solves
    ctl.lamh = nullptr;
    ctl.gram = wsD + h.ogram;
    ctl.aw = wsD + h.ores;
    ctl.r = ctl.aw + (h.m + 3) / 4 * 4;
    ctl.K = h.K;
    ctl.host_stop = c->bflags_dev + s;
    d.xpad = reinterpret_cast<T *>(wsT + h.oxp);
    d.ypad = reinterpret_cast<T *>(wsT + h.oyp);
    d.Q = reinterpret_cast<T *>(wsT + h.oQ);
    d.yk = reinterpret_cast<T *>(wsT + h.oyk);
    d.s = reinterpret_cast<T *>(wsT + h.os);
    d.w = reinterpret_cast<T *>(wsT + h.ow);
    d.tn = reinterpret_cast<T *>(wsT + h.otn);
    d.tm = reinterpret_cast<T *>(wsT + h.otm);
    d.b = static_cast<const T *>(bv[s]);
    d.x = static_cast<T *>(xv[s]);
    d.ldq = h.ldq;
    d.dimq = h.dimq;
    d.dims = h.dims;
    d.partials = wsD + h.opart;
    d.has_coldom = h.d->has_coldom ? 1 : 0;
    d.reorth = o.reorth != 0;
    double *hd = hdp.data() + (size_t)s * CD_COUNT;
    hd[CD_TAUE] = o.use_dp ? o.tau * o.noise_norm : 0.0;
    hd[CD_LAMBDA] = o.lambda;
    hd[CD_ETAEPS] = 100.0 * (sizeof(T) == 4 ? 5.9604644775390625e-08 : 1.1102230246251565e-16) * 2.0;
    hd[CD_USEDP] = o.use_dp ? 1.0 : 0.0;
    hd[CD_KMAX] = o.k_max;
    hd[CD_RNS] = o.rns_eps;
    c->bflags[s] = 0;
  }
  HIPC(hipMemcpyAsync(c->bsd.p, hsd.data(), sizeof(SliceDev<T>) * ns, hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(wsD, hdp.data(), sizeof(double) * hdp.size(), hipMemcpyHostToDevice, st));
  HIPC(hipMemcpyAsync(wsI, hip_.data(), sizeof(int) * hip_.size(), hipMemcpyHostToDevice, st));
  const SliceDev<T> *sd = c->bsd.as<const SliceDev<T>>();

  std::vector<int> active(ns), mapbuf;
  for (int s = 0; s < ns; ++s) active[s] = s;
  build_map(sh, active, mapbuf, bl);
  gkb_status stt = upload_map(c, mapbuf);
  if (stt != GKB_OK) return stt;
  BatchDev<T> bd{sd, c->bmap.as<const int>(), c->bmap.as<const int>() + bl.na, bl.na, 0};

  const EpiCfg plain{IN_ONE, PREV_NONE, BS_NONE, 0, BS_NONE};
  auto opA = [&](int in, int out, EpiCfg e) {
    launch_b_pad_image<T>(bd, bl, in, st);
    TraceScope ts(c, "fwd");
    launch_b_fwd<T>(bd, bl, out, e, st);
  };
  auto opBt = [&](int in, int out, EpiCfg e) {
    launch_b_pad_image<T>(bd, bl, in, st);
    TraceScope ts(c, "back_adj");
    launch_b_back_adj<T>(bd, bl, out, e, st);
  };
  auto opB = [&](int in, int out, EpiCfg e) {
    launch_b_pad_sino<T>(bd, bl, in, 0, st);
    TraceScope ts(c, "back");
    launch_b_back<T>(bd, bl, out, e, st);
  };
  auto opAt = [&](int in, int out, EpiCfg e) {
    launch_b_pad_sino<T>(bd, bl, in, 1, st);
    TraceScope ts(c, "fwd_adj");
    launch_b_fwd_adj<T>(bd, bl, out, e, st);
  };
  // w <- M^T s_{k+1} - t_{k+1} q_k   (first: w <- M^T s_1)
  auto apply_Mt = [&](bool first) {
    const EpiCfg e0{IN_INV_TNEXT, PREV_NONE, BS_NONE, 0, BS_NONE};
    const EpiCfg e1 = first ? plain : EpiCfg{IN_ONE, PREV_NEG_TNEXT, BS_Q_PREV, 0, BS_NONE};
    if (mode == MODE_BA) {
      opBt(BS_S, BS_TM, e0);
      opAt(BS_TM, BS_W, e1);
    } else {
      opAt(BS_S, BS_TN, e0);
      opBt(BS_TN, BS_W, e1);
    }
  };

  // start-up (k = 0 in every slice): r_0 = -b, ||b||; s~_1 = rhs, t_1; q_1, alpha_1
  launch_b_resid_init<T>(bd, bl, st);
  if (mode == MODE_BA) {
    opB(BS_B, BS_S, EpiCfg{IN_ONE, PREV_NONE, BS_NONE, 1, BS_NONE});
  } else {
    launch_b_copy<T>(bd, bl, BS_B, BS_S, st);
    launch_b_norm_to<T>(bd, bl, BS_S, BF_VM, NORM_T1, st);
  }
  apply_Mt(true);
  launch_b_norm_to<T>(bd, bl, BS_W, BF_VQ, NORM_ALPHA1, st);
  launch_b_normalize<T>(bd, bl, st);
  launch_b_report<T>(sd, ns, 0, c->brep.as<double>(), st);
  HIPC(hipGetLastError());
  std::vector<double> rep(4 * (size_t)ns);
  HIPC(hipMemcpyAsync(rep.data(), c->brep.p, sizeof(double) * rep.size(), hipMemcpyDeviceToHost, st));
  HIPC(hipStreamSynchronize(st));
  std::vector<gkb_solve_info> inf(ns);
  std::vector<int> loop;
  for (int s = 0; s < ns; ++s) {
    const double t1 = rep[4 * s], bnorm = rep[4 * s + 2];
    const double a1 = t1 > 0.0 ? rep[4 * s + 1] : 0.0;
    if (!std::isfinite(bnorm) || !std::isfinite(t1) || !std::isfinite(a1))
      return fail(GKB_ENONFINITE, "non-finite value in b of slice " + std::to_string(s));
    inf[s] = gkb_solve_info{};
    inf[s].t1 = t1;
    inf[s].alpha1 = a1;
    int *hi = hip_.data() + (size_t)s * CI_COUNT;
    if (!(t1 > 0.0) || !(a1 > 0.0)) {
      hi[CI_STOP] = 1;
      hi[CI_REASON] = GKB_STOP_BREAKDOWN;
      inf[s].reason = GKB_STOP_BREAKDOWN;
      inf[s].residual = bnorm;
      inf[s].proj_residual = t1;
    } else {
      hi[CI_K] = 1;
      loop.push_back(s);
    }
  }
  for (int s = 0; s < ns; ++s)
    if (inf[s].reason == GKB_STOP_BREAKDOWN) HIPC(hipMemsetAsync(xv[s], 0, sizeof(T) * (size_t)sh[s].n, st));
  HIPC(hipMemcpyAsync(wsI, hip_.data(), sizeof(int) * hip_.size(), hipMemcpyHostToDevice, st));

  if (!loop.empty()) {
    active = loop;
    build_map(sh, active, mapbuf, bl);
    stt = upload_map(c, mapbuf);
    if (stt != GKB_OK) return stt;
    bd = BatchDev<T>{sd, c->bmap.as<const int>(), c->bmap.as<const int>() + bl.na, bl.na, 0};
    const int L = 4;
    std::vector<hipEvent_t> evs(L, nullptr);
    for (auto &e : evs) HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // one iteration's launches over the active slices (the kernels read k
    // from the slices' control blocks; the launches do not depend on it)
    auto iteration = [&](int k) {
      // s~ <- M q_k - alpha_k/t_k s~, t_{k+1}, Y_k
      if (mode == MODE_BA) {
        opA(BS_Q_PREV, BS_Y_CUR, plain);
        opB(BS_Y_CUR, BS_S, EpiCfg{IN_ONE, PREV_NEG_ALPHA_OVER_T, BS_S, 1, BS_NONE});
      } else {
        opB(BS_Q_PREV, BS_TN, plain);
        opA(BS_TN, BS_S, EpiCfg{IN_ONE, PREV_NEG_ALPHA_OVER_T, BS_S, 1, BS_Y_CUR});
      }
      apply_Mt(false);
      {
        TraceScope ts(c, "reorth");
        launch_b_dcgs<T>(bd, bl, st);
        launch_b_cgs_update<T>(bd, bl, 1, st);
        launch_b_normalize<T>(bd, bl, st);
      }
      {
        TraceScope ts(c, "small_solve");
        launch_b_small_solve<T>(bd, bl, st);
      }
      {
        TraceScope ts(c, "residual");
        launch_b_resid<T>(bd, bl, st);
      }
    };
    // graph mode: the iteration is captured on the context's capture stream
    // and the executable graph replayed on the solve's stream; a new active
    // set (or unroll) is captured anew
    hipGraphExec_t gexec = nullptr;
    int set_version = 0, graph_key = -1;
    auto release_graph = [&]() {
      if (gexec) (void)hipGraphExecDestroy(gexec);
      gexec = nullptr;
    };
    for (int k = 1; k <= bl.kmax; ++k) {
      if (c->batch_graph) {
        const int key = set_version;
        if (!gexec || key != graph_key) {
          release_graph();
          if (!c->cap_stream) HIPC(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
          const bool tr = c->trace;
          c->trace = false;  // no event records inside the graph
          HIPC(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
          st = c->cap_stream;
          iteration(k);
          st = c->stream;
          c->trace = tr;
          hipGraph_t gr = nullptr;
          const hipError_t ce = hipStreamEndCapture(c->cap_stream, &gr);
          if (ce != hipSuccess) return fail(GKB_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ce));
          const hipError_t ie = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
          (void)hipGraphDestroy(gr);
          if (ie != hipSuccess) return fail(GKB_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(ie));
          graph_key = key;
        }
        TraceScope ts(c, "iteration");
        HIPC(hipGraphLaunch(gexec, st));
      } else {
        iteration(k);
      }
      HIPC(hipEventRecord(evs[k % L], st));
      if (k >= L) {
        HIPC(hipEventSynchronize(evs[(k - L + 1) % L]));
        std::vector<int> still;
        for (int s : active)
          if (!*(volatile int *)(c->bflags + s)) still.push_back(s);
        if (still.empty()) break;
        if (still.size() != active.size()) {
          active.swap(still);
          build_map(sh, active, mapbuf, bl);
          stt = upload_map(c, mapbuf);
          if (stt != GKB_OK) {
            release_graph();
            return stt;
          }
          bd = BatchDev<T>{sd, c->bmap.as<const int>(), c->bmap.as<const int>() + bl.na, bl.na, 0};
          ++set_version;
        }
      }
    }
    release_graph();
    HIPC(hipGetLastError());
    // solutions of every slice that iterated: x = Q u (BA) or B (Q u) (AB)
    active = loop;
    build_map(sh, active, mapbuf, bl);
    stt = upload_map(c, mapbuf);
    if (stt != GKB_OK) return stt;
    bd = BatchDev<T>{sd, c->bmap.as<const int>(), c->bmap.as<const int>() + bl.na, bl.na, 1};
    if (mode == MODE_BA) {
      launch_b_solution<T>(bd, bl, BS_X, st);
    } else {
      launch_b_solution<T>(bd, bl, BS_TM, st);
      opB(BS_TM, BS_X, plain);
    }
    launch_b_report<T>(sd, ns, 1, c->brep.as<double>(), st);
    HIPC(hipGetLastError());
    HIPC(hipMemcpyAsync(rep.data(), c->brep.p, sizeof(double) * rep.size(), hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    for (auto &e : evs) (void)hipEventDestroy(e);
    for (int s : loop) {
      inf[s].k_stop = (int)rep[4 * s];
      inf[s].reason = (int)rep[4 * s + 1];
      inf[s].residual = rep[4 * s + 2];
      inf[s].proj_residual = rep[4 * s + 3];
    }
  }
  // optional histories
  for (int s = 0; s < ns; ++s) {
    const gkb_solve_opts &o = opts[s];
    if (!o.residual_history && !o.alpha_history && !o.t_history) continue;
    const Ctl &ctl = hsd[s].ctl;
    const int K = sh[s].K, ks = inf[s].k_stop;
    std::vector<double> buf(K + 2);
    if (o.residual_history) {
      HIPC(hipMemcpy(buf.data(), ctl.rho, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      for (int k = 1; k <= ks; ++k) o.residual_history[k - 1] = buf[k];
    }
    if (o.alpha_history) {
      HIPC(hipMemcpy(buf.data(), ctl.alpha, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      buf[1] = inf[s].alpha1;  // 0 (not 0/0) when t_1 = 0
      for (int k = 1; k <= K + 1; ++k) o.alpha_history[k - 1] = k <= ks + 1 ? buf[k] : 0.0;
    }
    if (o.t_history) {
      HIPC(hipMemcpy(buf.data(), ctl.t, sizeof(double) * (K + 2), hipMemcpyDeviceToHost));
      for (int k = 1; k <= K + 1; ++k) o.t_history[k - 1] = k <= ks + 1 ? buf[k] : 0.0;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  for (int s = 0; s < ns; ++s) {
    inf[s].seconds = secs;
    if (info) info[s] = inf[s];
  }
  return GKB_OK;
}

gkb_status batch_entry(gkb_ctx *c, int method, int ns, const gkb_geometry *geoms, int dtype,
                       const void *const *b, const gkb_solve_opts *opts, void *const *x, gkb_solve_info *info) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (method != GKB_METHOD_AB && method != GKB_METHOD_BA) return fail(GKB_EINVAL, "method must be AB or BA");
  if (ns < 1 || ns > 1024) return fail(GKB_EINVAL, "n_slices must be in [1, 1024]");
  if (!geoms || !b || !opts || !x) return fail(GKB_EINVAL, "NULL array argument");
  for (int s = 0; s < ns; ++s) {
    gkb_status st = validate_geom(&geoms[s], dtype);
    if (st != GKB_OK) return fail(st, "slice " + std::to_string(s) + ": " + g_err);
    if (geoms[s].kind == GKB_CONE3D) return fail(GKB_EUNSUPPORTED, "batched solves take 2D slices");
    if (opts[s].precond) return fail(GKB_EUNSUPPORTED, "batched solves run without the learned filter");
    if (opts[s].x_true || opts[s].rre_history)
      return fail(GKB_EUNSUPPORTED, "batched solves record no reconstruction-error history");
    st = validate_opts(&opts[s]);
    if (st != GKB_OK) return fail(st, "slice " + std::to_string(s) + ": " + g_err);
    if (!b[s] || !x[s]) return fail(GKB_EINVAL, "slice " + std::to_string(s) + ": data pointer is NULL");
  }
  HIPC(hipSetDevice(c->device));
  const int mode = method == GKB_METHOD_AB ? MODE_AB : MODE_BA;
  return dtype == GKB_F32 ? batch_impl<float>(c, mode, ns, geoms, dtype, b, opts, x, info)
                          : batch_impl<double>(c, mode, ns, geoms, dtype, b, opts, x, info);
}

}  // namespace

// --------------------------------------------------------------------------
// C ABI
// --------------------------------------------------------------------------
extern "C" {

gkb_status gkb_create(gkb_ctx **ctx, int device, void *hip_stream) {
  if (!ctx) return fail(GKB_EINVAL, "ctx out-pointer is NULL");
  *ctx = nullptr;
  int ndev = 0;
  HIPC(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(GKB_EINVAL, "device index out of range");
  HIPC(hipSetDevice(device));
  gkb_status sst = resolve_scratch(device);
  if (sst != GKB_OK) return sst;
  auto *c = new gkb_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);  // NULL: the default stream
  *ctx = c;
  return GKB_OK;
}

void gkb_destroy(gkb_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  c->flush_trace();
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->host_flag) (void)hipHostFree(c->host_flag);
  if (c->bflags) (void)hipHostFree(c->bflags);
  if (c->bpin) (void)hipHostFree(c->bpin);
  for (hipEvent_t e : c->bpin_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

gkb_status gkb_set_stream(gkb_ctx *c, void *hip_stream) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (c->own_stream) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
    c->own_stream = false;
  }
  c->stream = static_cast<hipStream_t>(hip_stream);  // NULL: the default stream
  return GKB_OK;
}

const char *gkb_last_error(void) { return g_err.c_str(); }

gkb_status gkb_forward(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *x, void *y) {
  return projector_call(c, g, dtype, x, y, OP_A);
}
gkb_status gkb_back(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *y, void *x) {
  return projector_call(c, g, dtype, y, x, OP_B);
}
gkb_status gkb_forward_adjoint(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *y, void *x) {
  return projector_call(c, g, dtype, y, x, OP_AT);
}
gkb_status gkb_back_noalloc(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *y, void *x) {
  return back_noalloc(c, g, dtype, y, x);
}

gkb_status gkb_check_geometry(const gkb_geometry *g, int dtype, int stride, gkb_check_stats *stats, int *orders_ok) {
  if (!stats) return fail(GKB_EINVAL, "stats is NULL");
  if (stride < 1) return fail(GKB_EINVAL, "stride must be >= 1");
  gkb_status st = validate_geom(g, dtype);
  if (st != GKB_OK) return st;
  HostTables h;
  CheckStat cs[4] = {};
  int ok = 1;
  if (g->kind == GKB_CONE3D) {
    build_cone_tables(g, h);
    if (!(h.min_ddom > 0.5 * (g->n_det_v - 1) * g->det_pitch_v))
      return fail(GKB_EUNSUPPORTED, "cone beam: some ray would step along z");
    check_tables_cone(g, h, dtype == GKB_F32, stride, cs);
  } else {
    build_tables(g, h);
    if (h.gd.nc_bt > 8 || h.gd.nc_at > 8)
      return fail(GKB_EUNSUPPORTED, "more than 8 interpolation candidates per line");
    ok = check_tables_2d(g, h, dtype == GKB_F32, stride, cs) ? 1 : 0;
  }
  for (int i = 0; i < 4; ++i) {
    stats[i].units = cs[i].units;
    stats[i].reads = cs[i].reads;
    stats[i].out_of_bounds = cs[i].out_of_bounds;
    stats[i].uncovered = cs[i].uncovered;
    stats[i].max_uncovered_weight = cs[i].max_uncovered_weight;
  }
  if (orders_ok) *orders_ok = ok;
  return GKB_OK;
}
gkb_status gkb_back_adjoint(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *x, void *y) {
  return projector_call(c, g, dtype, x, y, OP_BT);
}

gkb_status gkb_ab_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                        void *x, gkb_solve_info *info) {
  return solve_entry(c, g, dtype, b, o, x, info, MODE_AB);
}
gkb_status gkb_ba_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                        void *x, gkb_solve_info *info) {
  return solve_entry(c, g, dtype, b, o, x, info, MODE_BA);
}
gkb_status gkb_gkb_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                         void *x, gkb_solve_info *info) {
  return solve_entry(c, g, dtype, b, o, x, info, MODE_GKB);
}
gkb_status gkb_ab_gmres_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                              void *x, gkb_solve_info *info) {
  return gm_entry(c, g, dtype, b, o, x, info, MODE_AB);
}
gkb_status gkb_ba_gmres_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                              void *x, gkb_solve_info *info) {
  return gm_entry(c, g, dtype, b, o, x, info, MODE_BA);
}

gkb_status gkb_ab_hybrid_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                               const gkb_hybrid_opts *h, void *x, gkb_solve_info *info) {
  return hy_entry(c, g, dtype, b, o, h, x, info, MODE_AB);
}

gkb_status gkb_ba_hybrid_solve(gkb_ctx *c, const gkb_geometry *g, int dtype, const void *b, const gkb_solve_opts *o,
                               const gkb_hybrid_opts *h, void *x, gkb_solve_info *info) {
  return hy_entry(c, g, dtype, b, o, h, x, info, MODE_BA);
}

gkb_status gkb_batch_solve(gkb_ctx *c, int method, int n_slices, const gkb_geometry *geoms, int dtype,
                           const void *const *b, const gkb_solve_opts *opts, void *const *x, gkb_solve_info *info) {
  return batch_entry(c, method, n_slices, geoms, dtype, b, opts, x, info);
}

gkb_status gkb_net_create(gkb_ctx *c, gkb_net **net, int channels, int ksize, int layers, unsigned long long seed) {
  if (!c || !net) return fail(GKB_EINVAL, "NULL argument");
  *net = nullptr;
  if (channels != kNetC || ksize != kNetK || layers != 4)
    return fail(GKB_EUNSUPPORTED, "the built network has 32 channels, kernel 9 and 4 layers");
  HIPC(hipSetDevice(c->device));
  auto nt = std::make_unique<gkb_net>();
  nt->device = c->device;
  const size_t pb = sizeof(float) * kNetParams;
  HIPC(nt->W.ensure(pb));
  HIPC(nt->m.ensure(pb));
  HIPC(nt->v.ensure(pb));
  HIPC(nt->grad.ensure(pb));
  const size_t n1 = (size_t)kNetC * kNetK, n2 = (size_t)kNetC * kNetC * kNetK;
  HIPC(nt->prep.ensure(4 * sizeof(float) * n1 + 4 * 2 * n2 + 256 * 8));
  char *p = nt->prep.as<char>();
  auto take = [&](size_t bytes) {
    char *q = p;
    p += (bytes + 255) & ~size_t(255);
    return q;
  };
  nt->nw.w1 = reinterpret_cast<float *>(take(sizeof(float) * n1));
  nt->nw.w1t = reinterpret_cast<float *>(take(sizeof(float) * n1));
  nt->nw.w4 = reinterpret_cast<float *>(take(sizeof(float) * n1));
  nt->nw.w4t = reinterpret_cast<float *>(take(sizeof(float) * n1));
  nt->nw.w2b = reinterpret_cast<__bf16 *>(take(2 * n2));
  nt->nw.w3b = reinterpret_cast<__bf16 *>(take(2 * n2));
  nt->nw.w2t = reinterpret_cast<__bf16 *>(take(2 * n2));
  nt->nw.w3t = reinterpret_cast<__bf16 *>(take(2 * n2));
  std::vector<float> w;
  he_init(seed, w);
  HIPC(hipMemcpy(nt->W.p, w.data(), pb, hipMemcpyHostToDevice));
  HIPC(hipMemset(nt->m.p, 0, pb));
  HIPC(hipMemset(nt->v.p, 0, pb));
  HIPC(hipMemset(nt->grad.p, 0, pb));
  gkb_status st = net_prepare(nt.get(), c->stream);
  if (st != GKB_OK) return st;
  HIPC(hipStreamSynchronize(c->stream));
  *net = nt.release();
  return GKB_OK;
}

void gkb_net_destroy(gkb_net *net) {
  if (!net) return;
  (void)hipSetDevice(net->device);
  (void)hipDeviceSynchronize();
  delete net;
}

gkb_status gkb_net_set_weights(gkb_net *net, const float *w, long long count) {
  if (!net || !w) return fail(GKB_EINVAL, "NULL argument");
  if (count != kNetParams) return fail(GKB_EINVAL, "expected 19008 weights");
  for (long long i = 0; i < count; ++i)
    if (!std::isfinite(w[i])) return fail(GKB_ENONFINITE, "non-finite weight");
  HIPC(hipSetDevice(net->device));
  HIPC(hipMemcpy(net->W.p, w, sizeof(float) * kNetParams, hipMemcpyHostToDevice));
  HIPC(hipMemset(net->m.p, 0, sizeof(float) * kNetParams));
  HIPC(hipMemset(net->v.p, 0, sizeof(float) * kNetParams));
  net->step = 0;
  gkb_status st = net_prepare(net, nullptr);
  if (st != GKB_OK) return st;
  HIPC(hipDeviceSynchronize());
  return GKB_OK;
}

gkb_status gkb_net_get_weights(const gkb_net *net, float *w, long long count) {
  if (!net || !w) return fail(GKB_EINVAL, "NULL argument");
  if (count != kNetParams) return fail(GKB_EINVAL, "expected 19008 weights");
  HIPC(hipSetDevice(net->device));
  HIPC(hipDeviceSynchronize());
  HIPC(hipMemcpy(w, net->W.p, sizeof(float) * kNetParams, hipMemcpyDeviceToHost));
  return GKB_OK;
}

gkb_status gkb_net_save(const gkb_net *net, const char *path) {
  if (!net || !path) return fail(GKB_EINVAL, "NULL argument");
  std::vector<float> w(kNetParams);
  gkb_status st = gkb_net_get_weights(net, w.data(), kNetParams);
  if (st != GKB_OK) return st;
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(GKB_EINVAL, std::string("cannot open ") + path);
  const char magic[8] = {'G', 'K', 'B', 'N', 'E', 'T', '1', '\0'};
  const int32_t hdr[4] = {kNetC, kNetK, 4, kNetParams};
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(int32_t), 4, f) == 4 &&
            std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  ok = (std::fclose(f) == 0) && ok;
  return ok ? GKB_OK : fail(GKB_EINVAL, std::string("write failed: ") + path);
}

gkb_status gkb_net_load(gkb_net *net, const char *path) {
  if (!net || !path) return fail(GKB_EINVAL, "NULL argument");
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(GKB_EINVAL, std::string("cannot open ") + path);
  char magic[8];
  int32_t hdr[4];
  std::vector<float> w(kNetParams);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "GKBNET1", 8) == 0 &&
            std::fread(hdr, sizeof(int32_t), 4, f) == 4 && hdr[0] == kNetC && hdr[1] == kNetK && hdr[2] == 4 &&
            hdr[3] == kNetParams && std::fread(w.data(), sizeof(float), w.size(), f) == w.size();
  std::fclose(f);
  if (!ok) return fail(GKB_EINVAL, std::string("not a network file of this architecture: ") + path);
  return gkb_net_set_weights(net, w.data(), kNetParams);
}

gkb_status gkb_net_apply(gkb_ctx *c, const gkb_net *net, const gkb_geometry *g, const void *y, void *out) {
  gkb_status st = net_check(c, net);
  if (st != GKB_OK) return st;
  if (!y || !out) return fail(GKB_EINVAL, "data pointer is NULL");
  st = validate_geom(g, GKB_F32);
  if (st != GKB_OK) return st;
  HIPC(hipSetDevice(c->device));
  long long rows;
  int L;
  net_shape(g, rows, L);
  st = net_scratch(c, rows, L);
  if (st != GKB_OK) return st;
  net_chain(c, net, NET_MASKS, Col<const float>{static_cast<const float *>(y), 0, 0, nullptr},
            static_cast<float *>(out), rows, L, nullptr, c->stream);
  HIPC(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_net_frozen_apply(gkb_ctx *c, const gkb_net *net, const gkb_geometry *g, const void *b, const void *y,
                                void *out, int transpose) {
  gkb_status st = net_check(c, net);
  if (st != GKB_OK) return st;
  if (!b || !y || !out) return fail(GKB_EINVAL, "data pointer is NULL");
  st = validate_geom(g, GKB_F32);
  if (st != GKB_OK) return st;
  HIPC(hipSetDevice(c->device));
  long long rows;
  int L;
  net_shape(g, rows, L);
  st = net_scratch(c, rows, L);
  if (st != GKB_OK) return st;
  net_chain(c, net, NET_MASKS, Col<const float>{static_cast<const float *>(b), 0, 0, nullptr}, c->nout.as<float>(),
            rows, L, nullptr, c->stream);
  net_chain(c, net, transpose ? NET_FT : NET_F, Col<const float>{static_cast<const float *>(y), 0, 0, nullptr},
            static_cast<float *>(out), rows, L, nullptr, c->stream);
  HIPC(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_net_grad(gkb_ctx *c, gkb_net *net, const gkb_geometry *g, int batch, const void *b, const void *x,
                        int objective, double *loss, float *grad) {
  gkb_status st = net_check(c, net);
  if (st != GKB_OK) return st;
  if (!b || !x) return fail(GKB_EINVAL, "data pointer is NULL");
  if (batch < 1) return fail(GKB_EINVAL, "batch must be >= 1");
  if (objective != GKB_NET_FBP && objective != GKB_NET_FROZEN) return fail(GKB_EINVAL, "unknown objective");
  st = validate_geom(g, GKB_F32);
  if (st != GKB_OK) return st;
  if (g->kind == GKB_CONE3D) return fail(GKB_EUNSUPPORTED, "training takes 2D geometries");
  HIPC(hipSetDevice(c->device));
  st = net_grad_impl(c, net, g, batch, static_cast<const float *>(b), static_cast<const float *>(x), objective, loss);
  if (st != GKB_OK) return st;
  if (grad) HIPC(hipMemcpy(grad, net->grad.p, sizeof(float) * kNetParams, hipMemcpyDeviceToHost));
  return GKB_OK;
}

gkb_status gkb_net_train_step(gkb_ctx *c, gkb_net *net, const gkb_geometry *g, int batch, const void *b,
                              const void *x, int objective, double lr, double *loss) {
  if (!(lr > 0.0) || !std::isfinite(lr)) return fail(GKB_EINVAL, "lr must be > 0");
  gkb_status st = gkb_net_grad(c, net, g, batch, b, x, objective, loss, nullptr);
  if (st != GKB_OK) return st;
  net->step += 1;
  launch_net_adam(net->W.as<float>(), net->m.as<float>(), net->v.as<float>(), net->grad.as<float>(), kNetParams, lr,
                  0.9, 0.999, 1e-8, net->step, c->stream);
  st = net_prepare(net, c->stream);
  if (st != GKB_OK) return st;
  HIPC(hipGetLastError());
  return GKB_OK;
}

gkb_status gkb_autotune(gkb_ctx *c, const gkb_geometry *g, int dtype, gkb_tuning *t) {
  return autotune(c, g, dtype, t);
}
gkb_status gkb_set_tuning(gkb_ctx *c, const gkb_geometry *g, int dtype, const gkb_tuning *t) {
  return set_tuning(c, g, dtype, t);
}

gkb_status gkb_set_batch_mode(gkb_ctx *c, int mode) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  if (mode != GKB_BATCH_LAUNCHES && mode != GKB_BATCH_GRAPH) return fail(GKB_EINVAL, "unknown batch mode");
  c->batch_graph = mode == GKB_BATCH_GRAPH ? 1 : 0;
  return GKB_OK;
}

gkb_status gkb_trace_enable(gkb_ctx *c, int on) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  c->trace = on != 0;
  return GKB_OK;
}
gkb_status gkb_trace_only(gkb_ctx *c, const char *kernel) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  c->trace_only = kernel ? kernel : "";
  return GKB_OK;
}
gkb_status gkb_trace_reset(gkb_ctx *c) {
  if (!c) return fail(GKB_EINVAL, "context is NULL");
  c->flush_trace();
  c->stats.clear();
  return GKB_OK;
}
gkb_status gkb_trace_get(gkb_ctx *c, const char *kernel, int *count, double *total_ms) {
  if (!c || !kernel) return fail(GKB_EINVAL, "NULL argument");
  c->flush_trace();
  auto it = c->stats.find(kernel);
  if (count) *count = it == c->stats.end() ? 0 : it->second.count;
  if (total_ms) *total_ms = it == c->stats.end() ? 0.0 : it->second.ms;
  return GKB_OK;
}

}  // extern "C"
