// Host-side geometry tables of the 2D and cone-beam projectors: the values
// the kernels read per ray, view and tile, formed in double, and the scalar
// layout of the padded buffers.  Built once per geometry by the library
// (uploaded to the device) and by the host emulation of the kernels' address
// arithmetic.
#pragma once

#include <vector>

#include "../../include/gkb.h"
#include "internal.h"

namespace gkb {

struct HostTables {
  // per ray
  std::vector<double> base, slope, w, h, t0, dt, dperp, dpar;
  std::vector<int> meta, meta_bt;
  std::vector<int> order_fwd, order_bt;  // workgroup dispatch orders of A and B^T
  std::vector<double> wpad;  // fan: 1/|d_dom| in padded sinogram layout
  // per view
  std::vector<double> p0, p1, p2, p3, p4;
  // per bin (fan): (cos, sin) of the fan angle, padded like a sinogram row
  std::vector<double> gcs;
  // fan A^T: per (32x2 pixel tile, view) bound of the candidate half-width, [tile][view]
  std::vector<double> htile;
  bool has_coldom = false;
  double min_along = 1e300;  // fan: smallest source distance of a B^T crossing
  // cone beam, per (view, column)
  std::vector<double> cbase1, cslope1, clmid, clslope, cdxy2, ch1, cpk;
  std::vector<int> cmeta, cmeta_bt;
  bool has_xdom = false, has_ydom = false;
  double min_ddom = 0.0;
  GeomDev gd{};
};

std::vector<double> view_angles(const gkb_geometry *g);
// Lines [lo, hi] (clipped to [0, nlines - 1]; lo > hi when none) on which a
// ray with crossing c(L) = c_mid + (L - mid) * slope has c in [cmin, cmax].
void line_range(double c_mid, double slope, double mid, int nlines, double cmin, double cmax, int &lo, int &hi);
void build_tables(const gkb_geometry *g, HostTables &t);       // GKB_PAR2D, GKB_FAN2D
void build_cone_tables(const gkb_geometry *g, HostTables &t);  // GKB_CONE3D

// Host emulation of the projector kernels' address arithmetic (selfcheck.cpp).
struct CheckStat {
  long long units, reads, out_of_bounds, uncovered;
  double max_uncovered_weight;
  double thr;  // weights above this count as uncovered
};
// stats[0..3]: A, B, A^T, B^T.  Returns false if a dispatch order is not a
// permutation of the launch's workgroups.
bool check_tables_2d(const gkb_geometry *g, const HostTables &t, bool f32, int stride, CheckStat stats[4]);
void check_tables_cone(const gkb_geometry *g, const HostTables &t, bool f32, int stride, CheckStat stats[4]);

}  // namespace gkb
