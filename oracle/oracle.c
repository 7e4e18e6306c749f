/*
 * FP64 CPU oracle for the AB-/BA-GKB method with an unmatched projector pair.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU path.
 *
 * Everything here is written as plainly as possible, in double precision,
 * with no blocking or fusion beyond what the definitions state:
 *
 *  - Joseph's ray-driven forward projector A (Joseph 1982; the paper's A,
 *    Sec. 1 eq. (1)): for every ray, step along the dominant image axis; at
 *    each crossing of a pixel row (column) interpolate linearly between the
 *    two nearest pixel centres of that row (column); multiply the sum by the
 *    step length 1/|d_dom| of the unit ray direction d.  Pixels outside the
 *    image are zero.  Ties |d_x| == |d_y| step along rows.
 *  - The pixel-driven back projector B (the unmatched B != A^T of Sec. 1):
 *    every pixel centre is projected onto the detector of every view and the
 *    sinogram is interpolated linearly between the two nearest bins; bins
 *    outside the detector are zero; no extra scale.
 *  - A^T and B^T are the exact transposes of the discrete A and B, written
 *    in scatter form: the same loops as A and B with the roles of input and
 *    output exchanged (the paper's modified-ASTRA transposes, Sec. 5).
 *  - GKB on M = AB (Alg. "AB-GKB"), M = BA (Alg. "BA-GKB") or M = A (Alg.
 *    "GKB"), read as the Paige-Saunders bidiagonalisation: iteration k forms
 *    s_{k+1}, t_{k+1}, solves the projected problem (eq. proj GKB) with the
 *    (k+1) x k lower bidiagonal C_k, applies the stopping rule, then forms
 *    q_{k+1}, alpha_{k+1} with one-sided reorthogonalisation of q against
 *    all previous q (two classical Gram-Schmidt passes).
 *  - The projected problem min ||C_k u - t_1 e_1||^2 + lambda^2 ||u||^2 is
 *    solved with the SVD of C_k (Sec. 3), computed by one-sided Jacobi.
 *  - Discrepancy principle (eq. DP): stop at the first k with
 *    ||A x_k - b|| <= tau ||e||, the residual evaluated literally with a
 *    fresh application of A to x_k.
 *  - The comparison methods AB-GMRES and BA-GMRES (Sec. 2.1, Algs.
 *    "AB-GMRES" and "BA-GMRES"): Arnoldi with modified Gram-Schmidt on
 *    M = AB or BA, the Hessenberg projected problem (eq. proj) solved with
 *    its SVD, the same stopping rules.
 *
 * Compiled with -ffp-contract=off so that every product is rounded as
 * written.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PAR2D 0
#define OR_FAN2D 1
#define OR_CONE3D 2
#define OR_DENSE 9

typedef struct {
  int kind;
  int nx, ny, nz;
  int nv;          /* views */
  int nu, nw;      /* detector bins along u, rows along v */
  double du, dw;   /* detector pitch (FAN2D: radians) */
  double D;        /* source -> isocentre */
  double SDD;      /* source -> detector (CONE3D) */
  const double *ang; /* nv view angles, radians */
  /* OR_DENSE: explicit matrices, row-major */
  int dm, dn;
  const double *dA;  /* dm x dn */
  const double *dB;  /* dn x dm */
} or_geom;

static long long g_m(const or_geom *g) {
  if (g->kind == OR_DENSE) return g->dm;
  if (g->kind == OR_CONE3D) return (long long)g->nv * g->nw * g->nu;
  return (long long)g->nv * g->nu;
}
static long long g_n(const or_geom *g) {
  if (g->kind == OR_DENSE) return g->dn;
  if (g->kind == OR_CONE3D) return (long long)g->nx * g->ny * g->nz;
  return (long long)g->nx * g->ny;
}

/* ---------------------------------------------------------------------- */
/* 2D parallel beam                                                          */
/* Ray (v,k): { p : p . (cos th, sin th) = s_k },  s_k = (k-(nu-1)/2) du.     */
/* ---------------------------------------------------------------------- */

/* adjoint == 0: y = A x.  adjoint == 1: x = A^T y (scatter). */
static void par_joseph(const or_geom *g, const double *x, double *y, int adjoint) {
  const int nx = g->nx, ny = g->ny, nu = g->nu;
  if (adjoint) memset((void *)x, 0, sizeof(double) * (size_t)nx * ny);
  for (int v = 0; v < g->nv; ++v) {
    const double c = cos(g->ang[v]), s = sin(g->ang[v]);
    if (fabs(c) >= fabs(s)) {
      const double w = 1.0 / fabs(c);
      /* rows: x*(j) = (s_k - y_j sin)/cos */
      if (!adjoint) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nu; ++k) {
          const double sk = (k - (nu - 1) / 2.0) * g->du;
          double acc = 0.0;
          for (int j = 0; j < ny; ++j) {
            const double yj = j - (ny - 1) / 2.0;
            const double xs = (sk - yj * s) / c;
            const double ci = xs + (nx - 1) / 2.0;
            const double fl = floor(ci);
            const int i0 = (int)fl;
            const double f = ci - fl;
            if (i0 >= 0 && i0 < nx) acc += (1.0 - f) * x[(size_t)j * nx + i0];
            if (i0 + 1 >= 0 && i0 + 1 < nx) acc += f * x[(size_t)j * nx + i0 + 1];
          }
          y[(size_t)v * nu + k] = w * acc;
        }
      } else {
        double *xo = (double *)x;
#pragma omp parallel for schedule(static)
        for (int j = 0; j < ny; ++j) {
          const double yj = j - (ny - 1) / 2.0;
          for (int k = 0; k < nu; ++k) {
            const double sk = (k - (nu - 1) / 2.0) * g->du;
            const double xs = (sk - yj * s) / c;
            const double ci = xs + (nx - 1) / 2.0;
            const double fl = floor(ci);
            const int i0 = (int)fl;
            const double f = ci - fl;
            const double val = w * y[(size_t)v * nu + k];
            if (i0 >= 0 && i0 < nx) xo[(size_t)j * nx + i0] += (1.0 - f) * val;
            if (i0 + 1 >= 0 && i0 + 1 < nx) xo[(size_t)j * nx + i0 + 1] += f * val;
          }
        }
      }
    } else {
      const double w = 1.0 / fabs(s);
      /* columns: y*(i) = (s_k - x_i cos)/sin */
      if (!adjoint) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k < nu; ++k) {
          const double sk = (k - (nu - 1) / 2.0) * g->du;
          double acc = 0.0;
          for (int i = 0; i < nx; ++i) {
            const double xi = i - (nx - 1) / 2.0;
            const double ys = (sk - xi * c) / s;
            const double cj = ys + (ny - 1) / 2.0;
            const double fl = floor(cj);
            const int j0 = (int)fl;
            const double f = cj - fl;
            if (j0 >= 0 && j0 < ny) acc += (1.0 - f) * x[(size_t)j0 * nx + i];
            if (j0 + 1 >= 0 && j0 + 1 < ny) acc += f * x[(size_t)(j0 + 1) * nx + i];
          }
          y[(size_t)v * nu + k] = w * acc;
        }
      } else {
        double *xo = (double *)x;
#pragma omp parallel for schedule(static)
        for (int i = 0; i < nx; ++i) {
          const double xi = i - (nx - 1) / 2.0;
          for (int k = 0; k < nu; ++k) {
            const double sk = (k - (nu - 1) / 2.0) * g->du;
            const double ys = (sk - xi * c) / s;
            const double cj = ys + (ny - 1) / 2.0;
            const double fl = floor(cj);
            const int j0 = (int)fl;
            const double f = cj - fl;
            const double val = w * y[(size_t)v * nu + k];
            if (j0 >= 0 && j0 < ny) xo[(size_t)j0 * nx + i] += (1.0 - f) * val;
            if (j0 + 1 >= 0 && j0 + 1 < ny) xo[(size_t)(j0 + 1) * nx + i] += f * val;
          }
        }
      }
    }
  }
}

/* adjoint == 0: x = B y (pixel driven).  adjoint == 1: y = B^T x (scatter). */
static void par_pixel(const or_geom *g, const double *yin, double *xout, const double *xin, double *yout,
                      int adjoint) {
  const int nx = g->nx, ny = g->ny, nu = g->nu, nv = g->nv;
  if (!adjoint) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
      const double yj = j - (ny - 1) / 2.0;
      for (int i = 0; i < nx; ++i) {
        const double xi = i - (nx - 1) / 2.0;
        double acc = 0.0;
        for (int v = 0; v < nv; ++v) {
          const double c = cos(g->ang[v]), s = sin(g->ang[v]);
          const double u = (xi * c + yj * s) / g->du + (nu - 1) / 2.0;
          const double fl = floor(u);
          const int k0 = (int)fl;
          const double f = u - fl;
          if (k0 >= 0 && k0 < nu) acc += (1.0 - f) * yin[(size_t)v * nu + k0];
          if (k0 + 1 >= 0 && k0 + 1 < nu) acc += f * yin[(size_t)v * nu + k0 + 1];
        }
        xout[(size_t)j * nx + i] = acc;
      }
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v) {
      const double c = cos(g->ang[v]), s = sin(g->ang[v]);
      double *row = yout + (size_t)v * nu;
      for (int k = 0; k < nu; ++k) row[k] = 0.0;
      for (int j = 0; j < ny; ++j) {
        const double yj = j - (ny - 1) / 2.0;
        for (int i = 0; i < nx; ++i) {
          const double xi = i - (nx - 1) / 2.0;
          const double u = (xi * c + yj * s) / g->du + (nu - 1) / 2.0;
          const double fl = floor(u);
          const int k0 = (int)fl;
          const double f = u - fl;
          const double val = xin[(size_t)j * nx + i];
          if (k0 >= 0 && k0 < nu) row[k0] += (1.0 - f) * val;
          if (k0 + 1 >= 0 && k0 + 1 < nu) row[k0 + 1] += f * val;
        }
      }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* 2D fan beam, curved equiangular detector                                  */
/* Source S = D (cos b, sin b); central direction c = -(cos b, sin b);        */
/* bin k at fan angle g_k = (k-(nu-1)/2) du, counter-clockwise from c; ray    */
/* direction d = -(cos(b+g_k), sin(b+g_k)).                                  */
/* ---------------------------------------------------------------------- */
static void fan_joseph_ray(const or_geom *g, int v, int k, const double *x, double *xo, double yval,
                           double *out) {
  const int nx = g->nx, ny = g->ny, nu = g->nu;
  const double b = g->ang[v];
  const double Sx = g->D * cos(b), Sy = g->D * sin(b);
  const double gam = (k - (nu - 1) / 2.0) * g->du;
  const double dx = -cos(b + gam), dy = -sin(b + gam);
  double acc = 0.0;
  if (fabs(dy) >= fabs(dx)) {
    const double w = 1.0 / fabs(dy);
    for (int j = 0; j < ny; ++j) {
      const double yj = j - (ny - 1) / 2.0;
      const double xs = Sx + (yj - Sy) * dx / dy;
      const double ci = xs + (nx - 1) / 2.0;
      const double fl = floor(ci);
      const int i0 = (int)fl;
      const double f = ci - fl;
      if (x) {
        if (i0 >= 0 && i0 < nx) acc += (1.0 - f) * x[(size_t)j * nx + i0];
        if (i0 + 1 >= 0 && i0 + 1 < nx) acc += f * x[(size_t)j * nx + i0 + 1];
      } else {
        if (i0 >= 0 && i0 < nx) xo[(size_t)j * nx + i0] += (1.0 - f) * w * yval;
        if (i0 + 1 >= 0 && i0 + 1 < nx) xo[(size_t)j * nx + i0 + 1] += f * w * yval;
      }
    }
    acc *= w;
  } else {
    const double w = 1.0 / fabs(dx);
    for (int i = 0; i < nx; ++i) {
      const double xi = i - (nx - 1) / 2.0;
      const double ys = Sy + (xi - Sx) * dy / dx;
      const double cj = ys + (ny - 1) / 2.0;
      const double fl = floor(cj);
      const int j0 = (int)fl;
      const double f = cj - fl;
      if (x) {
        if (j0 >= 0 && j0 < ny) acc += (1.0 - f) * x[(size_t)j0 * nx + i];
        if (j0 + 1 >= 0 && j0 + 1 < ny) acc += f * x[(size_t)(j0 + 1) * nx + i];
      } else {
        if (j0 >= 0 && j0 < ny) xo[(size_t)j0 * nx + i] += (1.0 - f) * w * yval;
        if (j0 + 1 >= 0 && j0 + 1 < ny) xo[(size_t)(j0 + 1) * nx + i] += f * w * yval;
      }
    }
    acc *= w;
  }
  if (out) *out = acc;
}

static void fan_joseph(const or_geom *g, const double *x, double *y, int adjoint) {
  const int nu = g->nu, nv = g->nv;
  if (!adjoint) {
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v)
      for (int k = 0; k < nu; ++k) fan_joseph_ray(g, v, k, x, NULL, 0.0, &y[(size_t)v * nu + k]);
  } else {
    /* x = A^T y: scatter every ray into a private image per thread, then
       add the images in a fixed order. */
    const size_t n = (size_t)g->nx * g->ny;
    double *xo = (double *)x;
    memset(xo, 0, sizeof(double) * n);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nth * n, sizeof(double));
#pragma omp parallel
    {
      int t = 0;
#ifdef _OPENMP
      t = omp_get_thread_num();
#endif
      double *mine = priv + (size_t)t * n;
#pragma omp for schedule(static)
      for (int v = 0; v < nv; ++v)
        for (int k = 0; k < nu; ++k) fan_joseph_ray(g, v, k, NULL, mine, y[(size_t)v * nu + k], NULL);
    }
    for (int t = 0; t < nth; ++t)
      for (size_t p = 0; p < n; ++p) xo[p] += priv[(size_t)t * n + p];
    free(priv);
  }
}

static void fan_pixel(const or_geom *g, const double *yin, double *xout, const double *xin, double *yout,
                      int adjoint) {
  const int nx = g->nx, ny = g->ny, nu = g->nu, nv = g->nv;
  if (!adjoint) {
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
      const double yj = j - (ny - 1) / 2.0;
      for (int i = 0; i < nx; ++i) {
        const double xi = i - (nx - 1) / 2.0;
        double acc = 0.0;
        for (int v = 0; v < nv; ++v) {
          const double b = g->ang[v];
          const double Sx = g->D * cos(b), Sy = g->D * sin(b);
          const double cx = -cos(b), cy = -sin(b);
          const double wx = xi - Sx, wy = yj - Sy;
          const double gam = atan2(cx * wy - cy * wx, cx * wx + cy * wy);
          const double u = gam / g->du + (nu - 1) / 2.0;
          const double fl = floor(u);
          const int k0 = (int)fl;
          const double f = u - fl;
          if (k0 >= 0 && k0 < nu) acc += (1.0 - f) * yin[(size_t)v * nu + k0];
          if (k0 + 1 >= 0 && k0 + 1 < nu) acc += f * yin[(size_t)v * nu + k0 + 1];
        }
        xout[(size_t)j * nx + i] = acc;
      }
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v) {
      const double b = g->ang[v];
      const double Sx = g->D * cos(b), Sy = g->D * sin(b);
      const double cx = -cos(b), cy = -sin(b);
      double *row = yout + (size_t)v * nu;
      for (int k = 0; k < nu; ++k) row[k] = 0.0;
      for (int j = 0; j < ny; ++j) {
        const double yj = j - (ny - 1) / 2.0;
        for (int i = 0; i < nx; ++i) {
          const double xi = i - (nx - 1) / 2.0;
          const double wx = xi - Sx, wy = yj - Sy;
          const double gam = atan2(cx * wy - cy * wx, cx * wx + cy * wy);
          const double u = gam / g->du + (nu - 1) / 2.0;
          const double fl = floor(u);
          const int k0 = (int)fl;
          const double f = u - fl;
          const double val = xin[(size_t)j * nx + i];
          if (k0 >= 0 && k0 < nu) row[k0] += (1.0 - f) * val;
          if (k0 + 1 >= 0 && k0 + 1 < nu) row[k0 + 1] += f * val;
        }
      }
    }
  }
}

/* ---------------------------------------------------------------------- */
/* 3D cone beam, flat detector                                               */
/* Source S = D (cos b, sin b, 0).  The detector plane is perpendicular to    */
/* the central ray at distance SDD from the source; its u axis is             */
/* eu = (-sin b, cos b, 0), its v axis ez.  Pixel (k, l) centre:              */
/* S + SDD*c + (k-(nu-1)/2) du eu + (l-(nw-1)/2) dw ez, c = -(cos b, sin b,0).*/
/* Joseph-3D: step along the dominant axis of the ray direction; at every     */
/* crossing of a voxel plane interpolate bilinearly in that plane; weight     */
/* 1/|d_dom|.  B: voxel centre projected onto the detector, bilinear          */
/* interpolation over the 4 nearest detector pixels.                         */
/* ---------------------------------------------------------------------- */
static double vox(const or_geom *g, const double *x, int i, int j, int l) {
  if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || l < 0 || l >= g->nz) return 0.0;
  return x[((size_t)l * g->ny + j) * g->nx + i];
}
static void vox_add(const or_geom *g, double *x, int i, int j, int l, double val) {
  if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || l < 0 || l >= g->nz) return;
  x[((size_t)l * g->ny + j) * g->nx + i] += val;
}

/* source S, unit direction d and dominant axis of the ray of detector pixel
   (k, row) in view v */
static int cone_ray_setup(const or_geom *g, int v, int row, int k, double S[3], double d[3]) {
  const double b = g->ang[v];
  S[0] = g->D * cos(b);
  S[1] = g->D * sin(b);
  S[2] = 0.0;
  const double cdir[3] = {-cos(b), -sin(b), 0.0};
  const double eu[3] = {-sin(b), cos(b), 0.0};
  const double uu = (k - (g->nu - 1) / 2.0) * g->du;
  const double vv = (row - (g->nw - 1) / 2.0) * g->dw;
  double P[3];
  for (int a = 0; a < 3; ++a) P[a] = S[a] + g->SDD * cdir[a] + uu * eu[a] + (a == 2 ? vv : 0.0);
  double len = 0.0;
  for (int a = 0; a < 3; ++a) {
    d[a] = P[a] - S[a];
    len += d[a] * d[a];
  }
  len = sqrt(len);
  for (int a = 0; a < 3; ++a) d[a] /= len;
  int ax = 0;
  if (fabs(d[1]) > fabs(d[ax])) ax = 1;
  if (fabs(d[2]) > fabs(d[ax])) ax = 2;
  return ax;
}

static void cone_ray(const or_geom *g, int v, int row, int k, const double *x, double *xo, double yval,
                     double *out) {
  double S[3], d[3];
  const int ax = cone_ray_setup(g, v, row, k, S, d);
  const int dims[3] = {g->nx, g->ny, g->nz};
  const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
  const double w = 1.0 / fabs(d[ax]);
  double acc = 0.0;
  for (int t = 0; t < dims[ax]; ++t) {
    const double pa = t - (dims[ax] - 1) / 2.0;
    const double lam = (pa - S[ax]) / d[ax];
    const double p1 = S[a1] + lam * d[a1] + (dims[a1] - 1) / 2.0;
    const double p2 = S[a2] + lam * d[a2] + (dims[a2] - 1) / 2.0;
    const double f1 = floor(p1), f2 = floor(p2);
    const int i1 = (int)f1, i2 = (int)f2;
    const double r1 = p1 - f1, r2 = p2 - f2;
    for (int e2 = 0; e2 < 2; ++e2)
      for (int e1 = 0; e1 < 2; ++e1) {
        const double wt = (e1 ? r1 : 1.0 - r1) * (e2 ? r2 : 1.0 - r2);
        int idx[3];
        idx[ax] = t;
        idx[a1] = i1 + e1;
        idx[a2] = i2 + e2;
        if (x)
          acc += wt * vox(g, x, idx[0], idx[1], idx[2]);
        else
          vox_add(g, xo, idx[0], idx[1], idx[2], wt * w * yval);
      }
  }
  if (out) *out = w * acc;
}

static void cone_joseph(const or_geom *g, const double *x, double *y, int adjoint) {
  const int nu = g->nu, nw = g->nw, nv = g->nv;
  if (!adjoint) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int v = 0; v < nv; ++v)
      for (int r = 0; r < nw; ++r)
        for (int k = 0; k < nu; ++k) cone_ray(g, v, r, k, x, NULL, 0.0, &y[((size_t)v * nw + r) * nu + k]);
  } else {
    const size_t n = (size_t)g->nx * g->ny * g->nz;
    double *xo = (double *)x;
    memset(xo, 0, sizeof(double) * n);
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *priv = (double *)calloc((size_t)nth * n, sizeof(double));
#pragma omp parallel
    {
      int t = 0;
#ifdef _OPENMP
      t = omp_get_thread_num();
#endif
      double *mine = priv + (size_t)t * n;
#pragma omp for schedule(static)
      for (int v = 0; v < nv; ++v)
        for (int r = 0; r < nw; ++r)
          for (int k = 0; k < nu; ++k) cone_ray(g, v, r, k, NULL, mine, y[((size_t)v * nw + r) * nu + k], NULL);
    }
    for (int t = 0; t < nth; ++t)
      for (size_t p = 0; p < n; ++p) xo[p] += priv[(size_t)t * n + p];
    free(priv);
  }
}

/* detector coordinates (u, w) of the point (xi, yj, zl) in the view with
   source angle b, given cos b and sin b */
static void cone_pixel_coords_cs(const or_geom *g, double cb, double sb, double xi, double yj, double zl, double *u,
                                 double *w) {
  const double Sx = g->D * cb, Sy = g->D * sb;
  const double cx = -cb, cy = -sb;
  const double ex = -sb, ey = cb;
  const double px = xi - Sx, py = yj - Sy, pz = zl;
  const double depth = px * cx + py * cy; /* distance along the central ray */
  const double mag = g->SDD / depth;
  *u = (px * ex + py * ey) * mag / g->du + (g->nu - 1) / 2.0;
  *w = pz * mag / g->dw + (g->nw - 1) / 2.0;
}

static void cone_pixel_coords(const or_geom *g, int v, double xi, double yj, double zl, double *u, double *w) {
  const double b = g->ang[v];
  cone_pixel_coords_cs(g, cos(b), sin(b), xi, yj, zl, u, w);
}

/* (B y) at voxel (i, j, l): the sum over views of the bilinear interpolation
   of y at the voxel's detector coordinates. */
static double cone_back_voxel(const or_geom *g, const double *yin, int i, int j, int l) {
  const int nx = g->nx, ny = g->ny, nz = g->nz, nu = g->nu, nw = g->nw, nv = g->nv;
  double acc = 0.0;
  for (int v = 0; v < nv; ++v) {
    double u, w;
    cone_pixel_coords(g, v, i - (nx - 1) / 2.0, j - (ny - 1) / 2.0, l - (nz - 1) / 2.0, &u, &w);
    const double fu = floor(u), fw = floor(w);
    const int k0 = (int)fu, r0 = (int)fw;
    const double a = u - fu, c = w - fw;
    for (int e2 = 0; e2 < 2; ++e2)
      for (int e1 = 0; e1 < 2; ++e1) {
        const int kk = k0 + e1, rr = r0 + e2;
        if (kk < 0 || kk >= nu || rr < 0 || rr >= nw) continue;
        acc += (e1 ? a : 1.0 - a) * (e2 ? c : 1.0 - c) * yin[((size_t)v * nw + rr) * nu + kk];
      }
  }
  return acc;
}

static void cone_pixel(const or_geom *g, const double *yin, double *xout, const double *xin, double *yout,
                       int adjoint) {
  const int nx = g->nx, ny = g->ny, nz = g->nz, nu = g->nu, nw = g->nw, nv = g->nv;
  if (!adjoint) {
#pragma omp parallel for collapse(2) schedule(static)
    for (int l = 0; l < nz; ++l)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) xout[((size_t)l * ny + j) * nx + i] = cone_back_voxel(g, yin, i, j, l);
  } else {
#pragma omp parallel for schedule(static)
    for (int v = 0; v < nv; ++v) {
      double *view = yout + (size_t)v * nw * nu;
      for (size_t q = 0; q < (size_t)nw * nu; ++q) view[q] = 0.0;
      for (int l = 0; l < nz; ++l)
        for (int j = 0; j < ny; ++j)
          for (int i = 0; i < nx; ++i) {
            double u, w;
            cone_pixel_coords(g, v, i - (nx - 1) / 2.0, j - (ny - 1) / 2.0, l - (nz - 1) / 2.0, &u, &w);
            const double fu = floor(u), fw = floor(w);
            const int k0 = (int)fu, r0 = (int)fw;
            const double a = u - fu, c = w - fw;
            const double val = xin[((size_t)l * ny + j) * nx + i];
            for (int e2 = 0; e2 < 2; ++e2)
              for (int e1 = 0; e1 < 2; ++e1) {
                const int kk = k0 + e1, rr = r0 + e2;
                if (kk < 0 || kk >= nu || rr < 0 || rr >= nw) continue;
                view[(size_t)rr * nu + kk] += (e1 ? a : 1.0 - a) * (e2 ? c : 1.0 - c) * val;
              }
          }
    }
  }
}

/* Cone beam at sampled outputs: the same definitions as cone_joseph (A) and
   cone_pixel (B), evaluated only at the listed detector pixels (A, index
   (v * nw + r) * nu + k) or voxels (B, index (l * ny + j) * nx + i), for
   checks at sizes where the whole operator is too slow on the CPU.
   Returns -1 for a geometry that is not a cone beam or an index out of range. */
int or_cone_forward_sampled(const or_geom *g, const double *x, const long long *ids, long long count,
                            double *out) {
  if (g->kind != OR_CONE3D) return -1;
  const long long m = g_m(g);
  for (long long s = 0; s < count; ++s)
    if (ids[s] < 0 || ids[s] >= m) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (long long s = 0; s < count; ++s) {
    const long long id = ids[s];
    const int k = (int)(id % g->nu), r = (int)((id / g->nu) % g->nw), v = (int)(id / ((long long)g->nu * g->nw));
    cone_ray(g, v, r, k, x, NULL, 0.0, &out[s]);
  }
  return 0;
}

int or_cone_back_sampled(const or_geom *g, const double *y, const long long *ids, long long count, double *out) {
  if (g->kind != OR_CONE3D) return -1;
  const long long n = g_n(g);
  for (long long s = 0; s < count; ++s)
    if (ids[s] < 0 || ids[s] >= n) return -1;
#pragma omp parallel for schedule(dynamic, 16)
  for (long long s = 0; s < count; ++s) {
    const long long id = ids[s];
    const int i = (int)(id % g->nx), j = (int)((id / g->nx) % g->ny), l = (int)(id / ((long long)g->nx * g->ny));
    out[s] = cone_back_voxel(g, y, i, j, l);
  }
  return 0;
}

/* (A^T y) at the listed voxels (index (l * ny + j) * nx + i): the transpose
   of cone_joseph read one output at a time.  Every ray of every view is set
   up as in cone_ray; on the voxel plane along the ray's dominant axis that
   holds the voxel, the ray's bilinear weight on the voxel (nonzero when its
   crossing lies within one voxel in both in-plane coordinates), times
   1/|d_dom| and the ray's value, is summed. */
int or_cone_forward_adjoint_sampled(const or_geom *g, const double *y, const long long *ids, long long count,
                                    double *out) {
  if (g->kind != OR_CONE3D) return -1;
  const long long n = g_n(g);
  for (long long s = 0; s < count; ++s)
    if (ids[s] < 0 || ids[s] >= n) return -1;
  const int nx = g->nx, ny = g->ny, nz = g->nz, nu = g->nu, nw = g->nw, nv = g->nv;
  const int dims[3] = {nx, ny, nz};
  for (long long s = 0; s < count; ++s) {
    const long long id = ids[s];
    const int p[3] = {(int)(id % nx), (int)((id / nx) % ny), (int)(id / ((long long)nx * ny))};
    double acc = 0.0;
#pragma omp parallel for collapse(2) reduction(+ : acc) schedule(static)
    for (int v = 0; v < nv; ++v)
      for (int r = 0; r < nw; ++r)
        for (int k = 0; k < nu; ++k) {
          double S[3], d[3];
          const int ax = cone_ray_setup(g, v, r, k, S, d);
          const int a1 = (ax + 1) % 3, a2 = (ax + 2) % 3;
          const double pa = p[ax] - (dims[ax] - 1) / 2.0;
          const double lam = (pa - S[ax]) / d[ax];
          const double p1 = S[a1] + lam * d[a1] + (dims[a1] - 1) / 2.0;
          const double p2 = S[a2] + lam * d[a2] + (dims[a2] - 1) / 2.0;
          const double w1 = 1.0 - fabs(p1 - p[a1]), w2 = 1.0 - fabs(p2 - p[a2]);
          if (w1 <= 0.0 || w2 <= 0.0) continue;
          acc += w1 * w2 / fabs(d[ax]) * y[((size_t)v * nw + r) * nu + k];
        }
    out[s] = acc;
  }
  return 0;
}

/* (B^T x) at the listed detector pixels (index (v * nw + r) * nu + k): the
   transpose of cone_pixel read one output at a time, i.e. the sum over every
   voxel of the bilinear weight with which the voxel's projection in view v
   reaches pixel (k, r), times the voxel's value. */
int or_cone_back_adjoint_sampled(const or_geom *g, const double *x, const long long *ids, long long count,
                                 double *out) {
  if (g->kind != OR_CONE3D) return -1;
  const long long m = g_m(g);
  for (long long s = 0; s < count; ++s)
    if (ids[s] < 0 || ids[s] >= m) return -1;
  const int nx = g->nx, ny = g->ny, nz = g->nz;
  for (long long s = 0; s < count; ++s) {
    const long long id = ids[s];
    const int k = (int)(id % g->nu), r = (int)((id / g->nu) % g->nw), v = (int)(id / ((long long)g->nu * g->nw));
    const double cb = cos(g->ang[v]), sb = sin(g->ang[v]);
    double acc = 0.0;
#pragma omp parallel for collapse(2) reduction(+ : acc) schedule(static)
    for (int l = 0; l < nz; ++l)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          double u, w;
          cone_pixel_coords_cs(g, cb, sb, i - (nx - 1) / 2.0, j - (ny - 1) / 2.0, l - (nz - 1) / 2.0, &u, &w);
          const double fu = floor(u), fw = floor(w);
          const int e1 = k - (int)fu, e2 = r - (int)fw;
          if (e1 < 0 || e1 > 1 || e2 < 0 || e2 > 1) continue;
          const double a = u - fu, c = w - fw;
          acc += (e1 ? a : 1.0 - a) * (e2 ? c : 1.0 - c) * x[((size_t)l * ny + j) * nx + i];
        }
    out[s] = acc;
  }
  return 0;
}

/* ---------------------------------------------------------------------- */
/* dense operators (explicit tiny matrices for the Krylov pins)              */
/* ---------------------------------------------------------------------- */
static void dense_mv(const double *Mt, int rows, int cols, const double *in, double *out, int trans) {
  if (!trans) {
    for (int r = 0; r < rows; ++r) {
      double acc = 0.0;
      for (int c = 0; c < cols; ++c) acc += Mt[(size_t)r * cols + c] * in[c];
      out[r] = acc;
    }
  } else {
    for (int c = 0; c < cols; ++c) out[c] = 0.0;
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) out[c] += Mt[(size_t)r * cols + c] * in[r];
  }
}

/* ---------------------------------------------------------------------- */
/* public projector entry points                                             */
/* ---------------------------------------------------------------------- */
void or_forward(const or_geom *g, const double *x, double *y) {
  switch (g->kind) {
    case OR_PAR2D: par_joseph(g, x, y, 0); break;
    case OR_FAN2D: fan_joseph(g, x, y, 0); break;
    case OR_CONE3D: cone_joseph(g, x, y, 0); break;
    case OR_DENSE: dense_mv(g->dA, g->dm, g->dn, x, y, 0); break;
  }
}
void or_forward_adjoint(const or_geom *g, const double *y, double *x) {
  switch (g->kind) {
    case OR_PAR2D: par_joseph(g, x, (double *)y, 1); break;
    case OR_FAN2D: fan_joseph(g, x, (double *)y, 1); break;
    case OR_CONE3D: cone_joseph(g, x, (double *)y, 1); break;
    case OR_DENSE: dense_mv(g->dA, g->dm, g->dn, y, x, 1); break;
  }
}
void or_back(const or_geom *g, const double *y, double *x) {
  switch (g->kind) {
    case OR_PAR2D: par_pixel(g, y, x, NULL, NULL, 0); break;
    case OR_FAN2D: fan_pixel(g, y, x, NULL, NULL, 0); break;
    case OR_CONE3D: cone_pixel(g, y, x, NULL, NULL, 0); break;
    case OR_DENSE: dense_mv(g->dB, g->dn, g->dm, y, x, 0); break;
  }
}
void or_back_adjoint(const or_geom *g, const double *x, double *y) {
  switch (g->kind) {
    case OR_PAR2D: par_pixel(g, NULL, NULL, x, y, 1); break;
    case OR_FAN2D: fan_pixel(g, NULL, NULL, x, y, 1); break;
    case OR_CONE3D: cone_pixel(g, NULL, NULL, x, y, 1); break;
    case OR_DENSE: dense_mv(g->dB, g->dn, g->dm, x, y, 1); break;
  }
}

/* ---------------------------------------------------------------------- */
/* small dense linear algebra                                                */
/* ---------------------------------------------------------------------- */
static double dot(const double *a, const double *b, long long n) {
  double s = 0.0;
  for (long long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}
static double nrm2(const double *a, long long n) { return sqrt(dot(a, a, n)); }

/*
 * One-sided Jacobi SVD (Hestenes) of a dense rows x cols matrix W (row-major,
 * rows >= cols), overwritten.  On return: sig[cols] (unsorted), U = W with
 * normalised columns (rows x cols), V (cols x cols, row-major).
 */
int or_jacobi_svd(int rows, int cols, double *W, double *sig, double *V) {
  for (int i = 0; i < cols; ++i)
    for (int j = 0; j < cols; ++j) V[(size_t)i * cols + j] = (i == j) ? 1.0 : 0.0;
  int sweeps = 0;
  for (; sweeps < 100; ++sweeps) {
    int rotated = 0;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        double a = 0.0, b = 0.0, c = 0.0;
        for (int r = 0; r < rows; ++r) {
          const double wp = W[(size_t)r * cols + p], wq = W[(size_t)r * cols + q];
          a += wp * wp;
          b += wq * wq;
          c += wp * wq;
        }
        if (c == 0.0 || fabs(c) <= DBL_EPSILON * sqrt(a * b)) continue;
        rotated = 1;
        /* rotation that zeroes the (p,q) inner product */
        const double zeta = (b - a) / (2.0 * c);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
        for (int r = 0; r < rows; ++r) {
          const double wp = W[(size_t)r * cols + p], wq = W[(size_t)r * cols + q];
          W[(size_t)r * cols + p] = cs * wp - sn * wq;
          W[(size_t)r * cols + q] = sn * wp + cs * wq;
        }
        for (int r = 0; r < cols; ++r) {
          const double vp = V[(size_t)r * cols + p], vq = V[(size_t)r * cols + q];
          V[(size_t)r * cols + p] = cs * vp - sn * vq;
          V[(size_t)r * cols + q] = sn * vp + cs * vq;
        }
      }
    if (!rotated) break;
  }
  for (int p = 0; p < cols; ++p) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += W[(size_t)r * cols + p] * W[(size_t)r * cols + p];
    s = sqrt(s);
    sig[p] = s;
    if (s > 0.0)
      for (int r = 0; r < rows; ++r) W[(size_t)r * cols + p] /= s;
  }
  return sweeps;
}

/*
 * Projected problem (eq. proj GKB) with Tikhonov term:
 *   u = argmin ||C_k u - t1 e1||^2 + lam^2 ||u||^2
 * with C_k the (k+1) x k lower bidiagonal with diagonal alpha[0..k-1] and
 * subdiagonal t[1..k] (t[0] = t_1).  Through the SVD C_k = U S V^T:
 *   u = sum_i  s_i/(s_i^2 + lam^2) * t1 * U[0][i] * V[:, i];
 * for lam == 0 singular values <= (k+1)*eps*s_max are dropped (pseudo-inverse).
 * Also returns ||C_k u - t1 e1|| in *pres and the singular values in sig_out
 * (optional, length k, unsorted).
 */
void or_proj_solve(int k, const double *alpha, const double *t, double lam, double *u, double *pres,
                   double *sig_out) {
  const int rows = k + 1, cols = k;
  double *W = (double *)calloc((size_t)rows * cols, sizeof(double));
  double *V = (double *)calloc((size_t)cols * cols, sizeof(double));
  double *sig = (double *)calloc((size_t)cols, sizeof(double));
  for (int i = 0; i < k; ++i) {
    W[(size_t)i * cols + i] = alpha[i];
    W[(size_t)(i + 1) * cols + i] = t[i + 1];
  }
  or_jacobi_svd(rows, cols, W, sig, V);
  double smax = 0.0;
  for (int i = 0; i < cols; ++i) smax = fmax(smax, sig[i]);
  for (int i = 0; i < cols; ++i) u[i] = 0.0;
  for (int i = 0; i < cols; ++i) {
    if (lam == 0.0 && !(sig[i] > (k + 1) * DBL_EPSILON * smax)) continue;
    const double coef = sig[i] / (sig[i] * sig[i] + lam * lam) * t[0] * W[i]; /* W[0][i] = U[0][i] */
    for (int r = 0; r < cols; ++r) u[r] += coef * V[(size_t)r * cols + i];
  }
  if (pres) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) {
      double cu = 0.0;
      if (r < k) cu += alpha[r] * u[r];
      if (r >= 1) cu += t[r] * u[r - 1];
      if (r == 0) cu -= t[0];
      s += cu * cu;
    }
    *pres = sqrt(s);
  }
  if (sig_out)
    for (int i = 0; i < cols; ++i) sig_out[i] = sig[i];
  free(W);
  free(V);
  free(sig);
}

/* ---------------------------------------------------------------------- */
/* GKB driver                                                                */
/* ---------------------------------------------------------------------- */
#define OR_MODE_AB 0
#define OR_MODE_BA 1
#define OR_MODE_GKB 2

#define OR_STOP_DP 1
#define OR_STOP_KMAX 2
#define OR_STOP_BREAKDOWN 3
#define OR_STOP_DP_NOT_REACHED 4
#define OR_STOP_RNS 6

typedef struct {
  int k_max;
  double lambda;
  int use_dp;
  double tau;
  double noise_norm;
  int reorth; /* 0 none, 1 CGS2 (two classical passes), 2 MGS (one modified pass) */
  double rns_eps; /* > 0: residual norm stagnation test, eq. (RNS); 0 = off */
  const double *xtrue; /* optional [n] exact image: with rre, RRE(x_k) of eq. (RE) per iteration */
  double *rre;         /* optional [k_max]: ||x_k - xtrue|| / ||xtrue||, k = 1..k_stop */
} or_opts;

typedef struct {
  int k_stop;
  int reason;
  double residual;       /* ||A x - b|| at k_stop */
  double proj_residual;  /* ||C_k u - t1 e1|| at k_stop */
  double t1, alpha1;
} or_info;

/* M and M^T applied through the projector pair.  tmp_m / tmp_n are scratch. */
static void apply_M(const or_geom *g, int mode, const double *in, double *out, double *tmp) {
  if (mode == OR_MODE_AB) { /* out (m) = A (B in) */
    or_back(g, in, tmp);
    or_forward(g, tmp, out);
  } else if (mode == OR_MODE_BA) { /* out (n) = B (A in) */
    or_forward(g, in, tmp);
    or_back(g, tmp, out);
  } else {
    or_forward(g, in, out);
  }
}
static void apply_Mt(const or_geom *g, int mode, const double *in, double *out, double *tmp) {
  if (mode == OR_MODE_AB) { /* out (m) = B^T (A^T in) */
    or_forward_adjoint(g, in, tmp);
    or_back_adjoint(g, tmp, out);
  } else if (mode == OR_MODE_BA) { /* out (n) = A^T (B^T in) */
    or_back_adjoint(g, in, tmp);
    or_forward_adjoint(g, tmp, out);
  } else {
    or_forward_adjoint(g, in, out);
  }
}

/*
 * Runs AB-GKB / BA-GKB / GKB.  Outputs:
 *   x (n) solution at k_stop; rho[k_max] residual history ||A x_k - b||;
 *   pres[k_max] projected residuals; alpha[k_max+1], t[k_max+2] (t[0] = t_1);
 *   optional Qout (dimq x (k_max+1), column i contiguous) and Sout (dims x
 *   (k_max+1)) for invariant checks; optional uout (k_max) = u at k_stop.
 * Returns 0, or -1 on invalid arguments.
 */
int or_gkb(const or_geom *g, int mode, const double *b, const or_opts *o, double *x, double *rho, double *pres,
           double *alpha, double *t, double *Qout, double *Sout, double *uout, or_info *info) {
  const long long m = g_m(g), n = g_n(g);
  if (o->k_max < 1) return -1;
  if (o->use_dp && !(o->tau > 0.0)) return -1;
  if (!(o->rns_eps >= 0.0)) return -1;
  const long long dims = (mode == OR_MODE_AB) ? m : (mode == OR_MODE_BA ? n : m); /* s vectors */
  const long long dimq = (mode == OR_MODE_AB) ? m : n;                            /* q vectors */
  const int K = o->k_max;
  double *S = (double *)calloc((size_t)dims * (K + 1), sizeof(double));
  double *Q = (double *)calloc((size_t)dimq * (K + 1), sizeof(double));
  double *p = (double *)calloc((size_t)(dims > dimq ? dims : dimq), sizeof(double));
  double *qt = (double *)calloc((size_t)dimq, sizeof(double));
  double *tmp = (double *)calloc((size_t)(m > n ? m : n), sizeof(double));
  double *xk = (double *)calloc((size_t)n, sizeof(double));
  double *ax = (double *)calloc((size_t)m, sizeof(double));
  double *u = (double *)calloc((size_t)K, sizeof(double));
  double *c1 = (double *)calloc((size_t)K + 1, sizeof(double));
  double *qu = (double *)calloc((size_t)dimq, sizeof(double));
  double bnorm_scale = 0.0;

  for (int i = 0; i <= K; ++i) alpha[i] = 0.0;
  for (int i = 0; i < K + 2; ++i) t[i] = 0.0;
  for (int i = 0; i < K; ++i) {
    rho[i] = 0.0;
    pres[i] = 0.0;
  }
  info->k_stop = 0;
  info->reason = 0;
  info->residual = 0.0;
  info->proj_residual = 0.0;
  memset(x, 0, sizeof(double) * (size_t)n);

  /* right-hand side of the projected system: AB and GKB start from b, BA from B b */
  double *r = S; /* s_1 column */
  if (mode == OR_MODE_BA)
    or_back(g, b, r);
  else
    memcpy(r, b, sizeof(double) * (size_t)dims);
  t[0] = nrm2(r, dims);
  info->t1 = t[0];
  if (!(t[0] > 0.0)) {
    info->reason = OR_STOP_BREAKDOWN;
    info->residual = nrm2(b, m);
    goto done;
  }
  for (long long i = 0; i < dims; ++i) r[i] /= t[0];
  apply_Mt(g, mode, r, qt, tmp);
  alpha[0] = nrm2(qt, dimq);
  info->alpha1 = alpha[0];
  if (!(alpha[0] > 0.0)) {
    info->reason = OR_STOP_BREAKDOWN;
    info->residual = nrm2(b, m);
    goto done;
  }
  for (long long i = 0; i < dimq; ++i) Q[i] = qt[i] / alpha[0];
  bnorm_scale = sqrt(alpha[0] * alpha[0]);

  for (int k = 1; k <= K; ++k) {
    double *qk = Q + (size_t)(k - 1) * dimq;
    double *sk = S + (size_t)(k - 1) * dims;
    double *sn = S + (size_t)k * dims;
    /* (i) s~ = M q_k - alpha_k s_k ; t_{k+1} = ||s~|| */
    apply_M(g, mode, qk, p, tmp);
    for (long long i = 0; i < dims; ++i) sn[i] = p[i] - alpha[k - 1] * sk[i];
    t[k] = nrm2(sn, dims);
    /* (ii) projected solve and solution */
    double pr = 0.0;
    or_proj_solve(k, alpha, t, o->lambda, u, &pr, NULL);
    pres[k - 1] = pr;
    for (long long i = 0; i < dimq; ++i) {
      double acc = 0.0;
      for (int c = 0; c < k; ++c) acc += Q[(size_t)c * dimq + i] * u[c];
      qu[i] = acc;
    }
    if (mode == OR_MODE_AB)
      or_back(g, qu, xk);
    else
      memcpy(xk, qu, sizeof(double) * (size_t)n);
    or_forward(g, xk, ax);
    for (long long i = 0; i < m; ++i) ax[i] -= b[i];
    rho[k - 1] = nrm2(ax, m);
    memcpy(x, xk, sizeof(double) * (size_t)n);
    if (o->xtrue && o->rre) { /* eq. (RE) on the iterate x_k */
      double e2 = 0.0, t2 = 0.0;
      for (long long i = 0; i < n; ++i) {
        const double d = xk[i] - o->xtrue[i];
        e2 += d * d;
        t2 += o->xtrue[i] * o->xtrue[i];
      }
      o->rre[k - 1] = sqrt(e2) / sqrt(t2);
    }
    info->k_stop = k;
    info->residual = rho[k - 1];
    info->proj_residual = pr;
    if (uout)
      for (int c = 0; c < K; ++c) uout[c] = c < k ? u[c] : 0.0;
    /* (iii) discrepancy principle */
    if (o->use_dp && rho[k - 1] <= o->tau * o->noise_norm) {
      info->reason = OR_STOP_DP;
      goto done;
    }
    /* (iii') residual norm stagnation, eq. (RNS): the change of ||A x - b||
     * from x_{k-1} to x_k, relative to ||A x_{k-1} - b||, is below eps;
     * x_k is returned */
    if (o->rns_eps > 0.0 && k >= 2 && fabs(rho[k - 2] - rho[k - 1]) < o->rns_eps * rho[k - 2]) {
      info->reason = OR_STOP_RNS;
      goto done;
    }
    /* breakdown threshold: 100 eps max_i ||(alpha_i, t_{i+1})|| */
    {
      double sc = bnorm_scale;
      const double cand = sqrt(alpha[k - 1] * alpha[k - 1] + t[k] * t[k]);
      if (cand > sc) sc = cand;
      bnorm_scale = sc;
    }
    const double eta = 100.0 * DBL_EPSILON * bnorm_scale;
    if (!(t[k] > eta)) {
      info->reason = OR_STOP_BREAKDOWN;
      goto done;
    }
    for (long long i = 0; i < dims; ++i) sn[i] /= t[k];
    if (k == K) break;
    /* (iv) q~ = M^T s_{k+1} - t_{k+1} q_k; reorthogonalise; alpha_{k+1}, q_{k+1} */
    apply_Mt(g, mode, sn, qt, tmp);
    for (long long i = 0; i < dimq; ++i) qt[i] -= t[k] * qk[i];
    if (o->reorth == 1) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int c = 0; c < k; ++c) c1[c] = dot(Q + (size_t)c * dimq, qt, dimq);
        for (int c = 0; c < k; ++c)
          for (long long i = 0; i < dimq; ++i) qt[i] -= c1[c] * Q[(size_t)c * dimq + i];
      }
    } else if (o->reorth == 2) {
      for (int c = 0; c < k; ++c) {
        const double h = dot(Q + (size_t)c * dimq, qt, dimq);
        for (long long i = 0; i < dimq; ++i) qt[i] -= h * Q[(size_t)c * dimq + i];
      }
    }
    alpha[k] = nrm2(qt, dimq);
    if (!(alpha[k] > eta)) {
      info->reason = OR_STOP_BREAKDOWN;
      goto done;
    }
    for (long long i = 0; i < dimq; ++i) Q[(size_t)k * dimq + i] = qt[i] / alpha[k];
  }
  info->reason = o->use_dp ? OR_STOP_DP_NOT_REACHED : OR_STOP_KMAX;

done:
  if (Qout) memcpy(Qout, Q, sizeof(double) * (size_t)dimq * (K + 1));
  if (Sout) memcpy(Sout, S, sizeof(double) * (size_t)dims * (K + 1));
  free(S);
  free(Q);
  free(p);
  free(qt);
  free(tmp);
  free(xk);
  free(ax);
  free(u);
  free(c1);
  free(qu);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* AB-GMRES and BA-GMRES (the paper's comparison methods, Sec. 2.1)          */
/* ---------------------------------------------------------------------- */
/*
 * AB-GMRES (Alg. "AB-GMRES") and BA-GMRES (Alg. "BA-GMRES") from x_0 = 0.
 * Arnoldi (eq. (Arn iter)) on M = AB with q in R^m and r_0 = b (AB), or on
 * M = BA with q in R^n and r_0 = B b (BA): q_1 = r_0 / ||r_0||; at step k,
 * w = M q_k is orthogonalised against q_1..q_k by one modified Gram-Schmidt
 * pass as printed (h_{i,k} = q_i^T w, w -= h_{i,k} q_i), h_{k+1,k} = ||w||,
 * q_{k+1} = w / h_{k+1,k}.  The projected problem (eq. proj)
 *   u_k = argmin ||H_k u - ||r_0|| e_1||
 * with the (k+1) x k upper Hessenberg H_k is solved through its SVD (Jacobi;
 * singular values <= (k+1) eps s_max dropped).  x_k = B Q_k u_k (AB) or
 * Q_k u_k (BA).  The stopping rules act on the data residual ||A x_k - b||
 * (eqs. DP and RNS), evaluated literally with a fresh application of A;
 * breakdown when h_{k+1,k} <= 100 eps max_i ||H_k(:, i)|| (the Krylov space is
 * invariant and x_k its least-squares solution).  No Tikhonov term
 * (lambda must be 0).
 * Outputs: x (n) at k_stop; rho[k_max]; pres[k_max] = ||H_k u_k - ||r_0|| e_1||;
 * optional Hout ((k_max+1) x k_max row-major, h_{i,j} at [(i-1) k_max + j-1]);
 * optional Qout (dimq x (k_max+1), column i contiguous); info->t1 = ||r_0||,
 * info->alpha1 = h_{2,1}.  Returns 0, or -1 on invalid arguments.
 */
int or_gmres(const or_geom *g, int mode, const double *b, const or_opts *o, double *x, double *rho, double *pres,
             double *Hout, double *Qout, or_info *info) {
  const long long m = g_m(g), n = g_n(g);
  if (o->k_max < 1 || o->lambda != 0.0) return -1;
  if (mode != OR_MODE_AB && mode != OR_MODE_BA) return -1;
  if (o->use_dp && !(o->tau > 0.0)) return -1;
  if (!(o->rns_eps >= 0.0)) return -1;
  const long long dimq = (mode == OR_MODE_AB) ? m : n;
  const int K = o->k_max;
  double *Q = (double *)calloc((size_t)dimq * (K + 1), sizeof(double));
  double *H = (double *)calloc((size_t)(K + 1) * K, sizeof(double));
  double *w = (double *)calloc((size_t)dimq, sizeof(double));
  double *tmp = (double *)calloc((size_t)(m > n ? m : n), sizeof(double));
  double *qu = (double *)calloc((size_t)dimq, sizeof(double));
  double *xk = (double *)calloc((size_t)n, sizeof(double));
  double *ax = (double *)calloc((size_t)m, sizeof(double));
  double *u = (double *)calloc((size_t)K, sizeof(double));
  double *W = (double *)calloc((size_t)(K + 1) * K, sizeof(double));
  double *V = (double *)calloc((size_t)K * K, sizeof(double));
  double *sig = (double *)calloc((size_t)K, sizeof(double));
  double scale = 0.0;
  for (int i = 0; i < K; ++i) {
    rho[i] = 0.0;
    pres[i] = 0.0;
  }
  info->k_stop = 0;
  info->reason = 0;
  info->residual = 0.0;
  info->proj_residual = 0.0;
  info->alpha1 = 0.0;
  memset(x, 0, sizeof(double) * (size_t)n);

  /* r_0 = b (AB) or B b (BA) */
  if (mode == OR_MODE_BA)
    or_back(g, b, w);
  else
    memcpy(w, b, sizeof(double) * (size_t)dimq);
  const double beta = nrm2(w, dimq);
  info->t1 = beta;
  if (!(beta > 0.0)) {
    info->reason = OR_STOP_BREAKDOWN;
    info->residual = nrm2(b, m);
    goto done;
  }
  for (long long i = 0; i < dimq; ++i) Q[i] = w[i] / beta;

  for (int k = 1; k <= K; ++k) {
    const double *qk = Q + (size_t)(k - 1) * dimq;
    /* w = M q_k, orthogonalised against q_1..q_k (modified Gram-Schmidt) */
    apply_M(g, mode, qk, w, tmp);
    for (int i = 1; i <= k; ++i) {
      const double *qi = Q + (size_t)(i - 1) * dimq;
      const double h = dot(qi, w, dimq);
      H[(size_t)(i - 1) * K + (k - 1)] = h;
      for (long long r = 0; r < dimq; ++r) w[r] -= h * qi[r];
    }
    const double hk1 = nrm2(w, dimq);
    H[(size_t)k * K + (k - 1)] = hk1;
    if (k == 1) info->alpha1 = hk1;
    if (hk1 > 0.0) { /* q_{k+1}, used by the next step (and the Arnoldi relation) */
      double *qn = Q + (size_t)k * dimq;
      for (long long i = 0; i < dimq; ++i) qn[i] = w[i] / hk1;
    }
    {
      double cn = 0.0;
      for (int i = 0; i <= k; ++i) cn += H[(size_t)i * K + (k - 1)] * H[(size_t)i * K + (k - 1)];
      if (sqrt(cn) > scale) scale = sqrt(cn);
    }
    /* projected problem through the SVD of H_k: u = sum_i (beta U[0][i] / s_i) V[:, i] */
    for (int r = 0; r <= k; ++r)
      for (int c = 0; c < k; ++c) W[(size_t)r * k + c] = H[(size_t)r * K + c];
    or_jacobi_svd(k + 1, k, W, sig, V);
    double smax = 0.0;
    for (int i = 0; i < k; ++i) smax = fmax(smax, sig[i]);
    for (int i = 0; i < k; ++i) u[i] = 0.0;
    for (int i = 0; i < k; ++i) {
      if (!(sig[i] > (k + 1) * DBL_EPSILON * smax)) continue;
      const double coef = beta * W[i] / sig[i]; /* W[0][i] = U[0][i] */
      for (int r = 0; r < k; ++r) u[r] += coef * V[(size_t)r * k + i];
    }
    {
      double s2 = 0.0;
      for (int r = 0; r <= k; ++r) {
        double hu = r == 0 ? -beta : 0.0;
        for (int c = 0; c < k; ++c) hu += H[(size_t)r * K + c] * u[c];
        s2 += hu * hu;
      }
      pres[k - 1] = sqrt(s2);
    }
    /* x_k = (B) Q_k u_k and the literal residual ||A x_k - b|| */
    for (long long i = 0; i < dimq; ++i) {
      double acc = 0.0;
      for (int c = 0; c < k; ++c) acc += Q[(size_t)c * dimq + i] * u[c];
      qu[i] = acc;
    }
    if (mode == OR_MODE_AB)
      or_back(g, qu, xk);
    else
      memcpy(xk, qu, sizeof(double) * (size_t)n);
    or_forward(g, xk, ax);
    for (long long i = 0; i < m; ++i) ax[i] -= b[i];
    rho[k - 1] = nrm2(ax, m);
    memcpy(x, xk, sizeof(double) * (size_t)n);
    if (o->xtrue && o->rre) {
      double e2 = 0.0, t2 = 0.0;
      for (long long i = 0; i < n; ++i) {
        const double d = xk[i] - o->xtrue[i];
        e2 += d * d;
        t2 += o->xtrue[i] * o->xtrue[i];
      }
      o->rre[k - 1] = sqrt(e2) / sqrt(t2);
    }
    info->k_stop = k;
    info->residual = rho[k - 1];
    info->proj_residual = pres[k - 1];
    if (o->use_dp && rho[k - 1] <= o->tau * o->noise_norm) {
      info->reason = OR_STOP_DP;
      goto done;
    }
    if (o->rns_eps > 0.0 && k >= 2 && fabs(rho[k - 2] - rho[k - 1]) < o->rns_eps * rho[k - 2]) {
      info->reason = OR_STOP_RNS;
      goto done;
    }
    if (!(hk1 > 100.0 * DBL_EPSILON * scale)) {
      info->reason = OR_STOP_BREAKDOWN;
      goto done;
    }
    if (k == K) {
      info->reason = o->use_dp ? OR_STOP_DP_NOT_REACHED : OR_STOP_KMAX;
      goto done;
    }
  }
done:
  if (Hout) memcpy(Hout, H, sizeof(double) * (size_t)(K + 1) * K);
  if (Qout) memcpy(Qout, Q, sizeof(double) * (size_t)dimq * (K + 1));
  free(Q);
  free(H);
  free(w);
  free(tmp);
  free(qu);
  free(xk);
  free(ax);
  free(u);
  free(W);
  free(V);
  free(sig);
  return 0;
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
