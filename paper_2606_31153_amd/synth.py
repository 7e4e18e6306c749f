"""Seeded synthetic inputs shared by the GPU path and the CPU oracle.

This module holds no arithmetic of the reconstruction method itself: it only
draws phantoms, Gaussian noise directions and the geometry descriptors of the
workloads, so that both sides see bit-identical inputs.

* Random-ellipse phantoms (2D) and random-ellipsoid phantoms (3D): densities
  add; each pixel is the mean of 4x4 (4x4x4 in 3D) point samples.  Coordinates
  are normalised so that the image half-width is 1.
* Noise: the paper adds white Gaussian noise at a relative level nu, i.e.
  ||e|| = nu * ||b_true|| (Sec. 5, the SNR values quoted for Examples 1-3 are
  20*log10(1/nu)).  ``noise_direction`` returns the Gaussian vector g;
  ``add_noise`` scales it to e = nu*||b_true||*g/||g||.
* Random numbers come from numpy's Philox4x32-10 counter-based generator keyed
  by (seed, purpose), so every draw is reproducible and independent of order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

PURPOSE_PHANTOM = 0
PURPOSE_NOISE = 1
PURPOSE_BATCH = 2

KIND_PAR2D = 0
KIND_FAN2D = 1
KIND_CONE3D = 2


def rng(seed: int, purpose: int) -> np.random.Generator:
    """Philox4x32-10 stream keyed by (seed, purpose)."""
    key = np.array([int(seed) & 0xFFFFFFFFFFFFFFFF, int(purpose) & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


# --------------------------------------------------------------------------
# geometry descriptors (plain data; each side derives its own tables)
# --------------------------------------------------------------------------
@dataclass
class Geometry:
    """Acquisition geometry.  Pixel pitch is 1; pixel (i, j) has centre
    (i-(nx-1)/2, j-(ny-1)/2) and is stored at x[j, i] (row-major, y grows
    with j).  Sinograms are stored [view][det_v][det_u].

    kind: KIND_PAR2D, KIND_FAN2D or KIND_CONE3D.
    det_pitch_u: detector spacing along u (length for PAR2D/CONE3D, radians
    for the equiangular FAN2D detector).
    angles: explicit view angles (radians) or None for v*angle_span/n_views.
    """

    kind: int
    nx: int
    ny: int
    nz: int = 1
    n_views: int = 1
    n_det_u: int = 1
    n_det_v: int = 1
    det_pitch_u: float = 1.0
    det_pitch_v: float = 1.0
    src_dist: float = 0.0
    src_det_dist: float = 0.0
    angle_span: float = math.pi
    angles: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def m(self) -> int:
        return self.n_views * self.n_det_u * self.n_det_v

    def view_angles(self) -> np.ndarray:
        if self.angles is not None:
            return np.asarray(self.angles, dtype=np.float64)
        return np.arange(self.n_views, dtype=np.float64) * (self.angle_span / self.n_views)

    def image_shape(self):
        return (self.ny, self.nx) if self.nz == 1 and self.kind != KIND_CONE3D else (self.nz, self.ny, self.nx)

    def sino_shape(self):
        if self.kind == KIND_CONE3D:
            return (self.n_views, self.n_det_v, self.n_det_u)
        return (self.n_views, self.n_det_u)


def par2d(n: int, n_views: int, n_det: Optional[int] = None, det_pitch: float = 1.0,
          angles: Optional[Sequence[float]] = None, ny: Optional[int] = None) -> Geometry:
    """2D parallel beam; default detector ceil(n*sqrt(2)) bins covers every
    pixel centre at every angle."""
    if n_det is None:
        n_det = int(math.ceil(n * math.sqrt(2.0)))
    return Geometry(kind=KIND_PAR2D, nx=n, ny=ny if ny is not None else n, n_views=n_views,
                    n_det_u=n_det, det_pitch_u=det_pitch, angle_span=math.pi,
                    angles=None if angles is None else np.asarray(angles, dtype=np.float64))


def fan2d(n: int, n_views: int, n_det: int, src_dist: Optional[float] = None,
          dgamma: Optional[float] = None) -> Geometry:
    """2D fan beam with a curved equiangular detector.  Source at
    src_dist*(cos b, sin b); default src_dist = 2n.  Default bin spacing makes
    the fan just cover the image's circumscribed circle:
    dgamma = 2*asin(R/D)/n_det with R = (n/2)*sqrt(2)."""
    if src_dist is None:
        src_dist = 2.0 * n
    if dgamma is None:
        r = 0.5 * n * math.sqrt(2.0)
        dgamma = 2.0 * math.asin(r / src_dist) / n_det
    return Geometry(kind=KIND_FAN2D, nx=n, ny=n, n_views=n_views, n_det_u=n_det,
                    det_pitch_u=dgamma, src_dist=src_dist, src_det_dist=src_dist,
                    angle_span=2.0 * math.pi)


def cone3d(n: int, n_views: int, n_det_u: int, n_det_v: int, src_dist: Optional[float] = None,
           src_det_dist: Optional[float] = None) -> Geometry:
    """3D cone beam, flat detector.  Default pitches make the volume's
    bounding cylinder project inside the detector."""
    if src_dist is None:
        src_dist = 2.0 * n
    if src_det_dist is None:
        src_det_dist = 2.0 * src_dist
    r = 0.5 * n * math.sqrt(2.0)
    pu = 2.0 * src_det_dist * math.tan(math.asin(r / src_dist)) / n_det_u
    pv = 2.0 * src_det_dist * (0.5 * n) / (src_dist - r) / n_det_v
    return Geometry(kind=KIND_CONE3D, nx=n, ny=n, nz=n, n_views=n_views, n_det_u=n_det_u,
                    n_det_v=n_det_v, det_pitch_u=pu, det_pitch_v=pv, src_dist=src_dist,
                    src_det_dist=src_det_dist, angle_span=2.0 * math.pi)


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
def ellipse_params(seed: int, count: int = 8) -> np.ndarray:
    """Rows (cx, cy, a, b, phi, rho) in normalised coordinates.  Centre at
    radius 0.5*sqrt(U) and uniform angle, semi-axes U[0.1, 0.45], orientation
    U[0, pi), density U[0, 1]; rejected unless |c| + max(a, b) <= 0.95."""
    g = rng(seed, PURPOSE_PHANTOM)
    out = []
    while len(out) < count:
        r = 0.5 * math.sqrt(g.random())
        psi = 2.0 * math.pi * g.random()
        a = 0.1 + 0.35 * g.random()
        b = 0.1 + 0.35 * g.random()
        phi = math.pi * g.random()
        rho = g.random()
        if r + max(a, b) <= 0.95:
            out.append((r * math.cos(psi), r * math.sin(psi), a, b, phi, rho))
    return np.array(out, dtype=np.float64)


def _supersample_axis(n: int, ss: int) -> np.ndarray:
    # normalised sample coordinates, half-width 1; pixel pitch 2/n
    centres = np.arange(n, dtype=np.float64) - (n - 1) / 2.0
    offs = (np.arange(ss, dtype=np.float64) + 0.5) / ss - 0.5
    return ((centres[:, None] + offs[None, :]) * (2.0 / n)).reshape(-1)


def rasterize_ellipses(params: np.ndarray, nx: int, ny: Optional[int] = None, ss: int = 4) -> np.ndarray:
    """Mean of ss x ss point samples per pixel; returns float64 [ny][nx]."""
    ny = nx if ny is None else ny
    half = max(nx, ny) / 2.0
    xs = _supersample_axis(nx, ss) * (nx / 2.0) / half
    ys = _supersample_axis(ny, ss) * (ny / 2.0) / half
    img = np.zeros((ys.size, xs.size))
    for cx, cy, a, b, phi, rho in params:
        c, s = math.cos(phi), math.sin(phi)
        # samples outside the ellipse's bounding box (plus a margin) are outside it
        ex = math.hypot(a * c, b * s) * 1.001 + 1e-9
        ey = math.hypot(a * s, b * c) * 1.001 + 1e-9
        i0, i1 = np.searchsorted(xs, cx - ex), np.searchsorted(xs, cx + ex, side="right")
        j0, j1 = np.searchsorted(ys, cy - ey), np.searchsorted(ys, cy + ey, side="right")
        if i0 >= i1 or j0 >= j1:
            continue
        X, Y = np.meshgrid(xs[i0:i1], ys[j0:j1])
        dx, dy = X - cx, Y - cy
        u = dx * c + dy * s
        v = -dx * s + dy * c
        img[j0:j1, i0:i1] += rho * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img.reshape(ny, ss, nx, ss).mean(axis=(1, 3))


def ellipse_phantom(n: int, seed: int, count: int = 8) -> np.ndarray:
    return rasterize_ellipses(ellipse_params(seed, count), n)


def gaussian_texture(n: int, seed: int) -> np.ndarray:
    """n x n Gaussian random field (float64, row-major): white noise filtered
    by a Gaussian of correlation length ell drawn log-uniformly from [2, 24]
    pixels, standardised, then shifted and scaled to the phantoms' density
    range (mean 0.3, standard deviation 0.15)."""
    g = rng(seed, PURPOSE_PHANTOM)
    ell = math.exp(g.uniform(math.log(2.0), math.log(24.0)))
    w = g.standard_normal((n, n))
    f = np.fft.fftfreq(n)
    f2 = f[:, None] ** 2 + f[None, :] ** 2
    z = np.fft.ifft2(np.fft.fft2(w) * np.exp(-2.0 * math.pi ** 2 * f2 * ell ** 2)).real
    z = (z - z.mean()) / (z.std() + 1e-12)
    return 0.3 + 0.15 * z


def ellipsoid_params(seed: int, count: int = 8) -> np.ndarray:
    """Rows (cx, cy, cz, a, b, c, q0, q1, q2, q3, rho): random centre at
    radius 0.5*U^(1/3) in a uniform direction, semi-axes U[0.1, 0.45],
    orientation from a uniform random unit quaternion, density U[0, 1];
    rejected unless |c| + max(a, b, c) <= 0.95."""
    g = rng(seed, PURPOSE_PHANTOM)
    out = []
    while len(out) < count:
        r = 0.5 * g.random() ** (1.0 / 3.0)
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        a, b, c = 0.1 + 0.35 * g.random(3)
        q = g.standard_normal(4)
        q /= np.linalg.norm(q)
        rho = g.random()
        if r + max(a, b, c) <= 0.95:
            out.append((*(r * d), a, b, c, *q, rho))
    return np.array(out, dtype=np.float64)


def _quat_rot(q) -> np.ndarray:
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def rasterize_ellipsoids(params: np.ndarray, n: int, ss: int = 2, zchunk: int = 8) -> np.ndarray:
    """Mean of ss^3 point samples per voxel; float32 [n][n][n] (z, y, x)."""
    ax = _supersample_axis(n, ss)
    out = np.zeros((n, n, n), dtype=np.float32)
    # per ellipsoid: its axis-aligned bounding box (samples outside it are outside)
    boxes = []
    for row in params:
        R = _quat_rot(row[6:10])
        ext = np.sqrt((R * np.asarray(row[3:6])[None, :]) ** 2 @ np.ones(3)) * 1.001 + 1e-9
        lo = [int(np.searchsorted(ax, row[i] - ext[i])) for i in range(3)]
        hi = [int(np.searchsorted(ax, row[i] + ext[i], side="right")) for i in range(3)]
        boxes.append((R, lo, hi))
    for z0 in range(0, n, zchunk):
        z1 = min(n, z0 + zchunk)
        acc = np.zeros(((z1 - z0) * ss, n * ss, n * ss), dtype=np.float32)
        for row, (R, lo, hi) in zip(params, boxes):
            cx, cy, cz, a, b, c = row[:6]
            rho = row[10]
            k0, k1 = max(lo[2], z0 * ss), min(hi[2], z1 * ss)
            if k0 >= k1 or lo[1] >= hi[1] or lo[0] >= hi[0]:
                continue
            dz = (ax[k0:k1] - cz)[:, None, None]
            dy = (ax[lo[1]:hi[1]] - cy)[None, :, None]
            dx = (ax[lo[0]:hi[0]] - cx)[None, None, :]
            # body coordinates = R^T (p - c)
            u = R[0, 0] * dx + R[1, 0] * dy + R[2, 0] * dz
            v = R[0, 1] * dx + R[1, 1] * dy + R[2, 1] * dz
            w = R[0, 2] * dx + R[1, 2] * dy + R[2, 2] * dz
            acc[k0 - z0 * ss:k1 - z0 * ss, lo[1]:hi[1], lo[0]:hi[0]] += \
                np.float32(rho) * ((u / a) ** 2 + (v / b) ** 2 + (w / c) ** 2 <= 1.0)
        out[z0:z1] = acc.reshape(z1 - z0, ss, n, ss, n, ss).mean(axis=(1, 3, 5))
    return out


# --------------------------------------------------------------------------
# noise
# --------------------------------------------------------------------------
def noise_direction(m: int, seed: int) -> np.ndarray:
    """Standard Gaussian vector g (float64) for the noise of problem `seed`."""
    return rng(seed, PURPOSE_NOISE).standard_normal(m)


def add_noise(b_true: np.ndarray, g: np.ndarray, nu: float):
    """b = b_true + e with e = nu*||b_true||*g/||g||.  Returns (b, ||e||)."""
    bt = np.asarray(b_true, dtype=np.float64).reshape(-1)
    e = (nu * np.linalg.norm(bt) / np.linalg.norm(g)) * np.asarray(g, dtype=np.float64).reshape(-1)
    return (bt + e).reshape(np.shape(b_true)), float(np.linalg.norm(e))


def snr_db(nu: float) -> float:
    """SNR of data with relative noise level nu: 20*log10(||b_true||/||e||)."""
    return 20.0 * math.log10(1.0 / nu)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def workload_par64() -> Geometry:
    """64x64 parallel beam, 90 views over [0, pi), 91 unit bins."""
    return par2d(64, 90, 91)


def workload_fan512() -> Geometry:
    """512x512 fan beam, 720 views over 2*pi, 1024 equiangular bins, D = 1024."""
    return fan2d(512, 720, 1024)


def workload_par512() -> Geometry:
    """512x512 parallel beam, 720 views, 725 unit bins."""
    return par2d(512, 720, 725)


def batch_slices(seed: int = 3000, count: int = 64):
    """Per-slice (n, n_views, nu, phantom_seed) for the batched workload:
    n = 128 + 32*U{0..12}, views = 180 + 30*U{0..18}, nu ~ U[0.5%, 5%]."""
    g = rng(seed, PURPOSE_BATCH)
    out = []
    for i in range(count):
        n = 128 + 32 * int(g.integers(0, 13))
        v = 180 + 30 * int(g.integers(0, 19))
        nu = 0.005 + 0.045 * g.random()
        out.append((n, v, nu, seed + i))
    return out
