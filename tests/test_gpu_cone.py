"""GPU parity of the 3D cone-beam projectors and solves (through the C ABI)
against the FP64 CPU oracle.

* The four operators element by element on ragged geometries: FP64 within
  1e-12 relative, FP32 within 1e-5 relative L2 and 1e-4 in max-norm.
* Adjoint identities <A x, y> = <x, A^T y>, <B^T x, y> = <x, B y> and bitwise
  determinism.
* The full 512^3 workload (720 views, 1024 x 768 flat detector): A and B at
  sampled detector pixels / voxels against the oracle's sampled evaluations,
  A^T and B^T through the adjoint identities against the checked A and B.
* AB- and BA-GKB on small cone geometries without rotation symmetry: FP64
  identical stopping iteration and x within 1e-10; FP32 within 1e-4."""
import math
import sys
import zlib

import numpy as np
import pytest

import oracle
from paper_2606_31153_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2606_31153_amd as gk  # noqa: E402

DEV = torch.device("cuda:0")


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = gk.Context(0)
    yield c
    c.close()


def cone(nx, ny, nz, nv, nu, nw, du, dw, D, SDD, angles=None):
    return synth.Geometry(kind=synth.KIND_CONE3D, nx=nx, ny=ny, nz=nz, n_views=nv, n_det_u=nu, n_det_v=nw,
                          det_pitch_u=du, det_pitch_v=dw, src_dist=D, src_det_dist=SDD,
                          angle_span=2 * math.pi,
                          angles=None if angles is None else np.asarray(angles, dtype=np.float64))


GEOMS = {
    "cube16": synth.cone3d(16, 12, 24, 20),
    "ragged": cone(20, 17, 11, 13, 31, 23, 1.3, 1.1, 30.0, 55.0),
    "angles": cone(14, 19, 9, 7, 29, 17, 1.2, 1.4, 26.0, 44.0,
                   angles=np.deg2rad([0.0, 17.0, 44.3, 91.0, 180.0, 233.0, 301.7])),
    "flat": cone(24, 24, 1, 10, 40, 3, 1.0, 1.0, 40.0, 80.0),
    "tall": cone(12, 12, 30, 9, 20, 40, 1.5, 1.5, 24.0, 50.0),
    # fine detector: two-column B^T windows
    "fine": cone(18, 15, 10, 11, 60, 40, 0.55, 0.6, 28.0, 50.0),
    # coarse detector: B^T windows beyond the uniform-window limits (the
    # per-voxel candidate loops)
    "coarse": cone(16, 14, 12, 9, 9, 8, 5.0, 6.0, 30.0, 60.0),
    # the full-size proportions at 32^3
    "cube32": synth.cone3d(32, 40, 64, 48),
}

OPS = {"A": ("gkb_forward", "A", "n"), "B": ("gkb_back", "B", "m"),
       "At": ("gkb_forward_adjoint", "At", "m"), "Bt": ("gkb_back_adjoint", "Bt", "n")}


def run_gpu(ctx, geom, op, inp, dtype):
    n_out = geom.m if op in ("A", "Bt") else geom.n
    xi = torch.tensor(np.asarray(inp).reshape(-1), dtype=dtype, device=DEV)
    xo = torch.full((n_out,), float("nan"), dtype=dtype, device=DEV)
    getattr(gk, OPS[op][0])(ctx, geom, xi, xo)
    torch.cuda.synchronize()
    return xo.cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("gname", list(GEOMS))
@pytest.mark.parametrize("op", list(OPS))
def test_cone_projector_fp64_matches_oracle(ctx, gname, op):
    g = GEOMS[gname]
    r = np.random.default_rng(zlib.crc32((gname + op).encode()))
    inp = r.standard_normal(g.n if OPS[op][2] == "n" else g.m)
    note("cone fp64 %s %s" % (gname, op))
    ref = np.asarray(getattr(oracle.Operator(g), OPS[op][1])(inp)).reshape(-1)
    got = run_gpu(ctx, g, op, inp, torch.float64)
    assert np.all(np.isfinite(got))
    assert rel(got, ref) <= 1e-12
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def smooth_input(g, op, seed):
    # a positive smooth volume (sum of Gaussian blobs) or its projection
    r = np.random.default_rng(seed)
    zz, yy, xx = np.meshgrid(np.arange(g.nz) - (g.nz - 1) / 2, np.arange(g.ny) - (g.ny - 1) / 2,
                             np.arange(g.nx) - (g.nx - 1) / 2, indexing="ij")
    vol = np.zeros((g.nz, g.ny, g.nx))
    for _ in range(5):
        c = r.uniform(-0.3, 0.3, 3) * np.array([g.nz, g.ny, g.nx])
        s = r.uniform(0.15, 0.3) * max(g.nx, g.ny)
        vol += r.uniform(0.5, 1.0) * np.exp(-((zz - c[0]) ** 2 + (yy - c[1]) ** 2 + (xx - c[2]) ** 2) / (2 * s * s))
    if OPS[op][2] == "n":
        return vol
    return oracle.Operator(g).A(vol)


@pytest.mark.parametrize("gname", list(GEOMS))
@pytest.mark.parametrize("op", list(OPS))
def test_cone_projector_fp32_matches_oracle(ctx, gname, op):
    g = GEOMS[gname]
    inp = np.asarray(smooth_input(g, op, 31), dtype=np.float32)
    note("cone fp32 %s %s" % (gname, op))
    ref = np.asarray(getattr(oracle.Operator(g), OPS[op][1])(inp.astype(np.float64))).reshape(-1)
    got = run_gpu(ctx, g, op, inp, torch.float32)
    assert np.all(np.isfinite(got))
    assert rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref))


@pytest.mark.parametrize("gname", ["cube16", "ragged", "tall"])
def test_cone_adjoint_identities_and_determinism(ctx, gname):
    g = GEOMS[gname]
    r = np.random.default_rng(3)
    x = r.standard_normal(g.n)
    y = r.standard_normal(g.m)
    note("cone adjoint %s" % gname)
    for F, Ft in (("A", "At"), ("Bt", "B")):
        Fx = run_gpu(ctx, g, F, x, torch.float64)
        Fty = run_gpu(ctx, g, Ft, y, torch.float64)
        assert abs(Fx @ y - x @ Fty) <= 1e-13 * np.linalg.norm(Fx) * np.linalg.norm(y)
    for op in OPS:
        inp = x if OPS[op][2] == "n" else y
        a = run_gpu(ctx, g, op, inp, torch.float32)
        b = run_gpu(ctx, g, op, inp, torch.float32)
        assert np.array_equal(a, b)


def test_cone_unmatched_pair():
    # B differs from A^T (relative Frobenius distance on a tiny geometry)
    g = synth.cone3d(4, 3, 7, 5)
    op = oracle.Operator(g)
    E = np.eye(g.m)
    At = np.stack([op.At(E[i]).reshape(-1) for i in range(g.m)], axis=1)
    B = np.stack([op.B(E[i]).reshape(-1) for i in range(g.m)], axis=1)
    assert np.linalg.norm(B - At) > 0.05 * np.linalg.norm(At)


def test_cone_full_size_512(ctx):
    """512^3 volume, 720 views, 1024 x 768 detector: A, B, A^T and B^T at
    sampled outputs against the oracle, A^T and B^T also through the adjoint
    identities."""
    g = synth.cone3d(512, 720, 1024, 768)
    note("cone 512: inputs")
    rx = synth.rng(5000, synth.PURPOSE_PHANTOM)
    x = rx.random(g.n, dtype=np.float32)
    y = synth.rng(5000, synth.PURPOSE_NOISE).random(g.m, dtype=np.float32)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    op = oracle.Operator(g)
    pick = np.random.default_rng(7)
    rays = np.sort(pick.choice(g.m, 3000, replace=False))
    voxels = np.sort(pick.choice(g.n, 600, replace=False))
    note("cone 512: A")
    Ax = torch.empty(g.m, dtype=torch.float32, device=DEV)
    gk.gkb_forward(ctx, g, xd, Ax)
    torch.cuda.synchronize()
    ref = op.A_at(x.astype(np.float64), rays)
    got = Ax[torch.from_numpy(rays).to(DEV)].double().cpu().numpy()
    assert rel(got, ref) <= 1e-5
    note("cone 512: B")
    By = torch.empty(g.n, dtype=torch.float32, device=DEV)
    gk.gkb_back(ctx, g, yd, By)
    torch.cuda.synchronize()
    ref = op.B_at(y.astype(np.float64), voxels)
    got = By[torch.from_numpy(voxels).to(DEV)].double().cpu().numpy()
    assert rel(got, ref) <= 1e-5
    del op
    note("cone 512: A^T")
    Aty = torch.empty(g.n, dtype=torch.float32, device=DEV)
    gk.gkb_forward_adjoint(ctx, g, yd, Aty)
    torch.cuda.synchronize()
    lhs = torch.dot(Ax.double(), yd.double()).item()
    rhs = torch.dot(xd.double(), Aty.double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # element by element at six random voxels and six on the faces, edges and
    # corners of the volume (where the candidate windows meet the padding),
    # against the oracle's A^T read one voxel at a time (every ray's weight)
    n1 = g.nx - 1
    edge = [(0, 0, 0), (n1, n1, n1), (0, n1 // 2, 7), (n1, 3, n1 // 2), (n1 // 3, 0, n1), (5, n1, 0)]
    vid = [(l * g.ny + j) * g.nx + i for i, j, l in edge] + list(pick.choice(g.n, 6, replace=False))
    vid = np.asarray(vid, dtype=np.int64)
    note("cone 512: A^T at %d sampled voxels against the oracle" % vid.size)
    ref = oracle.Operator(g).At_at(y.astype(np.float64), vid)
    got = Aty[torch.from_numpy(vid).to(DEV)].double().cpu().numpy()
    note("cone 512: A^T sampled rel %.3e, max abs %.3e of %.3e" % (rel(got, ref), np.max(np.abs(got - ref)),
                                                                   np.max(np.abs(ref))))
    assert rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))
    del Aty
    note("cone 512: B^T")
    Btx = torch.empty(g.m, dtype=torch.float32, device=DEV)
    gk.gkb_back_adjoint(ctx, g, xd, Btx)
    torch.cuda.synchronize()
    lhs = torch.dot(Btx.double(), yd.double()).item()
    rhs = torch.dot(xd.double(), By.double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    note("cone 512: B^T at sampled pixels against the oracle")
    # random pixels, and pixels of large row or column offset that still see
    # the volume (the rows' windows reach farthest in height there)
    pick = np.random.default_rng(9)
    nv, nw, nu = g.n_views, g.n_det_v, g.n_det_u

    def offset(n, lo, hi, count):
        e = pick.integers(lo, hi + 1, count)
        return np.where(pick.random(count) < 0.5, n // 2 - e, n // 2 - 1 + e)

    vv = pick.integers(0, nv, 48)
    rr = np.concatenate([pick.integers(0, nw, 16), offset(nw, 150, 250, 16), pick.integers(nw // 4, 3 * nw // 4, 16)])
    kk = np.concatenate([pick.integers(0, nu, 16), pick.integers(nu // 4, 3 * nu // 4, 16),
                         offset(nu, nu // 2 - 140, nu // 2 - 40, 16)])
    ids = (vv.astype(np.int64) * nw + rr) * nu + kk
    ref = oracle.Operator(g).Bt_at(x.astype(np.float64), ids)
    got = Btx[torch.from_numpy(ids).to(DEV)].double().cpu().numpy()
    note("cone 512: B^T sampled rel %.3e, max abs %.3e of %.3e" % (rel(got, ref), np.max(np.abs(got - ref)),
                                                                   np.max(np.abs(ref))))
    assert rel(got, ref) <= 1e-5
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.max(np.abs(ref))


SOLVE_GEOMS = [cone(14, 13, 9, 23, 25, 17, 1.3, 1.2, 26.0, 50.0),
               cone(16, 16, 12, 19, 27, 21, 1.25, 1.2, 30.0, 60.0)]


def cone_problem(g, seed, nu):
    op = oracle.Operator(g)
    x = smooth_input(g, "A", seed)
    b_true = op.A(x).reshape(-1)
    b, en = synth.add_noise(b_true, synth.noise_direction(b_true.size, seed), nu)
    return op, b, en


@pytest.mark.parametrize("mode", ["ab", "ba"])
@pytest.mark.parametrize("gi", [0, 1])
def test_cone_gkb_fp64_matches_oracle(ctx, mode, gi):
    g = SOLVE_GEOMS[gi]
    op, b, en = cone_problem(g, 800 + gi, 0.01)
    omode = oracle.MODE_AB if mode == "ab" else oracle.MODE_BA
    note("cone gkb fp64 %s %d" % (mode, gi))
    ref = oracle.gkb(op, omode, b, 25, use_dp=True, tau=1.0, noise_norm=en)
    bd = torch.tensor(b, dtype=torch.float64, device=DEV)
    xd = torch.full((g.n,), float("nan"), dtype=torch.float64, device=DEV)
    fn = gk.gkb_ab_solve if mode == "ab" else gk.gkb_ba_solve
    res = fn(ctx, g, bd, xd, 25, use_dp=True, tau=1.0, noise_norm=en)
    torch.cuda.synchronize()
    assert res.k_stop == ref.k_stop and res.reason == ref.reason
    xr = ref.x.reshape(-1)
    assert rel(xd.cpu().numpy(), xr) <= 1e-10
    assert np.allclose(res.rho, ref.rho, rtol=1e-10, atol=0)


@pytest.mark.parametrize("mode", ["ab", "ba"])
def test_cone_gkb_fp32_split(ctx, mode):
    g = SOLVE_GEOMS[1]
    op, b, en = cone_problem(g, 810, 0.01)
    omode = oracle.MODE_AB if mode == "ab" else oracle.MODE_BA
    note("cone gkb fp32 %s" % mode)
    ref = oracle.gkb(op, omode, b.astype(np.float32).astype(np.float64), 12)
    bd = torch.tensor(b, dtype=torch.float32, device=DEV)
    xd = torch.full((g.n,), float("nan"), dtype=torch.float32, device=DEV)
    fn = gk.gkb_ab_solve if mode == "ab" else gk.gkb_ba_solve
    res = fn(ctx, g, bd, xd, 12)
    torch.cuda.synchronize()
    assert res.k_stop == 12 and res.reason == gk.STOP_KMAX
    assert rel(xd.double().cpu().numpy(), ref.x.reshape(-1)) <= 1e-4


@pytest.mark.parametrize("mode", ["ab", "ba"])
def test_cone_rns_stop_and_rre_history(ctx, mode):
    # the stagnation stop (eq. RNS) and the per-iteration reconstruction
    # error (eq. RE) through the cone projectors (AB assembles x_k with the
    # cone B), FP64 against the oracle
    g = SOLVE_GEOMS[0]
    op, b, en = cone_problem(g, 820, 0.01)
    xt = smooth_input(g, "A", 820).reshape(-1)
    omode = oracle.MODE_AB if mode == "ab" else oracle.MODE_BA
    plain = oracle.gkb(op, omode, b, 25)
    ratio = np.abs(np.diff(plain.rho)) / plain.rho[:-1]
    j = next(j for j in range(4, ratio.size) if ratio[:j].min() > 1.21 * ratio[j])
    eps = float(np.sqrt(ratio[j] * min(ratio[:j].min(), 4 * ratio[j])))
    ref = oracle.gkb(op, omode, b, 25, rns_eps=eps, x_true=xt)
    assert (ref.k_stop, ref.reason) == (j + 2, oracle.STOP_RNS)
    note("cone rns/rre %s eps=%.3g k=%d" % (mode, eps, j + 2))
    bd = torch.tensor(b, dtype=torch.float64, device=DEV)
    xd = torch.full((g.n,), float("nan"), dtype=torch.float64, device=DEV)
    xtd = torch.tensor(xt, dtype=torch.float64, device=DEV)
    fn = gk.gkb_ab_solve if mode == "ab" else gk.gkb_ba_solve
    res = fn(ctx, g, bd, xd, 25, rns_eps=eps, x_true=xtd)
    torch.cuda.synchronize()
    assert (res.k_stop, res.reason) == (ref.k_stop, gk.STOP_RNS)
    assert rel(xd.cpu().numpy(), ref.x.reshape(-1)) <= 1e-10
    assert np.allclose(res.rre, ref.rre, rtol=1e-9, atol=0)


def test_cone_invalid(ctx):
    # a detector so tall that rays near its top would step along z
    g = cone(8, 8, 8, 4, 12, 200, 1.0, 1.0, 20.0, 30.0)
    x = torch.zeros(g.n, dtype=torch.float32, device=DEV)
    y = torch.zeros(g.m, dtype=torch.float32, device=DEV)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_forward(ctx, g, x, y)
    assert e.value.status == gk.GKB_EUNSUPPORTED
    # source inside the volume's circumcircle
    g = cone(32, 32, 8, 4, 12, 12, 1.0, 1.0, 20.0, 30.0)
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_forward(ctx, g, torch.zeros(g.n, dtype=torch.float32, device=DEV),
                       torch.zeros(g.m, dtype=torch.float32, device=DEV))
    assert e.value.status == gk.GKB_EINVAL
    # batched solves take 2D slices only
    g = GEOMS["cube16"]
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_batch_solve(ctx, gk.GKB_METHOD_BA, [g], [torch.ones(g.m, dtype=torch.float32, device=DEV)],
                           [torch.zeros(g.n, dtype=torch.float32, device=DEV)], [dict(k_max=3)])
    assert e.value.status == gk.GKB_EUNSUPPORTED
