"""The allocation-free back projection gkb_back_noalloc (scratch in the
library's fixed device array) against gkb_back, through the C ABI, on two
calls in a row with the second input smaller, plus the oracle's B.

gkb_back_noalloc runs the same kernels as gkb_back, so the outputs must be
equal bit for bit; both are also held to the FP32 (1e-5 relative L2) and FP64
(1e-12) projector bounds against the FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from paper_2606_31153_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2606_31153_amd as gk  # noqa: E402

TOL = {torch.float32: 1e-5, torch.float64: 1e-12}


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _sino(geom, seed):
    return np.random.default_rng(seed).standard_normal(geom.m)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_back_noalloc_matches_back_on_two_calls(dtype):
    dev = torch.device("cuda:0")
    ctx = gk.Context(0)
    # the second geometry needs less scratch than the first, so it reads a
    # region the first call left filled
    geoms = [("fan", synth.fan2d(96, 150, 200)), ("par", synth.par2d(40, 50, 57, ny=33))]
    for idx, (name, geom) in enumerate(geoms):
        note("back_noalloc: call %d %s nx=%d ny=%d views=%d bins=%d dtype=%s" %
             (idx + 1, name, geom.nx, geom.ny, geom.n_views, geom.n_det_u, dtype))
        y = _sino(geom, 700 + idx)
        yd = torch.tensor(y, dtype=dtype, device=dev)
        x_ref = torch.full((geom.n,), float("nan"), dtype=dtype, device=dev)
        x_na = torch.full((geom.n,), float("nan"), dtype=dtype, device=dev)
        gk.gkb_back(ctx, geom, yd, x_ref)
        gk.gkb_back_noalloc(ctx, geom, yd, x_na)
        torch.cuda.synchronize()
        a, b = x_na.cpu().numpy(), x_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        assert np.array_equal(a, b), "max |diff| %.3e" % np.max(np.abs(a - b))
        ref = oracle.Operator(geom).B(y).reshape(-1)
        assert _rel(a, ref) <= TOL[dtype]
    ctx.close()


def test_back_noalloc_rejects_oversized_and_cone_geometry():
    dev = torch.device("cuda:0")
    ctx = gk.Context(0)
    # 4000 views x 2100 bins in FP64 needs about 68 MB of scratch: refused before any launch
    big = synth.par2d(64, 4000, 2100)
    y = torch.zeros(big.m, dtype=torch.float64, device=dev)
    x = torch.zeros(big.n, dtype=torch.float64, device=dev)
    with pytest.raises(gk.GkbError) as ei:
        gk.gkb_back_noalloc(ctx, big, y, x)
    assert ei.value.status == gk.GKB_EINVAL
    cone = synth.cone3d(8, 4, 12, 10)
    yc = torch.zeros(cone.m, dtype=torch.float32, device=dev)
    xc = torch.zeros(cone.n, dtype=torch.float32, device=dev)
    with pytest.raises(gk.GkbError) as ei:
        gk.gkb_back_noalloc(ctx, cone, yc, xc)
    assert ei.value.status == gk.GKB_EUNSUPPORTED
    # the context still works after the refusals
    small = synth.par2d(16, 10, 23)
    ys = torch.tensor(_sino(small, 9), dtype=torch.float64, device=dev)
    xs = torch.zeros(small.n, dtype=torch.float64, device=dev)
    xr = torch.zeros(small.n, dtype=torch.float64, device=dev)
    gk.gkb_back_noalloc(ctx, small, ys, xs)
    gk.gkb_back(ctx, small, ys, xr)
    torch.cuda.synchronize()
    assert torch.equal(xs, xr)
    ctx.close()
