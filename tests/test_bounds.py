"""Host replay of the projector kernels' address arithmetic (gkb_check_geometry,
no GPU): every read inside its zero-padded line, volume or sinogram; every
candidate with a nonzero interpolation weight inside the window the kernel
reads; the dispatch orders of the 2D ray-driven kernels permutations of their
launches.  Run over the geometries the GPU tests use, the batched workload's
slices, and the full-size launch shapes the benchmark times (sampled).

These guard the window and segment index arithmetic of the gather kernels
against later changes, including the fan-beam forward projector's segment
loads, whose first version overflowed its loop test in wavefronts where every
ray misses the image (the 512 fan workload has such wavefronts near the edges
of its fan)."""
import math

import numpy as np
import pytest

import paper_2606_31153_amd as gk
from paper_2606_31153_amd import synth


def cone(nx, ny, nz, nv, nu, nw, du, dw, D, SDD, angles=None):
    return synth.Geometry(kind=synth.KIND_CONE3D, nx=nx, ny=ny, nz=nz, n_views=nv, n_det_u=nu, n_det_v=nw,
                          det_pitch_u=du, det_pitch_v=dw, src_dist=D, src_det_dist=SDD,
                          angle_span=2 * math.pi,
                          angles=None if angles is None else np.asarray(angles, dtype=np.float64))


GEOMS_2D = {
    "par_tiny": synth.par2d(8, 5, 13, angles=np.deg2rad([0.0, 30.0, 45.0, 90.0, 137.0])),
    "par_ragged": synth.par2d(37, 23, 55, ny=29),
    "par64": synth.workload_par64(),
    "par64_v89": synth.par2d(64, 89, 91),
    "par_pitch": synth.par2d(40, 31, 40, det_pitch=1.7),
    "par128_v179": synth.par2d(128, 179),
    "fan_tiny": synth.fan2d(8, 7, 17, src_dist=20.0),
    "fan_ragged": synth.fan2d(45, 33, 70),
    "fan96": synth.fan2d(96, 143, 160),
    "fan128": synth.fan2d(128, 180, 256),
    "fan_far": synth.fan2d(96, 60, 200, src_dist=1000.0),
}

GEOMS_CONE = {
    "cube16": synth.cone3d(16, 12, 24, 20),
    "ragged": cone(20, 17, 11, 13, 31, 23, 1.3, 1.1, 30.0, 55.0),
    "angles": cone(14, 19, 9, 7, 29, 17, 1.2, 1.4, 26.0, 44.0,
                   angles=np.deg2rad([0.0, 17.0, 44.3, 91.0, 180.0, 233.0, 301.7])),
    "flat": cone(24, 24, 1, 10, 40, 3, 1.0, 1.0, 40.0, 80.0),
    "tall": cone(12, 12, 30, 9, 20, 40, 1.5, 1.5, 24.0, 50.0),
    "fine": cone(18, 15, 10, 11, 60, 40, 0.55, 0.6, 28.0, 50.0),
    "coarse": cone(16, 14, 12, 9, 9, 8, 5.0, 6.0, 30.0, 60.0),
    "cube32": synth.cone3d(32, 40, 64, 48),
}


def assert_clean(stats, ok, ops=("A", "B", "At", "Bt")):
    assert ok, "a dispatch order is not a permutation of its launch"
    for op in ops:
        s = stats[op]
        assert s.units > 0 and s.reads > 0, op
        assert s.out_of_bounds == 0, (op, s.out_of_bounds)
        assert s.uncovered == 0, (op, s.uncovered, s.max_uncovered_weight)


@pytest.mark.parametrize("dtype", [gk.GKB_F32, gk.GKB_F64], ids=["f32", "f64"])
@pytest.mark.parametrize("name", list(GEOMS_2D))
def test_2d_geometries_replay_clean(name, dtype):
    stats, ok = gk.gkb_check_geometry(GEOMS_2D[name], dtype, 1)
    assert_clean(stats, ok)


@pytest.mark.parametrize("dtype", [gk.GKB_F32, gk.GKB_F64], ids=["f32", "f64"])
@pytest.mark.parametrize("name", list(GEOMS_CONE))
def test_cone_geometries_replay_clean(name, dtype):
    stats, ok = gk.gkb_check_geometry(GEOMS_CONE[name], dtype, 1)
    assert_clean(stats, ok)


def test_fan_segment_loads_are_replayed():
    # float fan beam with rays under a pixel apart takes the segment path of
    # A: 64 loads per wavefront and line instead of two per ray and line
    g = GEOMS_2D["fan128"]
    s32, _ = gk.gkb_check_geometry(g, gk.GKB_F32, 1)
    s64, _ = gk.gkb_check_geometry(g, gk.GKB_F64, 1)
    assert s32["A"].units == s64["A"].units == g.m
    assert s32["A"].reads != s64["A"].reads


def test_parallel_segment_loads_are_replayed():
    # float parallel beam with a detector pitch near one pixel takes the
    # 128-element segment path of A; a coarse pitch (1.7 pixels: 64 rays span
    # more than 128 elements of a line) keeps the per-ray gathers
    for name, seg in (("par128_v179", True), ("par_pitch", False)):
        g = GEOMS_2D[name]
        s32, _ = gk.gkb_check_geometry(g, gk.GKB_F32, 1)
        s64, _ = gk.gkb_check_geometry(g, gk.GKB_F64, 1)
        assert s32["A"].units == s64["A"].units == g.m
        assert (s32["A"].reads != s64["A"].reads) == seg, name


@pytest.mark.parametrize("name,stride", [("fan512", 31), ("par512", 31)])
def test_full_size_2d_launches_replay_clean(name, stride):
    g = synth.workload_fan512() if name == "fan512" else synth.workload_par512()
    stats, ok = gk.gkb_check_geometry(g, gk.GKB_F32, stride)
    assert_clean(stats, ok)


def test_full_size_cone_launches_replay_clean():
    g = synth.cone3d(512, 720, 1024, 768)
    stats, ok = gk.gkb_check_geometry(g, gk.GKB_F32, 2000003)
    assert_clean(stats, ok)


def test_batched_workload_slices_replay_clean():
    for n, v, nu, seed in synth.batch_slices()[::8]:
        stats, ok = gk.gkb_check_geometry(synth.par2d(n, v), gk.GKB_F32, 17)
        assert_clean(stats, ok)


def test_check_geometry_rejects_bad_arguments():
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_check_geometry(synth.par2d(16, 10), gk.GKB_F32, 0)
    assert e.value.status == gk.GKB_EINVAL
    with pytest.raises(gk.GkbError) as e:
        gk.gkb_check_geometry(synth.par2d(16, 10), 7, 1)
    assert e.value.status == gk.GKB_EINVAL
