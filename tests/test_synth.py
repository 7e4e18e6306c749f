"""Seeded input generators (host only): the training textures and the noise
model used for every workload."""
import numpy as np

from paper_2606_31153_amd import synth


def test_gaussian_texture_is_seeded_and_standardised():
    a = synth.gaussian_texture(64, 7)
    assert a.shape == (64, 64)
    assert np.array_equal(a, synth.gaussian_texture(64, 7))
    assert not np.array_equal(a, synth.gaussian_texture(64, 8))
    # white noise filtered, standardised (its divisor carries a 1e-12 guard),
    # then shifted and scaled
    assert abs(a.mean() - 0.3) < 1e-12 and abs(a.std() - 0.15) < 1e-9
    # a correlated field: neighbouring pixels agree far more than independent ones
    d = np.diff(a, axis=1)
    assert d.std() < 0.5 * a.std()


def test_noise_level_is_exact():
    b_true = np.linspace(1.0, 2.0, 1000)
    for nu in (0.005, 0.01, 0.05):
        b, en = synth.add_noise(b_true, synth.noise_direction(b_true.size, 3), nu)
        assert abs(en / np.linalg.norm(b_true) - nu) < 1e-14
        assert abs(np.linalg.norm(b - b_true) - en) < 1e-12
