"""Seeded generators: determinism and the statistics the workloads ask for."""
import numpy as np
import pytest

from paper_2103_09686_amd import synth


def test_deterministic():
    a = synth.uniform((16, 16), 3)
    b = synth.uniform((16, 16), 3)
    assert np.array_equal(a, b)
    x, _ = synth.boolean_spheres((32, 32), 4, 0.3, seed=1)
    y, _ = synth.boolean_spheres((32, 32), 4, 0.3, seed=1)
    assert np.array_equal(x, y)


def test_boolean_reaches_vf():
    f, vf = synth.boolean_spheres((64, 64), 4, 0.30, seed=0)
    assert f.shape == (1, 64, 64)
    assert 0.30 <= vf < 0.33
    assert set(np.unique(f)) <= {0.0, 1.0}


def test_grf_exact_vf_and_correlation_length():
    f = synth.grf_two_phase((128, 128), 12, 0.40, seed=0)
    assert f.sum() == round(0.40 * f.size)
    g = synth.gaussian_random_field((128, 128), 12, seed=1)
    # covariance of the continuous field at lag l is exp(-1/2) (statistical check)
    c = np.mean(g * np.roll(g, 12, axis=1))
    assert abs(c - np.exp(-0.5)) < 0.15


def test_three_phase_disjoint():
    f, (v1, v2) = synth.spheres_and_ellipsoids((48, 48, 48), 6, 0.20, (10, 4, 4), 0.15, seed=0)
    assert f.shape == (2, 48, 48, 48)
    assert np.all(f[0] * f[1] == 0)
    assert v1 >= 0.20 and v2 >= 0.15
    g, _ = synth.spheres_and_ellipsoids((64, 64), 4, 0.2, (8, 3), 0.15, seed=2)
    assert g.shape == (2, 64, 64) and np.all(g[0] * g[1] == 0)


def test_checkerboard():
    c = synth.checkerboard((8, 8), 2)[0]
    assert c[0, 0] == 1 and c[0, 2] == 0 and c[2, 2] == 1 and c.mean() == 0.5
