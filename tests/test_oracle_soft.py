"""Pins of the oracle's soft-threshold descriptor Sbar (Sec. 3.2.4) and of the
Appendix A map back to S2.

Routes independent of the oracle's own sums: the three defining conditions of
the logistic and its tanh special case (footnote), the paper's explicit
convolve - threshold - reduce pipeline with 1-based masks, probability counting
on binary fields (which fixes the Appendix A relation), closed forms (constant
field, single hot voxel), point symmetry, exact adjoint identities and central
finite differences.
"""
import itertools
import json
import os

import numpy as np
import pytest

from test_oracle_pins import paper_convolve, paper_mask

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def _gold():
    return json.load(open(GOLD))


def test_soft_threshold_conditions(ora):
    """f(0) = 0, f(1) = 1, f''(0.75) = 0, f' > 0 on (0, 1), and f -> H(x - 0.75) as alpha grows."""
    g = _gold()
    alpha = g["soft_threshold_alpha"]["value"]
    f = lambda u: ora.soft_threshold(u, alpha)
    assert abs(f(0.0)) < 1e-15 and abs(f(1.0) - 1.0) < 1e-15
    h = 1e-4
    d2 = (f(0.75 + h) - 2 * f(0.75) + f(0.75 - h)) / h ** 2
    d2_scale = (f(0.6 + h) - 2 * f(0.6) + f(0.6 - h)) / h ** 2
    assert abs(d2) < 1e-6 * abs(d2_scale)
    u = np.linspace(0.0, 1.0, 1001)
    assert np.all(np.diff(f(u)) > 0)
    hard = lambda x: ora.soft_threshold(x, 400.0)
    assert hard(0.70) < 1e-8 and hard(0.5) < 1e-20 and hard(0.80) > 1 - 1e-8
    # the values the conditions give at alpha = 10 (f(1/2) enters Appendix A)
    c1, c2, c3 = ora.soft_threshold_constants(alpha)
    assert c2 == -0.75
    assert c1 == pytest.approx(1.0827326, abs=5e-8)
    assert c3 == pytest.approx(-5.98511e-4, abs=5e-10)
    assert f(0.5) == pytest.approx(0.0815356, abs=5e-8)


def test_logistic_form_tanh_special_case(ora):
    """The oracle's threshold is the printed logistic c1/(1+exp(-alpha(x+c2))) + c3: with
    c1 = alpha = 2, c2 = 0, c3 = -1 (footnote to eq. softthreshold) it is tanh."""
    t = _gold()["tanh_special_case"]
    rng = np.random.default_rng(21)
    a, b = rng.random((6, 5)), rng.random((6, 5))
    rs = ora.box(2, 2)
    S = ora._native.sbar(a, b, rs, t["alpha"], (t["c1"], t["c2"], t["c3"]))
    for k, r in enumerate(rs):
        br = np.roll(b, shift=(-int(r[0]), -int(r[1])), axis=(0, 1))   # br[x] = b[x + r]
        assert S[k] == pytest.approx(np.mean(np.tanh(0.5 * (a + br)) ** 2), abs=1e-15)


def test_paper_pipeline_equals_oracle_sbar(ora):
    """Convolve with the explicit masks of eq. (convdef) (1-based), apply the logistic soft
    threshold (alpha = 10), reduce quadratically (eq. s3 with r_a = r_b) == oracle Sbar."""
    rng = np.random.default_rng(22)
    alpha = 10.0
    c = ora.soft_threshold_constants(alpha)
    for shape in [(8, 8), (5, 7)]:
        M = rng.random(shape)
        P, Q = 2, 3
        rs = ora.box(2, 2)
        rs = rs[np.abs(rs[:, 1]) <= Q]
        S_ora = ora._native.sbar(M, M, rs, alpha, c)
        for k, (p, q) in enumerate(rs):
            e = ora.soft_threshold(paper_convolve(M, paper_mask(P, Q, int(p), int(q)), P, Q), alpha)
            assert abs(float(np.sum(e * e) / M.size) - S_ora[k]) < 1e-14


def test_sbar_brute_force_cross_3d(ora):
    """3-D cross pair, every start point, u = (a(x) + b(x + r)) / 2, pure-Python loops."""
    rng = np.random.default_rng(23)
    a, b = rng.random((3, 4, 2)), rng.random((3, 4, 2))
    alpha = 10.0
    c = ora.soft_threshold_constants(alpha)
    rs = ora.box(3, 1)
    S = ora._native.sbar(a, b, rs, alpha, c)
    for k, r in enumerate(rs):
        acc = 0.0
        for x in itertools.product(range(3), range(4), range(2)):
            y = ((x[0] + r[0]) % 3, (x[1] + r[1]) % 4, (x[2] + r[2]) % 2)
            acc += float(ora.soft_threshold(0.5 * (a[x] + b[y]), alpha)) ** 2
        assert S[k] == pytest.approx(acc / 24.0, abs=1e-15)


def test_appendix_a_relation_on_binary_fields(ora):
    """On a binary field the realisation is 1 (both ends in the phase), f(1/2) (one end)
    or 0, so Sbar(r) = (1 - 2F) S(r) + 2F S(0) for r != 0 and Sbar(0) = S(0), F = f(1/2)^2
    (Appendix A); S comes from probability counting.  For two disjoint phases i != j
    the same counting gives Sbar_ij(r) = (1 - 2F) S_ij(r) + F (vf_i + vf_j)."""
    rng = np.random.default_rng(24)
    alpha = 10.0
    c = ora.soft_threshold_constants(alpha)
    F = float(ora.soft_threshold(0.5, alpha)) ** 2
    lab = rng.integers(0, 3, size=(8, 6))
    ph = [(lab == t).astype(np.float64) for t in range(3)]
    rs = ora.box(2, 2)

    def count(a, b, r):
        hits = 0
        for x in itertools.product(range(8), range(6)):
            y = ((x[0] + r[0]) % 8, (x[1] + r[1]) % 6)
            hits += int(a[x] == 1 and b[y] == 1)
        return hits / 48.0

    for i, j in [(1, 1), (2, 2), (1, 2)]:
        Sb = ora._native.sbar(ph[i], ph[j], rs, alpha, c)
        for k, r in enumerate(rs):
            S = count(ph[i], ph[j], r)
            if i == j and not r.any():
                assert Sb[k] == pytest.approx(S, abs=1e-15)
            elif i == j:
                assert Sb[k] == pytest.approx((1 - 2 * F) * S + 2 * F * count(ph[i], ph[i], (0, 0)), abs=1e-15)
            else:
                vf = ph[i].mean() + ph[j].mean()
                assert Sb[k] == pytest.approx((1 - 2 * F) * S + F * vf, abs=1e-15)


def test_stilde_equals_s2_on_binary(ora):
    """The Appendix A map inverts the relation: S~ == S2 on binary fields, every level and
    pair (two channels, two levels, coarse levels are no longer binary so level 2 is
    checked with a block-constant field)."""
    rng = np.random.default_rng(25)
    lab = rng.integers(0, 3, size=(8, 8))
    lab = np.repeat(np.repeat(lab, 2, axis=0), 2, axis=1)       # 16 x 16, constant on 2 x 2 blocks
    phi = np.stack([(lab == 1), (lab == 2)]).astype(np.float64)
    for desc in ("stilde",):
        spec = ora.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(3, 2), descriptor=desc)
        ref = ora.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(3, 2))
        np.testing.assert_allclose(ora.descriptor(phi, spec), ora.descriptor(phi, ref), rtol=0, atol=1e-14)


def test_sbar_closed_forms_and_symmetry(ora):
    alpha = 10.0
    c = ora.soft_threshold_constants(alpha)
    f = lambda u: float(ora.soft_threshold(u, alpha))
    rs = ora.box(2, 2)
    S = ora._native.sbar(np.full((6, 6), 0.37), np.full((6, 6), 0.37), rs, alpha, c)
    np.testing.assert_allclose(S, f(0.37) ** 2, rtol=1e-14)
    hot = np.zeros((6, 6))
    hot[2, 3] = 1.0
    S = ora._native.sbar(hot, hot, rs, alpha, c)
    for k, r in enumerate(rs):
        want = 1.0 / 36 if not r.any() else (2 * f(0.5) ** 2 + 34 * f(0.0) ** 2) / 36
        assert S[k] == pytest.approx(want, abs=1e-16)
    rng = np.random.default_rng(26)
    a, b = rng.random((6, 9)), rng.random((6, 9))
    np.testing.assert_allclose(ora._native.sbar(a, a, rs, alpha, c), ora._native.sbar(a, a, -rs, alpha, c),
                               rtol=0, atol=1e-15)
    np.testing.assert_allclose(ora._native.sbar(a, b, rs, alpha, c), ora._native.sbar(b, a, -rs, alpha, c),
                               rtol=0, atol=1e-15)


def test_correction_adjoint_is_transpose(ora):
    rng = np.random.default_rng(27)
    spec = ora.Spec(shape=(16, 16), n_channels=3, n_levels=2, max_disp=(2, 1), descriptor="stilde")
    x, y = rng.standard_normal(spec.K), rng.standard_normal(spec.K)
    lhs = float(np.dot(ora.correct_sbar(x, spec), y))
    rhs = float(np.dot(x, ora.correct_sbar_adjoint(y, spec)))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    with pytest.raises(ValueError):
        ora.Spec(shape=(16, 16), n_channels=2, pairs=((0, 1),), descriptor="stilde")


@pytest.mark.parametrize("desc", ["sbar", "stilde"])
def test_soft_loss_gradient_fd(ora, desc):
    """dE/dphi for the soft descriptors (two channels, two levels, cross pair) against
    central differences (f is smooth: error O(h^2))."""
    rng = np.random.default_rng(28)
    spec = ora.Spec(shape=(8, 8), n_channels=2, n_levels=2, max_disp=(2, 1), descriptor=desc)
    tgt = (rng.random((2, 8, 8)) < 0.3).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    E0, g0, _ = ora.loss_grad(tgt, S_des, spec)
    assert E0 == 0.0 and np.all(g0 == 0.0)
    phi = rng.random((2, 8, 8))
    E, g, _ = ora.loss_grad(phi, S_des, spec)
    h = 1e-5
    for idx in [(0, 0, 0), (1, 3, 4), (0, 7, 2), (1, 5, 5)]:
        p, m = phi.copy(), phi.copy()
        p[idx] += h
        m[idx] -= h
        fd = (ora.loss_grad(p, S_des, spec)[0] - ora.loss_grad(m, S_des, spec)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-13)


def test_soft_sampled_adjoint_matches_full(ora):
    rng = np.random.default_rng(29)
    spec = ora.Spec(shape=(8, 6, 4), n_channels=2, max_disp=(1,), descriptor="stilde")
    phi = rng.random((2, 8, 6, 4))
    G = rng.standard_normal(spec.K)
    full = ora.adjoint(phi, G, spec)
    vox = np.array([[0, 0, 0], [7, 5, 3], [3, 2, 1]])
    at = ora.adjoint_at_single_level(phi, G, spec, vox)
    for m, v in enumerate(vox):
        np.testing.assert_allclose(at[:, m], full[(slice(None),) + tuple(v)], rtol=1e-13, atol=1e-16)
