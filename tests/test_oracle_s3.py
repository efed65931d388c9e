"""Pins of the oracle's three-point correlation S3 (Sec. 3.2.2, eq. s3) and of its
Appendix A map (eq. s3rfroms3rbar).

Independent routes: probability counting on binary fields; the quadratic
reduction of the paper's explicit-mask ensembles (eq. convdef) with the logistic
soft threshold; exact invariants of the product form (symmetry in the two vectors,
the triangle relabelling S3(a, b) = S3(-a, b - a), S3(a, a) = S3(a, 0) = S2(a) on
binary fields); Appendix A giving back the counted S3 on binary fields; the
transpose of the map; central differences of the loss.
"""
import itertools

import numpy as np
import pytest

from test_oracle_pins import paper_convolve, paper_mask


def vec_index(vecs, r):
    return int(np.flatnonzero((vecs == np.array(r)).all(axis=1))[0])


def test_product_s3_probability_counting_3d(ora):
    rng = np.random.default_rng(51)
    f = (rng.random((4, 3, 5)) < 0.45).astype(np.float64)
    vecs = ora.box(3, 1)
    M = len(vecs)
    ia, ib = np.triu_indices(M)
    S = ora._native.s3(f, vecs, ia, ib, 0)
    for k, (a_i, b_i) in enumerate(zip(ia, ib)):
        a, b = vecs[a_i], vecs[b_i]
        hits = 0
        for x in itertools.product(range(4), range(3), range(5)):
            xa = tuple((x[t] + a[t]) % (4, 3, 5)[t] for t in range(3))
            xb = tuple((x[t] + b[t]) % (4, 3, 5)[t] for t in range(3))
            hits += int(f[x] == 1 and f[xa] == 1 and f[xb] == 1)
        assert S[k] == hits / 60.0


def test_soft_s3_is_the_quadratic_reduction_of_mask_ensembles(ora):
    """e_a = f(M * m_a) with the explicit 1-based masks of eq. (convdef), S3 = mean(e_a e_b)."""
    rng = np.random.default_rng(52)
    Mf = rng.random((6, 5))
    alpha = 10.0
    c = ora.soft_threshold_constants(alpha)
    P = Q = 1
    vecs = ora.box(2, 1)
    ia, ib = np.triu_indices(len(vecs))
    S = ora._native.s3(Mf, vecs, ia, ib, 1, alpha, c)
    ens = [ora.soft_threshold(paper_convolve(Mf, paper_mask(P, Q, int(p), int(q)), P, Q), alpha) for (p, q) in vecs]
    for k, (a_i, b_i) in enumerate(zip(ia, ib)):
        assert S[k] == pytest.approx(float(np.mean(ens[a_i] * ens[b_i])), abs=1e-15)


def test_product_s3_invariants(ora):
    rng = np.random.default_rng(53)
    f = rng.random((7, 6))
    vecs = ora.box(2, 2)
    full = {}
    for a_i in range(len(vecs)):
        for b_i in range(len(vecs)):
            full[(a_i, b_i)] = None
    ia, ib = np.meshgrid(np.arange(len(vecs)), np.arange(len(vecs)), indexing="ij")
    ia, ib = ia.ravel(), ib.ravel()
    S = ora._native.s3(f, vecs, ia, ib, 0).reshape(len(vecs), len(vecs))
    np.testing.assert_allclose(S, S.T, rtol=0, atol=1e-15)
    for a_i, a in enumerate(vecs):
        for b_i, b in enumerate(vecs):
            d = b - a
            if np.abs(d).max() <= 2:
                assert S[a_i, b_i] == pytest.approx(S[vec_index(vecs, -a), vec_index(vecs, d)], abs=1e-15)
    fb = (rng.random((7, 6)) < 0.4).astype(np.float64)
    Sb = ora._native.s3(fb, vecs, ia, ib, 0).reshape(len(vecs), len(vecs))
    S2 = ora._native.corr(fb, fb, vecs)
    z = vec_index(vecs, (0, 0))
    np.testing.assert_allclose(np.diag(Sb), S2, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Sb[:, z], S2, rtol=0, atol=1e-15)


def test_appendix_a_s3_map_on_binary(ora):
    """Sbar3 of a binary field mapped back by eq. (s3rfroms3rbar) (with the S2 map
    applied first) equals the counted three-point correlation, 2-D and 3-D."""
    rng = np.random.default_rng(54)
    for shape, P, P3 in [((12, 10), 4, 2), ((6, 6, 6), 2, 1)]:
        lab = rng.integers(0, 3, size=shape)
        phi = np.stack([(lab == 1), (lab == 2)]).astype(np.float64)
        st = ora.Spec(shape=shape, n_channels=2, max_disp=(P,), s3_max_disp=P3, descriptor="stilde")
        ref = ora.Spec(shape=shape, n_channels=2, max_disp=(P,), s3_max_disp=P3)
        np.testing.assert_allclose(ora.descriptor(phi, st), ora.descriptor(phi, ref), rtol=0, atol=1e-13)
        sb = ora.descriptor(phi, ora.Spec(shape=shape, n_channels=2, max_disp=(P,), s3_max_disp=P3,
                                          descriptor="sbar"))
        assert np.max(np.abs(sb - ora.descriptor(phi, ref))) > 1e-3


def test_s3_map_transpose_and_validation(ora):
    rng = np.random.default_rng(55)
    spec = ora.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(4, 3), s3_max_disp=1,
                    descriptor="stilde")
    x, y = rng.standard_normal(spec.K), rng.standard_normal(spec.K)
    lhs = float(np.dot(ora.correct_s3(x, spec), y))
    rhs = float(np.dot(x, ora.correct_s3_adjoint(y, spec)))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # the whole map (two-point map first, then the three-point map) and its transpose
    lhs = float(np.dot(ora.correct_s3(ora.correct_sbar(x, spec), spec), y))
    rhs = float(np.dot(x, ora.correct_sbar_adjoint(ora.correct_s3_adjoint(y, spec), spec)))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    with pytest.raises(ValueError):
        ora.Spec(shape=(16, 16), max_disp=(3,), s3_max_disp=2, descriptor="stilde")
    assert spec.K == sum(e[4] for e in spec.blocks())
    assert [e[0] for e in spec.blocks()] == ["s2", "s2", "s2", "s3", "s3"] * 2


@pytest.mark.parametrize("desc", ["s2", "sbar", "stilde"])
def test_s3_loss_gradient_fd(ora, desc):
    rng = np.random.default_rng(56)
    # the Appendix A map reads S2(r_a - r_b), so S~ needs 2 P3 <= P on every level: one level here
    L, P = (1, (2,)) if desc == "stilde" else (2, (2, 1))
    spec = ora.Spec(shape=(8, 6), n_channels=2, n_levels=L, max_disp=P, s3_max_disp=1, descriptor=desc)
    tgt = (rng.random((2, 8, 6)) < 0.35).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    E0, g0, _ = ora.loss_grad(tgt, S_des, spec)
    assert E0 == 0.0 and np.all(g0 == 0.0)
    phi = rng.random((2, 8, 6))
    E, g, _ = ora.loss_grad(phi, S_des, spec)
    h = 1e-5
    for idx in [(0, 0, 0), (1, 3, 4), (0, 7, 2), (1, 5, 5)]:
        p, m = phi.copy(), phi.copy()
        p[idx] += h
        m[idx] -= h
        fd = (ora.loss_grad(p, S_des, spec)[0] - ora.loss_grad(m, S_des, spec)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-13)


@pytest.mark.parametrize("desc", ["s2", "sbar"])
def test_s3_loss_gradient_fd_3d(ora, desc):
    """Three-point gradient against central differences on a 3-D field with three
    unequal axes, so that every axis of the vectors r_a, r_b, the slowest included,
    enters the adjoint's shifted reads."""
    rng = np.random.default_rng(57)
    sh = (6, 4, 8)
    spec = ora.Spec(shape=sh, n_channels=1, n_levels=1, max_disp=(1,), s3_max_disp=1, descriptor=desc)
    tgt = (rng.random((1,) + sh) < 0.35).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    phi = rng.random((1,) + sh)
    E, g, _ = ora.loss_grad(phi, S_des, spec)
    h = 1e-5
    for idx in [(0, 0, 0, 0), (0, 3, 1, 6), (0, 5, 3, 2), (0, 2, 2, 7)]:
        p, m = phi.copy(), phi.copy()
        p[idx] += h
        m[idx] -= h
        fd = (ora.loss_grad(p, S_des, spec)[0] - ora.loss_grad(m, S_des, spec)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-13)
