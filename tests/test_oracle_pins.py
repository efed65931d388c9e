"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against a route that does not use its formula:
the paper's own convolve-threshold-reduce pipeline with explicit masks
(Sec. 3.2.3, eq. convdef, 1-based indices exactly as printed), the Appendix A
correction, probability counting on binary fields (Sec. 3.2.1), closed forms,
invariants (point symmetry, sum rule), statistics of noise and of the Boolean
model, exact finite differences of a quadratic map, and the adjoint identity.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2103_09686_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


# ---------------------------------------------------------------------------
# the paper's pipeline, written from Sec. 3.2.3 with explicit masks
# ---------------------------------------------------------------------------
def paper_mask(P, Q, p, q):
    """Mask for r = (p, q): 1/2 at the tail (origin) and at the tip of r, a single 1
    for r = 0 (Sec. 3.2.3 and footnote).  Indexed [r + P, s + Q]."""
    m = np.zeros((2 * P + 1, 2 * Q + 1))
    m[0 + P, 0 + Q] += 0.5
    m[p + P, q + Q] += 0.5
    return m


def paper_convolve(M, m, P, Q):
    """(M * m)_{ij} = sum_{k,l,r,s} M_kl delta^k_{mod_I(i+r)+1} delta^l_{mod_J(j+s)+1} m_rs,
    eq. (convdef) with its 1-based indices i = 1..I, k = 1..I."""
    I, J = M.shape
    out = np.zeros((I, J))
    for i in range(1, I + 1):
        for j in range(1, J + 1):
            acc = 0.0
            for r in range(-P, P + 1):
                for s in range(-Q, Q + 1):
                    w = m[r + P, s + Q]
                    if w == 0.0:
                        continue
                    k = (i + r) % I + 1
                    l = (j + s) % J + 1
                    acc += M[k - 1, l - 1] * w
            out[i - 1, j - 1] = acc
    return out


def paper_S_bar_identity(M, P, Q, p, q):
    """Quadratic reduction of the identity-thresholded ensemble (Sec. 3.2.2, eq. s3 with
    r = p, s = q), i.e. S-bar for f_t(x) = x (Sec. 5.1, Fig. 6)."""
    e = paper_convolve(M, paper_mask(P, Q, p, q), P, Q)
    return float(np.sum(e * e) / M.size)


def appendix_a_correction(S_bar_r, S_bar_0, f_half, r_is_zero):
    """eq. (s2rfroms2rbar)."""
    if r_is_zero:
        return S_bar_r
    return (S_bar_r - 2 * f_half ** 2 * S_bar_0) / (1 - 2 * f_half ** 2)


def test_identity_threshold_pipeline_equals_oracle(ora):
    """Product-form S2 == paper pipeline with f_t(x)=x + Appendix A correction (f(1/2)=1/2)."""
    rng = np.random.default_rng(3)
    for shape in [(8, 8), (5, 7)]:
        M = rng.random(shape)
        P, Q = 2, 3
        rs = ora.box(2, 2)
        rs = rs[np.abs(rs[:, 1]) <= Q]
        S_ora = ora._native.corr(M, M, rs)
        Sb0 = paper_S_bar_identity(M, P, Q, 0, 0)
        for k, (p, q) in enumerate(rs):
            Sb = paper_S_bar_identity(M, P, Q, int(p), int(q))
            S_paper = appendix_a_correction(Sb, Sb0, 0.5, p == 0 and q == 0)
            assert abs(S_paper - S_ora[k]) < 1e-14


def test_hard_threshold_pipeline_equals_oracle_on_binary(ora):
    """Binary field: convolve, hard threshold H(x - 0.75), linear reduction gives the
    exact S2 (Sec. 3.2.3), and S(0) = volume fraction (Sec. 3.1, f~_C(binary) = f_C)."""
    rng = np.random.default_rng(4)
    M = (rng.random((8, 8)) < 0.4).astype(np.float64)
    P = Q = 3
    rs = ora.box(2, 3)
    S_ora = ora._native.corr(M, M, rs)
    for k, (p, q) in enumerate(rs):
        e = paper_convolve(M, paper_mask(P, Q, int(p), int(q)), P, Q)
        e = (e - 0.75 > 0).astype(np.float64)
        assert abs(e.sum() / M.size - S_ora[k]) < 1e-15
    zero = np.flatnonzero((rs == 0).all(axis=1))[0]
    assert S_ora[zero] == pytest.approx(M.mean(), abs=1e-15)


def test_probability_counting_cross_3d(ora):
    """S2^{a->b}(r) on binary 3-D fields = fraction of start points x with x in phase a
    and x + r in phase b (Sec. 3.2.1), counted by brute force."""
    rng = np.random.default_rng(5)
    a = (rng.random((4, 4, 4)) < 0.5).astype(np.float64)
    b = (rng.random((4, 4, 4)) < 0.3).astype(np.float64)
    rs = ora.box(3, 1)
    S = ora._native.corr(a, b, rs)
    for k, r in enumerate(rs):
        hits = 0
        for x in itertools.product(range(4), repeat=3):
            y = tuple((x[t] + r[t]) % 4 for t in range(3))
            hits += int(a[x] == 1 and b[y] == 1)
        assert S[k] == hits / 64.0


def test_symmetry_and_sum_rule(ora):
    rng = np.random.default_rng(6)
    a, b = rng.random((6, 10)), rng.random((6, 10))
    rs = ora.box(2, 2)
    Sab = ora._native.corr(a, b, rs)
    Sba_neg = ora._native.corr(b, a, -rs)
    Saa = ora._native.corr(a, a, rs)
    Saa_neg = ora._native.corr(a, a, -rs)
    np.testing.assert_allclose(Sab, Sba_neg, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Saa, Saa_neg, rtol=0, atol=1e-15)
    # sum over all N displacements = N mu_a mu_b
    allr = np.array([(i, j) for i in range(6) for j in range(10)])
    tot = ora._native.corr(a, b, allr).sum()
    assert tot == pytest.approx(60 * a.mean() * b.mean(), rel=1e-13)


def test_closed_forms(ora):
    rs = ora.box(2, 3)
    c = np.full((8, 8), 0.37)
    np.testing.assert_allclose(ora._native.corr(c, c, rs), 0.37 ** 2, rtol=1e-15)
    hot = np.zeros((8, 8))
    hot[2, 5] = 1.0
    S = ora._native.corr(hot, hot, rs)
    expect = np.where((rs == 0).all(axis=1), 1.0 / 64, 0.0)
    np.testing.assert_array_equal(S, expect)
    cb = synth.checkerboard((8, 8), 1)[0]
    S = ora._native.corr(cb, cb, rs)
    np.testing.assert_array_equal(S, np.where(rs.sum(axis=1) % 2 == 0, 0.5, 0.0))


def test_noise_statistics(ora):
    """U(0,1) i.i.d.: S(0) ~ 1/3 and S(r != 0) - mean^2 within 6 sigma^2/sqrt(N)."""
    f = synth.uniform((64, 64), seed=11)[0]
    rs = ora.half_box(2, 6)
    S = ora._native.corr(f, f, rs)
    N = f.size
    zero = np.flatnonzero((rs == 0).all(axis=1))[0]
    # S(0) = mean(f^2); Var(f^2) = 1/5 - 1/9 for U(0,1)
    assert abs(S[zero] - 1.0 / 3.0) < 6 * math.sqrt(1 / 5.0 - 1 / 9.0) / math.sqrt(N)
    rest = np.delete(S, zero)
    sigma2 = 1.0 / 12.0
    assert np.max(np.abs(rest - f.mean() ** 2)) < 6 * sigma2 / math.sqrt(N)


def test_boolean_model_law(ora):
    """Overlapping disks with n uniform pixel centres: E[S2(r)] =
    1 - 2 (1-|A|/N)^n + (1 - |A u (A+r)|/N)^n (textbook Boolean law, exact for lattice
    centres).  One large realisation must match within a statistical tolerance."""
    shape = (256, 256)
    radius = 4
    f, vf = synth.boolean_spheres(shape, radius, 0.30, seed=0)
    f = f[0]
    offs = [(i, j) for i in range(-radius, radius + 1) for j in range(-radius, radius + 1)
            if i * i + j * j <= radius * radius]
    A = set(offs)
    N = f.size
    # estimate n from the realised coverage: q = (1 - |A|/N)^n
    n = math.log(1 - vf) / math.log(1 - len(A) / N)
    rs = np.array([(0, 0), (0, 1), (1, 1), (0, 3), (2, 3), (0, 6), (5, 5), (0, 12), (9, 9)])
    S = ora._native.corr(f, f, rs)
    for k, r in enumerate(rs):
        union = len(A | {(i + r[0], j + r[1]) for (i, j) in A})
        law = 1 - 2 * (1 - len(A) / N) ** n + (1 - union / N) ** n
        assert abs(S[k] - law) < 0.012, (r, S[k], law)
    assert S[0] == pytest.approx(vf, abs=1e-15)


def test_adjoint_exact_fd_and_dot_product(ora):
    """S is bilinear, so central differences of sum G*S are exact up to rounding;
    and <J v, u> = <v, J^T u> with J v = corr(v_a, b) + corr(a, v_b)."""
    rng = np.random.default_rng(7)
    a, b = rng.random((6, 8)), rng.random((6, 8))
    rs = ora.box(2, 2)
    G = rng.standard_normal(len(rs))
    ga, gb = ora._native.corr_adjoint(a, b, rs, G)
    h = 0.5
    for x in [(0, 0), (3, 5), (5, 7)]:
        ap, am = a.copy(), a.copy()
        ap[x] += h
        am[x] -= h
        fd = (G @ ora._native.corr(ap, b, rs) - G @ ora._native.corr(am, b, rs)) / (2 * h)
        assert fd == pytest.approx(ga[x], abs=1e-14)
        bp, bm = b.copy(), b.copy()
        bp[x] += h
        bm[x] -= h
        fd = (G @ ora._native.corr(a, bp, rs) - G @ ora._native.corr(a, bm, rs)) / (2 * h)
        assert fd == pytest.approx(gb[x], abs=1e-14)
    va, vb = rng.standard_normal(a.shape), rng.standard_normal(b.shape)
    Jv = ora._native.corr(va, b, rs) + ora._native.corr(a, vb, rs)
    assert Jv @ G == pytest.approx(np.sum(va * ga) + np.sum(vb * gb), rel=1e-12)
    # sampled adjoint agrees with the dense one
    vox = np.array([[0, 0], [3, 5], [5, 7]])
    sa, sb = ora._native.corr_adjoint_at(a, b, rs, G, vox)
    np.testing.assert_allclose(sa, ga[tuple(vox.T)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(sb, gb[tuple(vox.T)], rtol=0, atol=1e-15)


def test_half_box_counts_and_order(ora):
    for d in (2, 3):
        for P in (0, 1, 2, 5):
            H = ora.half_box(d, P)
            B = ora.box(d, P)
            assert len(B) == (2 * P + 1) ** d
            assert len(H) == ((2 * P + 1) ** d + 1) // 2
            # H and -H cover B exactly once (apart from r = 0)
            s = {tuple(r) for r in H} | {tuple(-r) for r in H}
            assert s == {tuple(r) for r in B}
            # lexicographic, axis 0 slowest
            assert [tuple(r) for r in B] == sorted(tuple(r) for r in B)


def test_pool_adjoint_and_block_constant(ora):
    rng = np.random.default_rng(8)
    x = rng.random((2, 8, 8, 4))
    y = rng.random((2, 4, 4, 2))
    assert np.sum(ora.pool(x) * y) == pytest.approx(np.sum(x * ora.pool_adjoint(y)), rel=1e-14)
    # a field constant on 2x2 blocks: level-2 S(r) = level-1 S(2r)
    c = rng.random((1, 8, 8))
    f = np.repeat(np.repeat(c, 2, axis=1), 2, axis=2)
    spec = ora.Spec(shape=(16, 16), n_levels=2, max_disp=(6, 3))
    S = ora.descriptor(f, spec)
    lay = spec.layout()
    S1 = S[lay[0][2]:lay[0][2] + lay[0][3]]
    S2 = S[lay[1][2]:lay[1][2] + lay[1][3]]
    H1 = [tuple(r) for r in ora.half_box(2, 6)]
    for k, r in enumerate(ora.half_box(2, 3)):
        assert S2[k] == pytest.approx(S1[H1.index(tuple(2 * r))], abs=1e-15)


def test_paper_level_rule_and_weights(ora):
    """Appendix B: P = 31 gives 1/2/3 levels at 64/128/256 (coarsest side 2(P+1));
    Sec. 3.3: w_l = 2^(l-1) in 2-D."""
    g = json.load(open(GOLD))
    P = g["max_correlation_length"]["P"]
    for n, L in g["levels_for_size_at_P31"].items():
        if n == "cite":
            continue
        n = int(n)
        assert 1 + int(round(math.log2(n / (2 * (P + 1))))) == L
        assert (n >> (L - 1)) == 2 * (P + 1)
    spec = ora.Spec(shape=(256, 256), n_levels=3, max_disp=(31,))
    assert spec.level_weight == (1.0, 2.0, 4.0)
    assert [spec.level_weight[i] for i in range(3)] == [g["level_weight_2d"]["l=%d" % l] for l in (1, 2, 3)]


def test_loss_gradient_fd_and_stationary_target(ora):
    """dE/dphi (two levels, two channels, cross pair) against central differences,
    and dE/dphi = 0 exactly at the target field."""
    rng = np.random.default_rng(9)
    spec = ora.Spec(shape=(8, 8), n_channels=2, n_levels=2, max_disp=(3, 1))
    tgt = (rng.random((2, 8, 8)) < 0.3).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    E0, g0, _ = ora.loss_grad(tgt, S_des, spec)
    assert E0 == 0.0 and np.all(g0 == 0.0)
    phi = rng.random((2, 8, 8))
    E, g, _ = ora.loss_grad(phi, S_des, spec)
    h = 1e-3
    for idx in [(0, 0, 0), (1, 3, 4), (0, 7, 2), (1, 5, 5)]:
        p, m = phi.copy(), phi.copy()
        p[idx] += h
        m[idx] -= h
        fd = (ora.loss_grad(p, S_des, spec)[0] - ora.loss_grad(m, S_des, spec)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("desc", ["s2", "sbar"])
def test_loss_gradient_fd_3d(ora, desc):
    """The same check on a 3-D field with three unequal axes (two levels, two
    channels, auto and cross pairs): every axis, the slowest included, carries
    displacements, so a sign or index slip on any one axis of an adjoint shows."""
    rng = np.random.default_rng(19)
    sh = (8, 12, 10)
    spec = ora.Spec(shape=sh, n_channels=2, n_levels=2, max_disp=(2, 1), descriptor=desc)
    tgt = (rng.random((2,) + sh) < 0.3).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    phi = rng.random((2,) + sh)
    E, g, _ = ora.loss_grad(phi, S_des, spec)
    h = 1e-5
    for idx in [(0, 3, 5, 7), (1, 6, 1, 2), (0, 7, 11, 0), (1, 1, 8, 9)]:
        p, m = phi.copy(), phi.copy()
        p[idx] += h
        m[idx] -= h
        fd = (ora.loss_grad(p, S_des, spec)[0] - ora.loss_grad(m, S_des, spec)[0]) / (2 * h)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-13)


def test_loss_normalisation(ora):
    """E with every residual equal to delta is delta^2 (Z normalisation); G = dE/dS."""
    spec = ora.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(3, 2))
    S = np.linspace(0, 1, spec.K)
    E, G = ora.loss(S + 0.01, S, spec)
    assert E == pytest.approx(1e-4, rel=1e-12)
    w2 = np.concatenate([np.full(k, spec.level_weight[l] ** 2) for (l, _, _, k) in spec.layout()])
    np.testing.assert_allclose(G, 2 * w2 * 0.01 / np.sum(w2), rtol=1e-12)


def test_penalty(ora):
    """E^bc as printed in Sec. 3.1, H(0) = 0: zero (with zero gradient) on [0,1]."""
    phi = np.array([[[-0.5, 0.0, 0.3], [1.0, 1.25, 0.9]]])
    N = 6.0
    E, g = ora.penalty(phi)
    assert E == pytest.approx((0.5 / N) ** 2 + (0.25 / N) ** 2, rel=1e-14)
    assert g[0, 0, 1] == 0.0 and g[0, 1, 0] == 0.0 and g[0, 0, 2] == 0.0
    assert g[0, 0, 0] == pytest.approx(2 * (0.5 / N) * (-1 / N))
    assert g[0, 1, 1] == pytest.approx(2 * (0.25 / N) * (1 / N))


def test_lbfgs_two_loop_equals_dense_bfgs(ora):
    """Two-loop recursion == dense BFGS inverse update from gamma*I (Nocedal & Wright 6.17)."""
    rng = np.random.default_rng(10)
    n, m = 12, 5
    A = rng.standard_normal((n, n))
    A = A @ A.T + n * np.eye(n)
    s_hist = [rng.standard_normal(n) for _ in range(m)]
    y_hist = [A @ s for s in s_hist]
    g = rng.standard_normal(n)
    gamma = (s_hist[-1] @ y_hist[-1]) / (y_hist[-1] @ y_hist[-1])
    H = gamma * np.eye(n)
    for s, y in zip(s_hist, y_hist):
        rho = 1.0 / (y @ s)
        V = np.eye(n) - rho * np.outer(y, s)
        H = V.T @ H @ V + rho * np.outer(s, s)
    np.testing.assert_allclose(ora.lbfgs_direction(g, s_hist, y_hist), -H @ g, rtol=1e-10, atol=1e-12)


def test_projected_lbfgs_first_step_and_armijo(ora):
    """The oracle's projected L-BFGS: its first iteration is the projected steepest
    step x1 = clip(x0 - a g) with a = 2^-k / |g| for the smallest k that passes the
    Armijo test (brute force), every iteration keeps f non-increasing and passes
    Armijo against a fresh evaluation, and the gamma argument of the two-loop
    scales an empty history's direction."""
    rng = np.random.default_rng(62)
    spec = ora.Spec(shape=(8, 8), max_disp=(2,))
    tgt = (rng.random((1, 8, 8)) < 0.4).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    x0 = rng.random((1, 8, 8))
    x1, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, 1)
    E0, g0, _ = ora.loss_grad(x0, S_des, spec)
    a = 1.0 / np.sqrt(np.sum(g0 * g0))
    for k in range(20):
        xt = np.clip(x0 - a * g0, 0.0, 1.0)
        Et = ora.loss(ora.descriptor(xt, spec), S_des, spec)[0]
        if Et <= E0 + 1e-4 * np.sum(g0 * (xt - x0)):
            break
        a *= 0.5
    np.testing.assert_allclose(x1, xt, rtol=0, atol=1e-15)
    assert ev == [k + 1] and Es[0] == pytest.approx(Et, rel=1e-14)
    x, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, 12)
    assert all(b <= a_ for a_, b in zip([E0] + Es[:-1], Es)) and Es[-1] < 0.5 * E0
    assert np.all((x >= 0.0) & (x <= 1.0))
    g = rng.standard_normal(5)
    np.testing.assert_allclose(ora.lbfgs_direction(g, [], [], gamma=0.25), -0.25 * g, rtol=0, atol=0)


def _penalty_as_printed(phi):
    """E^bc of Sec. 3.1 term by term: sum over voxels of
    [ (M - 1) H(M - 1) / (IJ) + (-M) H(-M) / (IJ) ]^2 with H(0) = 0, per channel IJ."""
    N = float(np.prod(phi.shape[1:]))
    tot = 0.0
    for v in np.asarray(phi, np.float64).ravel():
        H_over = 1.0 if v - 1.0 > 0.0 else 0.0
        H_under = 1.0 if -v > 0.0 else 0.0
        t = (v - 1.0) * H_over / N + (-v) * H_under / N
        tot += t * t
    return tot


def test_penalised_loss_fd_inside_outside_and_on_the_box(ora):
    """L = E + lambda E^bc (Sec. 3.1, eq. L_func_dMCR, lambda = kappa E held constant):
    L matches E^bc summed term by term as printed; the gradient equals central
    differences of E(phi) + lambda0 E^bc(phi) (lambda0 of the unperturbed field) at
    voxels inside the box, below 0, above 1 and exactly at 0 and 1, where H(0) = 0
    leaves only dE/dphi; and it differs from the gradient of L with lambda varying."""
    rng = np.random.default_rng(70)
    spec = ora.Spec(shape=(8, 8), n_channels=2, max_disp=(2,))
    tgt = (rng.random((2, 8, 8)) < 0.3).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    phi = rng.uniform(-0.4, 1.4, (2, 8, 8))
    at0, at1 = (0, 1, 1), (1, 2, 3)
    phi[at0], phi[at1] = 0.0, 1.0
    inside, below, above = (0, 5, 5), (1, 0, 7), (0, 6, 2)
    phi[inside], phi[below], phi[above] = 0.55, -0.3, 1.25
    kappa = 40.0
    L, g, E = ora.penalised_loss_grad(phi, S_des, spec, kappa)
    E_only, gE, _ = ora.loss_grad(phi, S_des, spec)
    Ebc = _penalty_as_printed(phi)
    assert E == E_only and Ebc > 0.0
    assert L == pytest.approx(E + kappa * E * Ebc, rel=1e-14)
    lam0 = kappa * E

    def frozen(v):
        return ora.loss_grad(v, S_des, spec)[0] + lam0 * _penalty_as_printed(v)

    def varying(v):
        Ev = ora.loss_grad(v, S_des, spec)[0]
        return Ev + kappa * Ev * _penalty_as_printed(v)

    h = 1e-5
    N = 64.0
    for idx in (inside, below, above, at0, at1):
        p_, m_ = phi.copy(), phi.copy()
        p_[idx] += h
        m_[idx] -= h
        fd = (frozen(p_) - frozen(m_)) / (2 * h)
        # at 0 and 1 the one-sided quadratic of E^bc leaves lam0 h / (2 N^2) in the difference
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=lam0 * h / N ** 2), idx
    assert g[at0] == gE[at0] and g[at1] == gE[at1] and g[inside] == gE[inside]
    assert g[below] < gE[below] and g[above] > gE[above]
    p_, m_ = phi.copy(), phi.copy()
    p_[above] += h
    m_[above] -= h
    fd_var = (varying(p_) - varying(m_)) / (2 * h)
    assert abs(fd_var - g[above]) > 1e-3 * abs(g[above])


def _dense_lbfgs(ora, S_des, spec, x0, iters, c1, max_ls, bounds, kappa=1.0, lo=0.0, hi=1.0, m=10, stats=None):
    """The driver's rules restated with the dense BFGS inverse (Nocedal & Wright
    6.17 from gamma I) instead of the two-loop recursion: the valid pairs among the
    last m iterations since the last reset, gamma = s'y / y'y of the newest, a reset (no pairs, gamma = 1, first
    trial 1/|g|) after a failed search or a non-descent direction; with projection
    the direction is zeroed where it pushes an active bound outward and trials are
    clipped; with the penalty, lambda = kappa E of the search's start point.
    stats, if given, counts the resets for a non-descent direction in stats["nondescent"]."""
    pen = bounds == "penalty"
    clip = (lambda v: v) if pen else (lambda v: np.clip(v, lo, hi))

    def ev(v):
        E, gE, _ = ora.loss_grad(v, S_des, spec)
        if not pen:
            return E, 0.0, gE
        Ebc = _penalty_as_printed(v)
        N = float(np.prod(v.shape[1:]))
        t = np.where(v > hi, (v - hi) / N, 0.0) + np.where(v < lo, (lo - v) / N, 0.0)
        dt = np.where(v > hi, 1.0 / N, 0.0) - np.where(v < lo, 1.0 / N, 0.0)
        return E, Ebc, gE + kappa * E * 2.0 * t * dt

    x = clip(np.asarray(x0, np.float64))
    E, Ebc, g = ev(x)
    f = E + kappa * E * Ebc
    ring, gamma, moved = [], 1.0, False   # one entry per iteration: its pair or None
    out = []
    n = x.size
    for _ in range(iters):
        H = gamma * np.eye(n)
        for s_, y_ in [p_ for p_ in ring if p_ is not None]:
            rho = 1.0 / float(y_ @ s_)
            V = np.eye(n) - rho * np.outer(y_, s_)
            H = V.T @ H @ V + rho * np.outer(s_, s_)

        def proj(d_):
            if not pen:
                d_ = d_.copy()
                d_[((x <= lo) & (d_ < 0)) | ((x >= hi) & (d_ > 0))] = 0.0
            return d_

        d = proj(-(H @ g.ravel()).reshape(x.shape))
        if not np.sum(g * d) < 0:
            ring, gamma, moved = [None] * len(ring), 1.0, False
            d = proj(-g)
            if stats is not None:
                stats["nondescent"] = stats.get("nondescent", 0) + 1
        a = 1.0 if moved else 1.0 / np.sqrt(np.sum(g * g))
        lam = kappa * E
        ok = False
        for _ls in range(max_ls):
            xt = clip(x + a * d)
            Et, Ebct, gt = ev(xt)
            dd = np.sum(g * (xt - x))
            if dd < 0 and Et + lam * Ebct <= f + c1 * dd:
                ok = True
                break
            a /= 2
        pair = None
        if ok:
            s_, y_ = (xt - x).ravel(), (gt - g).ravel()
            if s_ @ y_ > np.finfo(float).eps * (y_ @ y_) and y_ @ y_ > 0:
                pair = (s_, y_)
                gamma = float(s_ @ y_) / float(y_ @ y_)
            x, E, g, f, moved = xt, Et, gt, Et + kappa * Et * Ebct, True
        ring = (ring + [pair])[-m:]
        if not ok:
            ring, gamma, moved = [None] * len(ring), 1.0, False
        out.append((x.copy(), f))
    return out


def test_projected_lbfgs_history_gamma_and_reset(ora):
    """The oracle's projected L-BFGS against the dense restatement over six
    iterations of a case whose fourth line search fails (c1 = 0.3, at most five
    trials): the first three iterations pin the gamma rule and the history order
    (accepted quasi-Newton steps at a = 1), the fourth moves nothing and clears the
    history, the fifth is again a projected steepest step with first trial 1/|g|."""
    rng = np.random.default_rng(67)
    spec = ora.Spec(shape=(8, 8), max_disp=(2,))
    tgt = (rng.random((1, 8, 8)) < 0.4).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    x0 = rng.random((1, 8, 8))
    ref = _dense_lbfgs(ora, S_des, spec, x0, 6, 0.3, 5, "project")
    for it in range(1, 7):
        x, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, it, c1=0.3, max_ls=5)
        np.testing.assert_allclose(x, ref[it - 1][0], rtol=0, atol=1e-12)
        assert Es[-1] == pytest.approx(ref[it - 1][1], rel=1e-10)
    assert ev[3] == 5 and Es[3] == Es[2] and ev[4] < 5 and Es[4] < Es[3]


@pytest.mark.parametrize("seed,m", [(61, 10), (63, 3)])
def test_projected_lbfgs_memory_window_and_nondescent_reset(ora, seed, m):
    """Twelve projected iterations against the dense restatement with a memory of
    m iterations: with m = 3 the oldest pairs leave the window from the fourth
    iteration on; in both runs a projected quasi-Newton direction stops being a
    descent direction (the restatement counts it), which clears the history and
    takes the projected steepest step."""
    rng = np.random.default_rng(seed)
    spec = ora.Spec(shape=(8, 8), max_disp=(2,))
    tgt = (rng.random((1, 8, 8)) < 0.4).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    x0 = rng.random((1, 8, 8))
    stats = {}
    ref = _dense_lbfgs(ora, S_des, spec, x0, 12, 1e-4, 20, "project", m=m, stats=stats)
    assert stats.get("nondescent", 0) >= 1
    x, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, 12, m=m)
    np.testing.assert_allclose(x, ref[-1][0], rtol=0, atol=1e-10)
    np.testing.assert_allclose(Es, [r[1] for r in ref], rtol=1e-9)


def test_penalty_lbfgs_matches_dense_restatement(ora):
    """Penalty mode of the oracle's L-BFGS (no projection; lambda = kappa E of the
    search's start point in the Armijo test, the accepted point's own lambda in f)
    against the dense restatement, from a start with voxels outside [0, 1]."""
    rng = np.random.default_rng(73)
    spec = ora.Spec(shape=(8, 8), max_disp=(2,))
    tgt = (rng.random((1, 8, 8)) < 0.35).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    x0 = rng.uniform(-0.3, 1.3, (1, 8, 8))
    # kappa large enough that the penalty decides a line search (the third iteration
    # backtracks once; with lambda taken at the trial point it would not)
    ref = _dense_lbfgs(ora, S_des, spec, x0, 6, 1e-4, 20, "penalty", kappa=2e4)
    x, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, 6, bounds="penalty", kappa=2e4)
    assert ev == [1, 1, 2, 1, 1, 1]
    np.testing.assert_allclose(x, ref[-1][0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Es, [r[1] for r in ref], rtol=1e-10)
    assert np.any(x < 0.0) or np.any(x > 1.0)


def test_penalty_lbfgs_start_objective_includes_penalty(ora):
    """Penalty mode from a start whose penalty term outweighs the data term
    (kappa E^bc > 1: eight voxels up to 2 above the box, kappa = 1e4).  The first
    trial step is short and leaves E^bc almost unchanged, so the first Armijo test
    passes only against the start's full L = E + lambda E^bc (Sec. 3.1, eq.
    L_func_dMCR); measured against E alone, every trial of that search would fail."""
    rng = np.random.default_rng(70)
    n = 16
    spec = ora.Spec(shape=(n, n), max_disp=(2,))
    tgt = (rng.random((1, n, n)) < 0.35).astype(np.float64)
    S_des = ora.descriptor(tgt, spec)
    x0 = rng.random((1, n, n))
    idx = rng.choice(n * n, 8, replace=False)
    x0.reshape(-1)[idx] = 1.0 + 2.0 * rng.random(8)
    kappa = 1e4
    assert kappa * _penalty_as_printed(x0) > 1.0
    ref = _dense_lbfgs(ora, S_des, spec, x0, 3, 1e-4, 20, "penalty", kappa=kappa)
    x, Es, ev = ora.reconstruct_lbfgs_projected(S_des, spec, x0, 3, bounds="penalty", kappa=kappa)
    assert ev == [1, 1, 1]
    np.testing.assert_allclose(x, ref[-1][0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(Es, [r[1] for r in ref], rtol=1e-10)


def test_level_slices_and_upsampling(ora):
    """The level-l slice of the multigrid descriptor is the single-level descriptor of
    the l-fold pooled field (what the coarse-to-fine stages reconstruct against), and
    nearest-neighbour upsampling is 2^d times the transpose of the mean pool."""
    rng = np.random.default_rng(61)
    spec = ora.Spec(shape=(16, 32), n_channels=2, n_levels=3, max_disp=(3, 2, 1), s3_max_disp=1)
    phi = rng.random((2, 16, 32))
    S = ora.descriptor(phi, spec)
    lv = ora.pyramid(phi, 3)
    for l in range(3):
        np.testing.assert_allclose(S[ora.level_slice(spec, l)], ora.descriptor(lv[l], ora.level_spec(spec, l)),
                                   rtol=0, atol=1e-15)
    g = rng.random((2, 8, 16))
    np.testing.assert_allclose(ora.upsample(g), 4 * ora.pool_adjoint(g), rtol=0, atol=1e-15)
    np.testing.assert_allclose(ora.pool(ora.upsample(g)), g, rtol=0, atol=1e-15)


def test_level_displacement_rule(ora):
    """P_l = min(P, n_l / 2 - 1) (no displacement aliases on a coarse level): the
    workloads' sizes, 512^2 with P = 64 over three levels keeps 64, 64, 63."""
    assert ora.level_disp((512, 512), 3, 64) == (64, 64, 63)
    assert ora.level_disp((128, 128, 128), 3, 32) == (32, 31, 15)
    assert ora.level_disp((64, 32), 2, 31) == (15, 7)
    spec = ora.Spec(shape=(512, 512), n_levels=3, max_disp=ora.level_disp((512, 512), 3, 64))
    assert spec.K == 24707


def test_sampled_descriptor_and_reference_reconstructions(ora):
    """descriptor_at (sampled displacements of one level and pair) equals the matching
    entries of the full descriptor; the SciPy L-BFGS-B reference keeps the box, lowers
    E and lands within a factor of the projected L-BFGS reference on the same loss;
    the sequential coarse-to-fine reference with one level is that same SciPy run, and
    with two levels returns the multigrid E of its own result."""
    rng = np.random.default_rng(72)
    spec = ora.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(3, 2))
    phi = rng.random((2, 16, 16))
    S = ora.descriptor(phi, spec)
    for (l, pair, off, k) in spec.layout():
        r = spec.disp(l, pair)
        sel = rng.choice(len(r), 5, replace=False)
        np.testing.assert_allclose(ora.descriptor_at(phi, spec, l, pair, r[sel]), S[off:off + k][sel], rtol=0,
                                   atol=1e-15)
    one = ora.Spec(shape=(8, 8), max_disp=(2,))
    tgt = (rng.random((1, 8, 8)) < 0.4).astype(np.float64)
    S_des = ora.descriptor(tgt, one)
    x0 = rng.random((1, 8, 8))
    E0 = ora.loss_grad(x0, S_des, one)[0]
    x, E, nit, nev = ora.reconstruct_lbfgsb(S_des, one, x0, maxiter=30)
    assert np.all((x >= 0) & (x <= 1)) and E < 0.1 * E0 and nev >= nit
    assert E == pytest.approx(ora.loss(ora.descriptor(x, one), S_des, one)[0], rel=1e-12)
    _, Es, _ = ora.reconstruct_lbfgs_projected(S_des, one, x0, 30)
    assert E <= 10 * Es[-1] and Es[-1] <= 10 * E
    xc, Ec = ora.reconstruct_coarse_to_fine(S_des, one, x0, maxiter=30)
    np.testing.assert_allclose(xc, x, rtol=0, atol=1e-12)
    two = ora.Spec(shape=(16, 16), n_levels=2, max_disp=(3, 2))
    tg2 = (rng.random((1, 16, 16)) < 0.4).astype(np.float64)
    S2 = ora.descriptor(tg2, two)
    x2, E2 = ora.reconstruct_coarse_to_fine(S2, two, rng.random((1, 16, 16)), maxiter=15)
    assert np.all((x2 >= 0) & (x2 <= 1))
    assert E2 == pytest.approx(ora.loss(ora.descriptor(x2, two), S2, two)[0], rel=1e-12)
    # a start that is constant over each coarsest-level block, against its own
    # descriptor: every level starts at zero error, so each stage hands the field on
    # unchanged, which holds only if the coarse result is repeated over its 2^d
    # children with its values carried over (not scaled)
    three = ora.Spec(shape=(16, 16), n_levels=3, max_disp=(3, 2, 1))
    x0 = np.kron(rng.random((1, 4, 4)), np.ones((1, 4, 4)))
    x3, E3 = ora.reconstruct_coarse_to_fine(ora.descriptor(x0, three), three, x0, maxiter=15)
    np.testing.assert_allclose(x3, x0, rtol=0, atol=1e-15)
    assert E3 == 0.0


def test_oracle_helpers_half_set_pairs_weights_and_Z():
    """The helpers the descriptor layout and the loss rest on, against hand counts:
    the point-symmetry half set, the pair order, the per-entry level weights
    w_l = 2^(d l / 2) (finest level l = 0; Sec. 3.3, eq. mg) and Z = sum_l w_l^2 K_l."""
    import oracle
    assert oracle.in_half((0, 0, 0)) and oracle.in_half((0, 1)) and not oracle.in_half((0, -1))
    assert oracle.in_half((1, -3)) and not oracle.in_half((-1, 5))
    assert oracle.in_half((0, 0, 2)) and not oracle.in_half((0, 0, -2))
    assert oracle.all_pairs(1) == [(0, 0)]
    assert oracle.all_pairs(3) == [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    # 2-D, two levels, two channels (pairs (0,0), (0,1), (1,1)), P = (2, 1): the auto
    # blocks take the half box ((2P+1)^2 + 1) / 2, the cross block the full box
    spec = oracle.Spec(shape=(16, 16), n_channels=2, n_levels=2, max_disp=(2, 1))
    K0, K1 = 2 * 13 + 25, 2 * 5 + 9
    assert spec.K == K0 + K1
    w = oracle.level_weights_per_entry(spec)
    assert np.all(w[:K0] == 1.0) and np.all(w[K0:] == 2.0)
    assert oracle.error_Z(spec) == K0 * 1.0 + K1 * 4.0
    # 3-D: w_1 = 2^(3/2)
    spec3 = oracle.Spec(shape=(8, 8, 8), n_channels=1, n_levels=2, max_disp=(1, 1))
    w3 = oracle.level_weights_per_entry(spec3)
    assert np.allclose(w3[14:], 2.0 ** 1.5) and np.all(w3[:14] == 1.0) and spec3.K == 28
