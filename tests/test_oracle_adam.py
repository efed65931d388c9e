"""Pins of the oracle's Adam (Kingma & Ba, Alg. 1; the paper's optimizer, Appendix B)
against properties the algorithm's definition fixes: the bias corrections make the
first step, and every step under a constant gradient, exactly lr * g / (|g| + eps);
every step is bounded by lr (1 - beta1) / sqrt(1 - beta2) when 1 - beta1 > sqrt(1 - beta2)
(Kingma & Ba, Sec. 2.1); zero momentum (beta1 = 0) on a constant-magnitude gradient gives
the sign method; projection keeps the box."""
import numpy as np
import pytest


def test_first_and_constant_gradient_steps(ora):
    rng = np.random.default_rng(41)
    g = rng.standard_normal(50) * 1e-3
    x0 = rng.random(50)
    m = v = np.zeros(50)
    x, t = x0.copy(), 0
    want = 1e-3 * g / (np.abs(g) + 1e-7)
    for t in range(1, 30):
        xn, m, v = ora.adam_step(x, g, m, v, t)
        np.testing.assert_allclose(x - xn, want, rtol=1e-9, atol=1e-15)
        x = xn


def test_step_bound(ora):
    rng = np.random.default_rng(42)
    lr, b1, b2 = 1e-3, 0.9, 0.999
    bound = lr * (1 - b1) / np.sqrt(1 - b2)
    x = np.zeros(200)
    m = v = np.zeros(200)
    worst = 0.0
    for t in range(1, 400):
        g = rng.standard_normal(200) * rng.choice([1e-6, 1.0, 1e3], size=200)
        xn, m, v = ora.adam_step(x, g, m, v, t, lr, b1, b2, eps=0.0)
        worst = max(worst, float(np.max(np.abs(xn - x))))
        x = xn
    assert worst <= bound * (1 + 1e-12)


def test_sign_method_and_projection(ora):
    g = np.array([2.0, -3.0, 0.5, -0.25])
    x = np.array([0.5, 0.5, 0.0005, 0.9995])
    m = v = np.zeros(4)
    xn, _, _ = ora.adam_step(x, g, m, v, 1, lr=0.01, beta1=0.0, beta2=0.0, eps=0.0, lo=0.0, hi=1.0)
    np.testing.assert_allclose(xn, [0.49, 0.51, 0.0, 1.0], rtol=0, atol=1e-15)


def test_adam_reconstruction_decreases_error(ora):
    from paper_2103_09686_amd import synth
    spec = ora.Spec(shape=(16, 16), max_disp=(4,))
    tgt, _ = synth.boolean_spheres((16, 16), 2, 0.3, seed=0)
    S_des = ora.descriptor(tgt, spec)
    phi0 = synth.uniform((16, 16), 1)
    E0 = ora.loss(ora.descriptor(phi0, spec), S_des, spec)[0]
    x, E, t = ora.reconstruct_adam(S_des, spec, phi0, 300, lr=1e-2)
    assert t == 300 and E < 0.1 * E0 and x.min() >= 0 and x.max() <= 1
