"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (the workload statement's numbers, applied per result):
  * descriptor: for each (level, pair), max_r |S_gpu - S_oracle| <= 1e-5 max_r |S_oracle|
  * gradient:   ||g_gpu - g_oracle||_2 <= 1e-4 ||g_oracle||_2
Inputs are float32 fields; the oracle evaluates the same float32 values in float64.
"""
import math

import numpy as np
import pytest

from paper_2103_09686_amd import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

S_TOL = 1e-5
G_TOL = 1e-4


@pytest.fixture(scope="module")
def dm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_09686_amd import dmcr
    dmcr.lib()
    return dmcr


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def specs(dm, ora, shape, C, L, P, pairs=(), path=0, flags=0):
    return (dm.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs, path=path, flags=flags),
            ora.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs))


def check_S(S_gpu, S_ora, ospec, label=""):
    for (l, pair, off, k) in ospec.layout():
        a = S_gpu[off:off + k]
        b = S_ora[off:off + k]
        err = np.max(np.abs(a - b))
        scale = np.max(np.abs(b))
        assert err <= S_TOL * scale + 1e-30, (label, l, pair, err, scale)


def check_grad(g_gpu, g_ora, label=""):
    num = np.linalg.norm((g_gpu - g_ora).ravel())
    den = np.linalg.norm(g_ora.ravel())
    assert num <= G_TOL * den, (label, num / max(den, 1e-300))


CASES = [
    # shape, C, L, P per level, pairs, path
    ((64, 64), 1, 1, (16,), (), 2),
    ((64, 64), 1, 1, (16,), (), 1),
    ((32, 64), 2, 2, (5, 3), (), 2),
    ((32, 64), 2, 2, (5, 3), (), 1),
    ((16, 16, 16), 2, 2, (4, 2), (), 2),
    ((16, 16, 16), 2, 2, (4, 2), (), 1),
    ((32, 16, 8), 1, 3, (3, 1, 0), (), 1),
    ((8, 32, 16), 3, 1, (3,), ((0, 2), (1, 1), (1, 2)), 1),
    ((128, 128), 1, 2, (31, 31), (), 1),
    ((2, 2), 1, 1, (0,), (), 1),
    ((4, 4, 4), 1, 2, (1, 0), (), 0),
    # the longest axis the LDS transforms take (1024), on each axis
    ((1024, 16), 1, 1, (7,), (), 1),
    ((16, 1024), 2, 1, (7,), (), 1),
    # the declared maxima: four channels (all ten pairs) and eight levels (down to 2 x 2)
    ((32, 32), 4, 2, (5, 3), (), 1),
    ((16, 8, 8), 4, 1, (2,), (), 2),
    ((256, 256), 1, 8, (7, 7, 7, 7, 7, 3, 1, 0), (), 0),
    # square planes: the contiguous axis and axis 1 in one fused pass (n = 32..256)
    ((8, 32, 32), 2, 1, (3,), (), 1),
    ((4, 64, 64), 1, 2, (1, 0), (), 1),
    ((8, 128, 128), 1, 1, (3,), (), 1),
    ((4, 256, 256), 2, 1, (1,), (), 1),
]


@pytest.mark.parametrize("C", [1, 2])
def test_fused_256_planes_parity(dm, ora, C):
    """256 x 256 planes through the fused one-pass plane transforms (opt-in flag)."""
    shape, P = (4, 256, 256), (1,)
    spec, ospec = specs(dm, ora, shape, C, 1, P, path=1, flags=dm.FLAG_FUSED_PLANES)
    B = 2
    phi = f32(np.stack([synth.uniform(shape, 200 + b, channels=C) for b in range(B)]))
    dphi = to_dev(phi)
    S = dm.dmcr_descriptor_forward(spec, dphi).cpu().numpy().astype(np.float64)
    dS = f32(np.random.default_rng(3).standard_normal((B, ospec.K)))
    g = dm.dmcr_descriptor_adjoint(spec, dphi, to_dev(dS)).cpu().numpy().astype(np.float64)
    for b in range(B):
        check_S(S[b], ora.descriptor(phi[b], ospec), ospec, "fwd b=%d" % b)
        check_grad(g[b], ora.adjoint(phi[b], dS[b], ospec), "adj b=%d" % b)


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_forward_adjoint_parity(dm, ora, case):
    shape, C, L, P, pairs, path = case
    spec, ospec = specs(dm, ora, shape, C, L, P, pairs, path)
    print("case", case, flush=True)
    B = 2
    phi = f32(np.stack([synth.uniform(shape, 100 + b, channels=C) for b in range(B)]))
    dphi = to_dev(phi)
    S = dm.dmcr_descriptor_forward(spec, dphi).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    dS = f32(rng.standard_normal((B, ospec.K)))
    g = dm.dmcr_descriptor_adjoint(spec, dphi, to_dev(dS)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    for b in range(B):
        S_ora = ora.descriptor(phi[b], ospec)
        check_S(S[b], S_ora, ospec, "fwd b=%d" % b)
        g_ora = ora.adjoint(phi[b], dS[b], ospec)
        check_grad(g[b], g_ora, "adj b=%d" % b)


def test_binary_field_volume_fraction_and_paths_agree(dm, ora):
    """Binary field: S_11(0) = volume fraction (Sec. 3.1); FFT and DIRECT agree."""
    f, vf = synth.boolean_spheres((64, 64), 4, 0.30, seed=0)
    d = to_dev(f[None])
    s_fft = dm.dmcr_descriptor_forward(dm.make_spec((64, 64), 1, 1, 16, path=1), d).cpu().numpy()[0]
    s_dir = dm.dmcr_descriptor_forward(dm.make_spec((64, 64), 1, 1, 16, path=2), d).cpu().numpy()[0]
    assert abs(s_fft[0] - vf) <= 1e-6 and abs(s_dir[0] - vf) <= 1e-6
    assert np.max(np.abs(s_fft - s_dir)) <= 1e-6


def test_loss_grad_and_error_parity(dm, ora):
    shape = (64, 64)
    spec, ospec = specs(dm, ora, shape, 1, 2, (16, 15))
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=0)
    S_des = ora.descriptor(tgt, ospec)
    phi = f32(synth.uniform(shape, 1))
    E, g = dm.dmcr_loss_grad(spec, to_dev(phi[None]), torch.from_numpy(S_des[None]).cuda())
    E = E.cpu().numpy()[0]
    g = g.cpu().numpy()[0].astype(np.float64)
    E_ora, g_ora, S_ora = ora.loss_grad(phi, S_des, ospec)
    assert abs(E - E_ora) <= 1e-4 * E_ora
    check_grad(g, g_ora, "loss_grad")
    # error kernel alone on identical S: float64 sum
    S32 = f32(S_ora)
    E2, G2 = dm.dmcr_error_cotangent(spec, to_dev(S32[None]), torch.from_numpy(S_des[None]).cuda())
    E_ref, G_ref = ora.loss(S32, S_des, ospec)
    assert abs(E2.cpu().item() - E_ref) <= 1e-12 * E_ref
    np.testing.assert_allclose(G2.cpu().numpy()[0], G_ref, rtol=1e-6, atol=1e-30)


def test_stationary_at_target(dm, ora):
    """grad E = 0 at the target itself (every residual zero)."""
    shape = (32, 32)
    spec, ospec = specs(dm, ora, shape, 1, 1, (8,))
    tgt, _ = synth.boolean_spheres(shape, 3, 0.3, seed=2)
    d = to_dev(tgt[None])
    S = dm.dmcr_descriptor_forward(spec, d)
    E, g = dm.dmcr_loss_grad(spec, d, S.double())
    assert E.item() == 0.0
    assert torch.count_nonzero(g).item() == 0


def test_pyramid_parity(dm, ora):
    shape = (32, 16, 8)
    spec = dm.Spec(shape=shape, n_channels=2, n_levels=3, max_disp=(1, 1, 0))
    phi = f32(np.stack([synth.uniform(shape, 5, channels=2)]))
    lv = dm.dmcr_pyramid(spec, to_dev(phi))
    ref = ora.pyramid(phi[0], 3)
    for l in (1, 2):
        np.testing.assert_allclose(lv[l - 1].cpu().numpy()[0], ref[l], rtol=2e-7, atol=0)


@pytest.mark.parametrize("shape,L", [((64, 32), 3), ((64, 32), 4), ((16, 32, 8), 3), ((32, 16, 16), 4)])
def test_pyramid_two_levels_per_pass(dm, ora, shape, L):
    """Levels l+1 and l+2 come from level l in one pass when the field is 16-byte
    aligned; a view 8 bytes off takes two one-level passes.  Both must equal each
    other bitwise and the oracle's mean pool."""
    spec = dm.Spec(shape=shape, n_channels=2, n_levels=L, max_disp=(0,))
    B = 2
    phi = f32(np.stack([synth.uniform(shape, 60 + b, channels=2) for b in range(B)]))
    a = to_dev(phi)
    flat = torch.zeros(a.numel() + 2, device="cuda")
    flat[2:] = a.reshape(-1)
    b = flat[2:].view(a.shape)                  # 8-byte aligned, not 16
    assert a.data_ptr() % 16 == 0 and b.data_ptr() % 16 == 8
    la = dm.dmcr_pyramid(spec, a)
    lb = dm.dmcr_pyramid(spec, b)
    for l in range(1, L):
        assert torch.equal(la[l - 1], lb[l - 1]), l
    for i in range(B):
        ref = ora.pyramid(phi[i], L)
        for l in range(1, L):
            np.testing.assert_allclose(la[l - 1].cpu().numpy()[i], ref[l], rtol=2e-7, atol=0)


@pytest.mark.parametrize("shape,C,B,L,P", [((512, 512), 1, 64, 3, 32), ((64, 64, 64), 2, 32, 3, 8),
                                           ((1024, 1024), 1, 16, 1, 16), ((128, 128, 128), 1, 8, 3, 32)],
                         ids=["2d512_b64_3lv", "3d64_c2_b32_3lv", "2d1024_b16_1lv", "3d128_b8_3lv"])
def test_side_lanes_equal_one_stream_bitwise(dm, shape, C, B, L, P):
    """A batch of B C N = 2^24 voxels runs on side lanes, a single field below that
    on one stream.  With three levels, the
    levels are chained by events: the coarser total gradient is prolonged inside
    each level's last inverse pass, and the pyramid takes two restrictions per
    pass.  With one FFT level, the cotangent-kernel pass forms G from S and the
    target itself, and the error reduction runs beside it.  Each field's loss and
    gradient must equal, bitwise, the same field evaluated alone on one stream."""
    spec = dm.make_spec(shape, C, L, P, path=1)
    print("lanes case", shape, C, B, L, flush=True)
    phi = to_dev(np.stack([synth.uniform(shape, 500 + b, channels=C) for b in range(B)]))
    S_t = dm.dmcr_descriptor_forward(spec, (phi * 0.5 + 0.1).contiguous()).double().contiguous()
    E, g = dm.dmcr_loss_grad(spec, phi, S_t)
    for b in (0, B // 2, B - 1):
        E1, g1 = dm.dmcr_loss_grad(spec, phi[b:b + 1].contiguous(), S_t[b:b + 1].contiguous())
        assert torch.equal(E1[0], E[b]) and torch.equal(g1[0], g[b]), b


def test_batched_equals_single_bitwise_and_repeatable(dm):
    shape = (64, 64)
    for path in (1, 2):
        spec = dm.make_spec(shape, 2, 2, 12, path=path)
        phi = to_dev(np.stack([synth.uniform(shape, 40 + b, channels=2) for b in range(4)]))
        S4 = dm.dmcr_descriptor_forward(spec, phi)
        S4b = dm.dmcr_descriptor_forward(spec, phi)
        assert torch.equal(S4, S4b)
        for b in range(4):
            S1 = dm.dmcr_descriptor_forward(spec, phi[b:b + 1].contiguous())
            assert torch.equal(S1[0], S4[b]), (path, b)
        dS = torch.randn_like(S4)
        g4 = dm.dmcr_descriptor_adjoint(spec, phi, dS)
        g1 = dm.dmcr_descriptor_adjoint(spec, phi[1:2].contiguous(), dS[1:2].contiguous())
        assert torch.equal(g1[0], g4[1])


def test_batch_independent_across_exchange_choice(dm, ora):
    """2-D 512^2 (512-point axis-0 pencils), FFT path: a batch of 33 fields has
    enough pencils for the strided passes to take the two-phase exchange, a single
    field does not.  Descriptor, loss and gradient of a field must be bitwise the
    same either way, and the batch must match the oracle."""
    shape = (512, 512)
    spec, ospec = specs(dm, ora, shape, 1, 1, (64,), path=1)
    B = 33
    phi = f32(np.stack([synth.uniform(shape, 700 + b) for b in range(B)]))
    dphi = to_dev(phi)
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=2)
    S_des = ora.descriptor(tgt, ospec)
    St = torch.from_numpy(np.ascontiguousarray(np.repeat(S_des[None], B, axis=0))).cuda()
    S = dm.dmcr_descriptor_forward(spec, dphi)
    E, g = dm.dmcr_loss_grad(spec, dphi, St)
    for b in (0, 17, 32):
        S1 = dm.dmcr_descriptor_forward(spec, dphi[b:b + 1].contiguous())
        E1, g1 = dm.dmcr_loss_grad(spec, dphi[b:b + 1].contiguous(), St[b:b + 1].contiguous())
        assert torch.equal(S1[0], S[b]) and torch.equal(E1[0], E[b]) and torch.equal(g1[0], g[b]), b
    Eo, go, _ = ora.loss_grad(phi[17], S_des, ospec)
    check_S(S[17].cpu().numpy().astype(np.float64), ora.descriptor(phi[17], ospec), ospec, "512 b=17")
    assert abs(E[17].item() - Eo) <= 1e-4 * Eo
    check_grad(g[17].cpu().numpy().astype(np.float64), go, "512 b=17")


def test_autograd_function_fd(dm, ora):
    """Differentiation check on a batch of 64 2-D 256^2 U(0,1) fields: S2Descriptor
    backward against central differences (h = 1e-3, FP64) of the oracle loss at 256
    voxels (4 per field), and against the oracle gradient of four whole fields."""
    shape = (256, 256)
    spec, ospec = specs(dm, ora, shape, 1, 1, (31,))
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=0)
    S_des = ora.descriptor(tgt, ospec)
    B = 64
    phi = f32(np.stack([synth.uniform(shape, s) for s in range(B)]))
    x = to_dev(phi).requires_grad_(True)
    S = dm.s2_descriptor(x, spec)
    Z = float(ospec.K)
    loss = (((S.double() - torch.from_numpy(S_des).cuda()) ** 2).sum(dim=1) / Z).sum()
    loss.backward()
    g = x.grad.cpu().numpy().astype(np.float64)
    for b in (0, 21, 42, 63):
        E, g_ora, _ = ora.loss_grad(phi[b], S_des, ospec)
        check_grad(g[b], g_ora, "autograd b=%d" % b)
    # central differences.  S is quadratic in phi, so a change h at voxel v moves
    # S(r) by exactly (h (phi(v + r) + phi(v - r)) + h^2 [r = 0]) / N (periodic),
    # checked below against a full recomputation; E(phi +- h e_v) then follows from
    # the oracle's loss on S +- that change.
    (_, pair, off, k) = ospec.layout()[0]
    R = ospec.disp(0, pair)
    n0, n1 = shape
    N = float(n0 * n1)
    is0 = np.all(R == 0, axis=1)
    rng = np.random.default_rng(0)
    h = 1e-3

    def dS(f, v, hh):
        a = f[(v[0] + R[:, 0]) % n0, (v[1] + R[:, 1]) % n1] + f[(v[0] - R[:, 0]) % n0, (v[1] - R[:, 1]) % n1]
        return (hh * a + hh * hh * is0) / N

    f0 = phi[0, 0].astype(np.float64)
    S0 = ora.descriptor(phi[0], ospec)
    v = (17, 200)
    p = phi[0].astype(np.float64).copy()
    p[0, v[0], v[1]] += h
    assert np.max(np.abs(ora.descriptor(p, ospec) - (S0 + dS(f0, v, h)))) <= 1e-15
    checked = 0
    for b in range(B):
        fb = phi[b, 0].astype(np.float64)
        Sb = S0 if b == 0 else ora.descriptor(phi[b], ospec)
        # the bound scales with the oracle's own gradient of this field (max over voxels)
        _, g_ref, _ = ora.loss_grad(phi[b], S_des, ospec)
        scale = np.max(np.abs(g_ref))
        for v in rng.integers(0, 256, size=(4, 2)):
            Ep = ora.loss(Sb + dS(fb, v, h), S_des, ospec)[0]
            Em = ora.loss(Sb + dS(fb, v, -h), S_des, ospec)[0]
            fd = (Ep - Em) / (2 * h)
            assert abs(fd - g[b, 0, v[0], v[1]]) <= 1e-4 * scale, (b, tuple(v), fd, g[b, 0, v[0], v[1]])
            checked += 1
    assert checked == 256
