"""GPU parity of the paper's soft-threshold descriptor Sbar (Sec. 3.2.4) and of
its Appendix A map S~, on the direct path, against the FP64 oracle.

Tolerances as for S2: per (level, pair) max |dS| <= 1e-5 max |S_oracle|;
||dg||_2 <= 1e-4 ||g_oracle||_2.  The GPU evaluates the logistic in float32
(hardware exp and reciprocal); the oracle in float64 from the same float32 field.
"""
import numpy as np
import pytest

from paper_2103_09686_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S_TOL = 1e-5
G_TOL = 1e-4
KINDS = {"sbar": 1, "stilde": 2}


@pytest.fixture(scope="module")
def dm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_09686_amd import dmcr
    dmcr.lib()
    return dmcr


def to_dev(x, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).cuda()


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def check_S(S_gpu, S_ora, ospec, label=""):
    for (l, pair, off, k) in ospec.layout():
        err = np.max(np.abs(S_gpu[off:off + k] - S_ora[off:off + k]))
        scale = np.max(np.abs(S_ora[off:off + k]))
        assert err <= S_TOL * scale + 1e-30, (label, l, pair, err, scale)


def check_grad(g_gpu, g_ora, label=""):
    num = np.linalg.norm((g_gpu - g_ora).ravel())
    den = np.linalg.norm(g_ora.ravel())
    assert num <= G_TOL * den, (label, num / max(den, 1e-300))


CASES = [
    # shape, C, L, P per level, pairs
    ((64, 64), 1, 1, (31,), ()),
    ((32, 64), 2, 2, (5, 3), ()),
    ((16, 16, 16), 2, 2, (3, 1), ()),
    ((8, 32, 16), 3, 1, (2,), ((0, 0), (1, 1), (2, 2), (0, 2), (1, 2))),
    ((4, 4), 1, 1, (1,), ()),
]


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_soft_forward_adjoint_parity(dm, ora, case, kind):
    shape, C, L, P, pairs = case
    print("soft case", kind, case, flush=True)
    spec = dm.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs, descriptor=KINDS[kind])
    ospec = ora.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs, descriptor=kind)
    B = 2
    phi = f32(np.stack([synth.uniform(shape, 300 + b, channels=C) for b in range(B)]))
    dphi = to_dev(phi)
    S = dm.dmcr_descriptor_forward(spec, dphi).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(8)
    dS = f32(rng.standard_normal((B, ospec.K)))
    g = dm.dmcr_descriptor_adjoint(spec, dphi, to_dev(dS)).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    for b in range(B):
        check_S(S[b], ora.descriptor(phi[b], ospec), ospec, "fwd %s b=%d" % (kind, b))
        check_grad(g[b], ora.adjoint(phi[b], dS[b], ospec), "adj %s b=%d" % (kind, b))


@pytest.mark.parametrize("kind", list(KINDS))
def test_soft_loss_grad_parity(dm, ora, kind):
    shape = (64, 64)
    spec = dm.Spec(shape=shape, n_levels=2, max_disp=(16, 15), descriptor=KINDS[kind])
    ospec = ora.Spec(shape=shape, n_levels=2, max_disp=(16, 15), descriptor=kind)
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=0)
    S_des = ora.descriptor(tgt, ospec)
    phi = f32(synth.uniform(shape, 1))
    E, g = dm.dmcr_loss_grad(spec, to_dev(phi[None]), to_dev(S_des[None], np.float64))
    E = E.cpu().numpy()[0]
    g = g.cpu().numpy()[0].astype(np.float64)
    E_ora, g_ora, _ = ora.loss_grad(phi, S_des, ospec)
    assert abs(E - E_ora) <= 1e-4 * E_ora
    check_grad(g, g_ora, "loss_grad " + kind)


def test_stilde_equals_s2_on_binary_gpu(dm, ora):
    """Appendix A on the GPU: S~ of a binary field equals the S2 of the FFT path."""
    f, vf = synth.boolean_spheres((64, 64), 4, 0.30, seed=0)
    d = to_dev(f[None])
    s2 = dm.dmcr_descriptor_forward(dm.Spec(shape=(64, 64), max_disp=(16,), path=1), d).cpu().numpy()[0]
    st = dm.dmcr_descriptor_forward(dm.Spec(shape=(64, 64), max_disp=(16,), descriptor=2), d).cpu().numpy()[0]
    sb = dm.dmcr_descriptor_forward(dm.Spec(shape=(64, 64), max_disp=(16,), descriptor=1), d).cpu().numpy()[0]
    assert abs(st[0] - vf) <= 1e-6 and abs(sb[0] - vf) <= 1e-6
    assert np.max(np.abs(st - s2)) <= 1e-5 * np.max(np.abs(s2))
    assert np.max(np.abs(sb[1:] - s2[1:])) > 1e-3       # Sbar itself is a different descriptor


def test_sbar_reconstruction_paper_setting(dm, ora):
    """The paper's own setting: Sbar (alpha = 10, uncorrected), 64^2, P = 31, one level,
    Boolean disks r = 4 vf 0.30, U(0,1) start, 100 L-BFGS iterations with projection on
    [0, 1]: the oracle's Sbar of the result confirms the GPU's error, which is within
    five times what SciPy's L-BFGS-B reaches on the oracle's loss in as many iterations
    (the bound-constrained L-BFGS-B handles the many voxels at 0 and 1 better than a
    projected L-BFGS)."""
    shape = (64, 64)
    ospec = ora.Spec(shape=shape, max_disp=(31,), descriptor="sbar")
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=0)
    S_des = ora.descriptor(tgt, ospec)
    phi0 = synth.uniform(shape, 1).astype(np.float32)
    x = torch.from_numpy(phi0[None]).cuda()
    spec = dm.Spec(shape=shape, max_disp=(31,), descriptor=1)
    St = to_dev(S_des[None], np.float64)
    E0 = dm.dmcr_loss_grad(spec, x, St)[0].item()
    code, res = dm.dmcr_reconstruct(spec, St, x, dm.Bounds(0.0, 1.0, dm.BOUNDS_PROJECT),
                                    dm.Opt(max_iter=100, tol_derr=0.0))
    r = res[0]
    print("sbar reconstruction", E0, r, flush=True)
    xf = x.cpu().numpy()[0].astype(np.float64)
    assert xf.min() >= 0.0 and xf.max() <= 1.0
    E_check = ora.loss(ora.descriptor(xf, ospec), S_des, ospec)[0]
    assert abs(E_check - r["final_E"]) <= 1e-3 * E_check + 1e-12
    _, E_ref, _, _ = ora.reconstruct_lbfgsb(S_des, ospec, phi0.astype(np.float64), maxiter=100)
    print("oracle scipy E", E_ref, flush=True)
    assert r["final_E"] <= 5 * E_ref and r["final_E"] < 0.05 * E0
