"""GPU parity of the three-point blocks (eq. s3) and of their Appendix A map against
the FP64 oracle: product form, soft threshold (Sbar3) and S~3, 2-D and 3-D, several
channels and levels, with the two-point blocks on either path.

Tolerances as for S2: per block max |dS| <= 1e-5 max |S_oracle|; ||dg||_2 <= 1e-4 ||g||_2.
"""
import numpy as np
import pytest

from paper_2103_09686_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

S_TOL = 1e-5
G_TOL = 1e-4
KIND = {0: "s2", 1: "sbar", 2: "stilde"}


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


def check_blocks(S_gpu, S_ora, ospec, label):
    for (kind, l, key, off, k) in ospec.blocks():
        err = np.max(np.abs(S_gpu[off:off + k] - S_ora[off:off + k]))
        scale = np.max(np.abs(S_ora[off:off + k]))
        assert err <= S_TOL * scale + 1e-30, (label, kind, l, key, err, scale)


def check_grad(g_gpu, g_ora, label):
    num = np.linalg.norm((g_gpu - g_ora).ravel())
    den = np.linalg.norm(g_ora.ravel())
    assert num <= G_TOL * den, (label, num / max(den, 1e-300))


CASES = [
    # shape, C, L, P, P3, desc, path
    ((32, 32), 1, 1, (6,), 3, 0, 2),
    ((32, 32), 1, 1, (6,), 3, 0, 1),
    ((32, 64), 2, 2, (4, 3), 2, 1, 0),
    ((32, 64), 2, 2, (4, 3), 1, 2, 0),
    ((16, 16, 16), 1, 2, (2, 2), 2, 0, 1),
    ((16, 8, 16), 2, 1, (2,), 1, 1, 0),
    ((16, 8, 16), 2, 1, (2,), 1, 2, 0),
    ((8, 8), 1, 2, (2, 1), 1, 1, 0),
    # 169 and 343 vectors: Gram tiles beyond one 96 x 96 super-tile
    ((64, 64), 1, 1, (12,), 6, 0, 0),
    ((64, 64), 2, 1, (12,), 6, 1, 0),
    ((64, 64), 1, 1, (12,), 6, 2, 0),
    ((16, 16, 16), 1, 1, (3,), 3, 0, 1),
    # M = 16 n + 1 (49, 81, 289 vectors): the last vector's Gram column and
    # cotangent column summed beside the 16-wide tiles; 289 spans three bands
    ((64, 64), 1, 1, (8,), 4, 0, 1),
    ((64, 64), 2, 2, (8, 4), 4, 1, 0),
    ((32, 32), 2, 1, (6,), 3, 2, 0),
    ((64, 64), 1, 1, (12,), 8, 0, 0),
    ((64, 64), 1, 1, (12,), 8, 1, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[str(i) for i in range(len(CASES))])
def test_s3_forward_adjoint_parity(dm, ora, case):
    shape, C, L, P, P3, desc, path = case
    print("s3 case", case, flush=True)
    spec = dm.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, s3_max_disp=P3, descriptor=desc, path=path)
    ospec = ora.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, s3_max_disp=P3, descriptor=KIND[desc])
    B = 2
    phi = f32(np.stack([synth.uniform(shape, 500 + b, channels=C) for b in range(B)]))
    dphi = to_dev(phi)
    S = dm.dmcr_descriptor_forward(spec, dphi).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(9)
    dS = f32(rng.standard_normal((B, ospec.K)))
    g = dm.dmcr_descriptor_adjoint(spec, dphi, to_dev(dS)).cpu().numpy().astype(np.float64)
    # a field's result does not depend on the batch it is evaluated in
    S1 = dm.dmcr_descriptor_forward(spec, dphi[1:2].contiguous()).cpu().numpy().astype(np.float64)
    g1 = dm.dmcr_descriptor_adjoint(spec, dphi[1:2].contiguous(), to_dev(dS[1:2])).cpu().numpy().astype(np.float64)
    assert np.array_equal(S1[0], S[1]) and np.array_equal(g1[0], g[1])
    for b in range(B):
        check_blocks(S[b], ora.descriptor(phi[b], ospec), ospec, "fwd b=%d" % b)
        check_grad(g[b], ora.adjoint(phi[b], dS[b], ospec), "adj b=%d" % b)


def test_s3_loss_grad_and_binary_map(dm, ora):
    """loss/gradient with S~3 against the oracle, and S~ of a binary field equals the
    product-form descriptor (two- and three-point blocks) on the GPU."""
    shape = (64, 64)
    spec = dm.Spec(shape=shape, max_disp=(8,), s3_max_disp=3, descriptor=2)
    ospec = ora.Spec(shape=shape, max_disp=(8,), s3_max_disp=3, descriptor="stilde")
    tgt, _ = synth.boolean_spheres(shape, 4, 0.30, seed=0)
    S_des = ora.descriptor(tgt, ospec)
    phi = f32(synth.uniform(shape, 1))
    E, g = dm.dmcr_loss_grad(spec, to_dev(phi[None]), to_dev(S_des[None], np.float64))
    E_ora, g_ora, _ = ora.loss_grad(phi, S_des, ospec)
    assert abs(E.item() - E_ora) <= 1e-4 * E_ora
    check_grad(g.cpu().numpy()[0].astype(np.float64), g_ora, "loss_grad")
    st = dm.dmcr_descriptor_forward(spec, to_dev(tgt[None])).cpu().numpy()[0]
    pr = dm.dmcr_descriptor_forward(dm.Spec(shape=shape, max_disp=(8,), s3_max_disp=3), to_dev(tgt[None]))
    pr = pr.cpu().numpy()[0]
    assert np.max(np.abs(st - pr)) <= 1e-5 * np.max(np.abs(pr))


def test_s3_forward_256(dm, ora):
    """2-D 256^2, P3 = 4 (81 vectors, 3321 pairs), product form: every entry against
    the oracle."""
    shape = (256, 256)
    spec = dm.Spec(shape=shape, max_disp=(8,), s3_max_disp=4)
    ospec = ora.Spec(shape=shape, max_disp=(8,), s3_max_disp=4)
    phi = f32(synth.uniform(shape, 3))
    S = dm.dmcr_descriptor_forward(spec, to_dev(phi[None])).cpu().numpy()[0].astype(np.float64)
    check_blocks(S, ora.descriptor(phi, ospec), ospec, "256")
