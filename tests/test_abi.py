"""The C-ABI library loads on the CPU, exports every symbol include/dmcr.h declares,
and its host-only planning (descriptor size, offsets, validation) agrees with the
oracle's layout.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmcr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmcr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def dm():
    from paper_2103_09686_amd import dmcr
    if not os.path.exists(dmcr.LIB_PATH):
        from paper_2103_09686_amd import build_lib
        build_lib.build(verbose=False)
    dmcr.lib()
    return dmcr


def test_exports_every_declared_symbol(dm):
    names = declared_functions()
    assert len(names) >= 10
    raw = ctypes.CDLL(dm.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_struct_sizes_match_header(dm):
    # dmcr_spec: 4 + 12 + 4 + 4 + 32 + 64 + 4 + 128 + 4 + 4 + 4 (descriptor) + 4 + 8 (alpha)
    assert ctypes.sizeof(dm.c_spec) == 280
    assert dm.c_spec.alpha.offset == 272
    assert ctypes.sizeof(dm.c_result) == 32
    # dmcr_opt: 3 x 4 + pad + 2 x 8 (tol_derr, c1) + method 4 + pad + 4 x 8 (lr, beta1, beta2, eps)
    assert ctypes.sizeof(dm.c_opt) == 72
    assert dm.c_opt.lr.offset == 40


def test_adam_options_validated(dm):
    spec = dm.Spec(shape=(32, 32), max_disp=(4,))
    lb = dm.dmcr_reconstruct_workspace_size(spec, 2, dm.Opt(m=10))
    ad = dm.dmcr_reconstruct_workspace_size(spec, 2, dm.Opt(m=10, method=dm.OPT_ADAM))
    assert ad < lb   # Adam keeps two vectors per element, L-BFGS 2m
    for kw in [dict(lr=0.0), dict(lr=float("nan")), dict(beta1=1.0), dict(beta2=-0.1), dict(eps=0.0)]:
        with pytest.raises(dm.DmcrError):
            dm.dmcr_reconstruct_workspace_size(spec, 1, dm.Opt(method=dm.OPT_ADAM, **kw))
    with pytest.raises(dm.DmcrError):
        dm.dmcr_reconstruct_workspace_size(spec, 1, dm.Opt(method=2))


@pytest.mark.parametrize("shape,C,L,P,pairs", [
    ((64, 64), 1, 1, (16,), ()),
    ((512, 512), 1, 3, (64, 64, 63), ()),
    ((128, 128, 128), 2, 3, (32, 31, 15), ()),
    ((32, 16, 8), 3, 2, (3, 1), ((0, 2), (1, 1))),
])
def test_descriptor_size_and_offsets_match_oracle(dm, ora, shape, C, L, P, pairs):
    spec = dm.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs)
    ospec = ora.Spec(shape=shape, n_channels=C, n_levels=L, max_disp=P, pairs=pairs)
    assert dm.dmcr_descriptor_size(spec) == ospec.K
    offs = dm.dmcr_descriptor_offsets(spec)
    assert offs == [e[2] for e in ospec.layout()] + [ospec.K]


def test_config_sizes_quoted_in_the_workloads(dm):
    """K of the named workloads: 64^2 P=16 -> 545; 512^2 P=64 L=3 -> 24707;
    3-D 128^3 C=2 P=32 L=3 -> 1108929; 3-D 256^3 P=32 -> 137313."""
    assert dm.dmcr_descriptor_size(dm.make_spec((64, 64), 1, 1, 16)) == 545
    assert dm.dmcr_descriptor_size(dm.make_spec((512, 512), 1, 3, 64)) == 24707
    assert dm.dmcr_descriptor_size(dm.make_spec((128, 128, 128), 2, 3, 32)) == 1108929
    assert dm.dmcr_descriptor_size(dm.make_spec((256, 256, 256), 1, 1, 32)) == 137313


@pytest.mark.parametrize("kw,code", [
    (dict(shape=(48, 64)), -3),                       # not a power of two
    (dict(shape=(64, 64), max_disp=(-1,)), -1),        # P < 0
    (dict(shape=(8, 8), n_levels=4, max_disp=(0,)), -1),  # coarsest level below 2
    (dict(shape=(64, 64), n_channels=5), -1),
    (dict(shape=(64, 64), level_weight=(-1.0,)), -1),
    (dict(shape=(64, 64), level_weight=(float("nan"),)), -1),
    (dict(shape=(64, 64), n_levels=9), -1),
    (dict(shape=(64, 64), n_channels=2, pairs=((1, 0),)), -1),
    (dict(shape=(64, 64, 64), max_disp=(20,), path=2), -3),  # DIRECT halo does not fit LDS
    (dict(shape=(64, 64), flags=4), -1),                       # unknown flag bit
    (dict(shape=(2048, 8), max_disp=(3,), path=1), -3),         # FFT axis above 1024
])
def test_validation(dm, kw, code):
    spec = dm.Spec(**kw)
    with pytest.raises(dm.DmcrError) as e:
        dm.dmcr_descriptor_size(spec)
    assert e.value.code == code


def test_workspace_grows_with_batch(dm):
    spec = dm.make_spec((64, 64), 1, 2, 16)
    a = dm.dmcr_workspace_size(spec, 1)
    b = dm.dmcr_workspace_size(spec, 8)
    assert b > a > 0
    r = dm.dmcr_reconstruct_workspace_size(spec, 8, dm.Opt())
    assert r > b


def test_status_strings(dm):
    L = dm.lib()
    for code in (0, -1, -2, -3, -4, -5, 1):
        assert L.dmcr_status_string(code)


def test_soft_descriptor_validation(dm):
    """Soft-threshold descriptors run on the direct path only; S~ needs the auto pairs."""
    base = dict(shape=(64, 64), n_channels=2, max_disp=(8,))
    assert dm.dmcr_descriptor_size(dm.Spec(descriptor=dm.DESC_SBAR, **base)) > 0
    assert dm.dmcr_descriptor_size(dm.Spec(descriptor=dm.DESC_STILDE, **base)) > 0
    bad = [(dict(descriptor=dm.DESC_SBAR, path=dm.PATH_FFT), -3),
           (dict(descriptor=dm.DESC_STILDE, pairs=((0, 1), (1, 1))), -1),
           (dict(descriptor=3), -1),
           (dict(descriptor=dm.DESC_SBAR, alpha=-1.0), -1)]
    for kw, code in bad:
        with pytest.raises(dm.DmcrError) as ei:
            dm.dmcr_descriptor_size(dm.Spec(**kw, **base))
        assert ei.value.code == code


def test_three_point_validation(dm, ora):
    ok = dm.Spec(shape=(64, 64), max_disp=(8,), s3_max_disp=4)
    assert dm.dmcr_descriptor_size(ok) == ora.Spec(shape=(64, 64), max_disp=(8,), s3_max_disp=4).K
    bad = [(dict(shape=(64, 64), max_disp=(12,), s3_max_disp=10), -3),       # more than 361 vectors
           (dict(shape=(32, 32, 32), max_disp=(4,), s3_max_disp=4), -3),
           (dict(shape=(64, 64), max_disp=(5,), s3_max_disp=3, descriptor=2), -1),   # S~3 needs 2 P3 <= P
           (dict(shape=(64, 64), max_disp=(8,), s3_max_disp=-1), -1)]
    for kw, code in bad:
        with pytest.raises(dm.DmcrError) as ei:
            dm.dmcr_descriptor_size(dm.Spec(**kw))
        assert ei.value.code == code, kw


def test_empty_batch_rejected(dm):
    spec = dm.Spec(shape=(64, 64))
    with pytest.raises(dm.DmcrError) as e:
        dm.dmcr_workspace_size(spec, 0)
    assert e.value.code == -1


def test_misaligned_buffers_rejected_before_any_launch(dm):
    """Fields and float64 buffers must be 8-byte aligned: a pointer 4 bytes off is
    rejected with DMCR_EINVAL before anything is launched (host-side check only,
    so fake device addresses are safe here)."""
    spec = dm.Spec(shape=(64, 64), max_disp=(8,))
    s = spec.c()
    K = dm.dmcr_descriptor_size(spec)
    ws_bytes = dm.dmcr_workspace_size(spec, 1)
    L = dm.lib()
    ws = ctypes.c_void_p(1 << 20)                        # 256-byte aligned fake address
    ok, bad = ctypes.c_void_p(1 << 24), ctypes.c_void_p((1 << 24) + 4)
    E = ctypes.c_void_p(1 << 25)
    assert L.dmcr_loss_grad(ctypes.byref(s), 1, bad, ok, E, ok, ws, ws_bytes, None) == -1     # phi
    assert L.dmcr_loss_grad(ctypes.byref(s), 1, ok, bad, E, ok, ws, ws_bytes, None) == -1     # target
    assert L.dmcr_loss_grad(ctypes.byref(s), 1, ok, ok, E, bad, ws, ws_bytes, None) == -1     # grad
    assert L.dmcr_descriptor_forward(ctypes.byref(s), 1, bad, ok, ws, ws_bytes, None) == -1
    assert L.dmcr_descriptor_adjoint(ctypes.byref(s), 1, ok, ok, bad, ws, ws_bytes, None) == -1
    s2 = dm.Spec(shape=(64, 64), n_levels=3, max_disp=(8,)).c()
    assert L.dmcr_pyramid(ctypes.byref(s2), 1, bad, ok, None) == -1
    assert L.dmcr_pyramid(ctypes.byref(s2), 1, ok, bad, None) == -1
    assert K > 0


def test_no_cpu_fallback(dm):
    """The binding computes nothing on the host: host tensors are refused before any
    call, and a missing library is an error, not a slower path."""
    import subprocess
    import sys
    import torch
    spec = dm.Spec(shape=(16, 16), max_disp=(3,))
    with pytest.raises(TypeError):
        dm.dmcr_descriptor_forward(spec, torch.zeros(1, 1, 16, 16))
    with pytest.raises(TypeError):
        dm.dmcr_loss_grad(spec, torch.zeros(1, 1, 16, 16), torch.zeros(1, dm.dmcr_descriptor_size(spec),
                                                                       dtype=torch.float64))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2103_09686_amd import dmcr\n"
            "dmcr.LIB_PATH = '/nonexistent/libdmcr.so'\n"
            "try:\n"
            "    dmcr.dmcr_descriptor_size(dmcr.Spec(shape=(16, 16)))\n"
            "except RuntimeError as e:\n"
            "    print('refused:', e)\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "refused: libdmcr.so is not built" in r.stdout, r.stdout + r.stderr


def test_displacement_clipped_to_the_level(dm, ora):
    """P_l larger than n_l/2 - 1 is clipped per level (a longer displacement aliases):
    the same descriptor as the clipped request."""
    big = dm.Spec(shape=(64, 64), n_levels=3, max_disp=(40, 40, 40))
    clipped = dm.Spec(shape=(64, 64), n_levels=3, max_disp=(31, 15, 7))
    assert dm.dmcr_descriptor_size(big) == dm.dmcr_descriptor_size(clipped) == \
        ora.Spec(shape=(64, 64), n_levels=3, max_disp=(31, 15, 7)).K
    assert dm.dmcr_descriptor_offsets(big) == dm.dmcr_descriptor_offsets(clipped)


def test_level_rule_of_appendix_b(dm, ora):
    """n_levels = 0 selects the paper's level rule (Appendix B: P = 31 gives one, two
    and three levels at 64, 128 and 256), checked through the raw C ABI."""
    L = dm.lib()
    for n, want in ((64, 1), (128, 2), (256, 3), (512, 4)):
        s = dm.Spec(shape=(n, n), n_levels=0, max_disp=(31,)).c()
        assert L.dmcr_level_count(ctypes.byref(s)) == want, n
        ospec = ora.Spec(shape=(n, n), n_levels=want, max_disp=tuple(min(31, (n >> l) // 2 - 1) for l in range(want)))
        assert L.dmcr_descriptor_size(ctypes.byref(s)) == ospec.K
    s = dm.Spec(shape=(32, 32, 32), n_levels=0, max_disp=(16,)).c()   # 32 < 2 (16 + 1): one level
    assert L.dmcr_level_count(ctypes.byref(s)) == 1


@pytest.mark.gpu
def test_default_level_weights_through_the_raw_abi(dm):
    """level_weight 0 selects w_l = 2^{d l / 2} inside the library (eq. mg and its
    footnote): through raw ctypes calls of dmcr_error_cotangent, E and G with zero
    weights equal those with the weights written out, and differ from unit weights."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L = dm.lib()
    for shape, nl in (((64, 64), 3), ((32, 32, 32), 2)):
        d = len(shape)
        K = dm.dmcr_descriptor_size(dm.Spec(shape=shape, n_levels=nl, max_disp=(4,)))
        rng = np.random.default_rng(5)
        S = torch.from_numpy(rng.random((1, K)).astype(np.float32)).cuda()
        St = torch.from_numpy(rng.random((1, K))).cuda()
        out = {}
        for name, w in (("zero", (0.0,) * nl), ("explicit", tuple(2.0 ** (0.5 * d * l) for l in range(nl))),
                        ("unit", (1.0,) * nl)):
            spec = dm.Spec(shape=shape, n_levels=nl, max_disp=(4,), level_weight=w)
            s = spec.c()
            nb = ctypes.c_size_t()
            assert L.dmcr_workspace_size(ctypes.byref(s), 1, ctypes.byref(nb)) == 0
            ws = dm.workspace(nb.value)
            E = torch.empty(1, dtype=torch.float64, device="cuda")
            G = torch.empty_like(S)
            rc = L.dmcr_error_cotangent(ctypes.byref(s), 1, ctypes.c_void_p(S.data_ptr()),
                                        ctypes.c_void_p(St.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                        ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                        ctypes.c_size_t(ws.numel()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert rc == 0
            torch.cuda.synchronize()
            out[name] = (E.item(), G.cpu().numpy())
        assert out["zero"][0] == out["explicit"][0] and np.array_equal(out["zero"][1], out["explicit"][1])
        assert out["zero"][0] != out["unit"][0]
