"""dmcr_loss_grad_noalloc (scratch in the library's static device array) against
dmcr_loss_grad (caller workspace), through raw ctypes calls of the C ABI: two
calls in a row, the second with a smaller input, each equal to the workspace
entry point's result within the parity bar (E to 1e-12 relative, the gradient to
1e-4 in norm; the kernels are the same, so the results are expected bitwise
equal), and a problem whose workspace exceeds the array is refused with
DMCR_ENOMEM before any launch."""
import ctypes

import numpy as np
import pytest

from paper_2103_09686_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_09686_amd import dmcr
    L = dmcr.lib()
    L.dmcr_loss_grad_noalloc.argtypes = [ctypes.POINTER(dmcr.c_spec), ctypes.c_int32] + [ctypes.c_void_p] * 5
    L.dmcr_loss_grad_noalloc.restype = ctypes.c_int
    return dmcr


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def run_both(dm, spec, B, seed):
    L = dm.lib()
    shape = spec.shape
    C = spec.n_channels
    phi = torch.from_numpy(synth.uniform(shape, seed, channels=B * C).reshape((B, C) + shape).astype(np.float32)).cuda()
    K = dm.dmcr_descriptor_size(spec)
    St = torch.from_numpy(np.random.default_rng(seed).random((B, K)) * 0.3).cuda()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    s = spec.c()
    # the workspace entry point
    nb = ctypes.c_size_t()
    assert L.dmcr_workspace_size(ctypes.byref(s), B, ctypes.byref(nb)) == 0
    ws = dm.workspace(nb.value)
    E_ws = torch.empty(B, dtype=torch.float64, device="cuda")
    g_ws = torch.empty_like(phi)
    assert L.dmcr_loss_grad(ctypes.byref(s), B, _vp(phi), _vp(St), _vp(E_ws), _vp(g_ws), _vp(ws),
                            ctypes.c_size_t(ws.numel()), stream) == 0
    # the static-scratch entry point
    E_na = torch.full((B,), float("nan"), dtype=torch.float64, device="cuda")
    g_na = torch.full_like(phi, float("nan"))
    rc = L.dmcr_loss_grad_noalloc(ctypes.byref(s), B, _vp(phi), _vp(St), _vp(E_na), _vp(g_na), stream)
    assert rc == 0, rc
    torch.cuda.synchronize()
    return (E_ws.cpu().numpy(), g_ws.cpu().numpy().astype(np.float64), E_na.cpu().numpy(),
            g_na.cpu().numpy().astype(np.float64), nb.value)


def test_noalloc_equals_workspace_entry_point_twice(dm):
    cases = [
        (dm.Spec(shape=(64, 64, 64), n_channels=2, n_levels=2, max_disp=(8, 4)), 2, 1),   # larger first
        (dm.Spec(shape=(128, 128), n_levels=2, max_disp=(16, 16)), 1, 2),              # then smaller
    ]
    sizes = []
    for spec, B, seed in cases:
        E_ws, g_ws, E_na, g_na, nbytes = run_both(dm, spec, B, seed)
        sizes.append(nbytes)
        print("case %s B=%d workspace %d bytes: E %s / %s, bitwise %s" % (
            spec.shape, B, nbytes, E_ws, E_na, np.array_equal(g_ws, g_na)), flush=True)
        assert np.all(np.isfinite(E_na)) and np.all(np.isfinite(g_na))
        np.testing.assert_allclose(E_na, E_ws, rtol=1e-12, atol=0)
        for b in range(B):
            assert np.linalg.norm(g_na[b] - g_ws[b]) <= 1e-4 * np.linalg.norm(g_ws[b])
    assert sizes[1] < sizes[0] <= 64 << 20


def test_noalloc_refuses_a_workspace_above_the_array(dm):
    """256^3 needs about 112 MB of scratch: refused before anything is launched
    (host-side check; the pointers are never dereferenced)."""
    L = dm.lib()
    spec = dm.Spec(shape=(256, 256, 256), max_disp=(32,))
    s = spec.c()
    nb = ctypes.c_size_t()
    assert L.dmcr_workspace_size(ctypes.byref(s), 1, ctypes.byref(nb)) == 0 and nb.value > 64 << 20
    fake = ctypes.c_void_p(1 << 24)
    assert L.dmcr_loss_grad_noalloc(ctypes.byref(s), 1, fake, fake, fake, fake, None) == -2
