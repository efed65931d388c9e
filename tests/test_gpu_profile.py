"""Kernel timing (dmcr_profile_start / dmcr_profile_stop), the source of the live
per-kernel figures of the benchmark line."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_09686_amd import dmcr
    dmcr.lib()
    return dmcr


def test_kernel_timing_table(dm):
    """dmcr_profile_start/stop: every launch of a 128^3 evaluation is timed, and the
    kernel times (taken from the dispatches themselves) fit inside the wall time of
    the evaluations they belong to."""
    import ctypes
    lib = dm.lib()

    class KStat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int32),
                    ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double)]

    lib.dmcr_profile_start.restype = ctypes.c_int
    lib.dmcr_profile_stop.restype = ctypes.c_int32
    lib.dmcr_profile_stop.argtypes = [ctypes.POINTER(KStat), ctypes.c_int32]
    shape = (128, 128, 128)
    spec = dm.make_spec(shape, 1, 1, 16)
    K = dm.dmcr_descriptor_size(spec)
    gen = torch.Generator(device="cuda").manual_seed(3)
    phi = torch.rand((1, 1) + shape, device="cuda", generator=gen)
    St = torch.rand((1, K), device="cuda", dtype=torch.float64, generator=gen) * 0.3
    E = torch.empty(1, dtype=torch.float64, device="cuda")
    g = torch.empty_like(phi)
    ws = dm.workspace(dm.dmcr_workspace_size(spec, 1))
    dm.dmcr_loss_grad(spec, phi, St, E, g, ws)
    E0, g0 = E.clone(), g.clone()
    torch.cuda.synchronize()
    steps = 5
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    assert lib.dmcr_profile_start() == 0
    t0.record()
    for _ in range(steps):
        dm.dmcr_loss_grad(spec, phi, St, E, g, ws)
    t1.record()
    stats = (KStat * 64)()
    nk = lib.dmcr_profile_stop(stats, 64)
    torch.cuda.synchronize()
    assert torch.equal(E, E0) and torch.equal(g, g0)      # timing changes no result
    assert 4 <= nk <= 64
    names = [stats[i].name.decode() for i in range(nk)]
    assert len(set(names)) == nk
    total = 0.0
    for i in range(nk):
        s = stats[i]
        assert s.launches % steps == 0 and s.launches > 0, names[i]
        assert s.total_ms > 0 and s.bytes > 0, names[i]
        total += s.total_ms
    # one stream: the kernels run one after another inside the timed interval
    assert total <= t0.elapsed_time(t1) * 1.01
    # recording is off again: a stop without a start reports an empty table
    assert lib.dmcr_profile_stop(stats, 64) == 0
