"""Continuous batching on the GPU: a request's result is the same alone and in the mix,
and a short mixed stream is served to the error tolerance."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_09686_amd import dmcr, serve
    dmcr.lib()
    return serve


@pytest.mark.parametrize("method", ["lbfgs", "adam"])
def test_alone_equals_in_the_mix(sv, method):
    from paper_2103_09686_amd import dmcr
    cache = sv.TargetCache()
    shape = (128, 128)
    stream = [(0.0, shape, 2, "boolean", 11), (0.0, shape, 2, "grf", 12), (0.0, shape, 2, "boolean", 13),
              (0.0, shape, 2, "grf", 14)]
    if method == "lbfgs":
        opt = dmcr.Opt(max_iter=60, tol_derr=1e-6)
    else:
        opt = dmcr.Opt(method=dmcr.OPT_ADAM, lr=1e-2, max_iter=60, tol_derr=1e-6)
    # alone: a group of one slot, one request
    ex1 = sv.GpuExecutor(opt=opt, max_slots=1, keep_fields=True)
    srv1 = sv.Server(ex1, budget_bytes=1 << 34, iters_per_tick=3, threads=1)
    alone = sv.gpu_requests(stream[:1], cache)
    srv1.run(alone)
    f_alone = list(srv1.groups.values())[0].fields[0]
    srv1.close()
    # in the mix: three other requests start first; the probe arrives two ticks later
    ex4 = sv.GpuExecutor(opt=opt, max_slots=4, keep_fields=True)
    srv4 = sv.Server(ex4, budget_bytes=1 << 34, iters_per_tick=3, threads=2)
    others = sv.gpu_requests(stream[1:], cache)
    for r in others:
        srv4.submit(r)
    srv4.tick()
    srv4.tick()
    probe = sv.gpu_requests(stream[:1], cache)[0]
    probe.rid = 99
    srv4.submit(probe)
    while not srv4.idle():
        srv4.tick()
    g = list(srv4.groups.values())[0]
    slot = [s for s, f in g.fields.items()]
    done = {r.rid: r for r in srv4.done}
    assert done[99].iters == alone[0].iters and done[99].final_E == alone[0].final_E
    # the probe took the first free slot after the three others: slot 3
    assert torch.equal(g.fields[3], f_alone)
    srv4.close()


@pytest.mark.parametrize("asynchronous", [False, True])
def test_short_mixed_stream_converges(sv, asynchronous):
    from paper_2103_09686_amd import dmcr
    cache = sv.TargetCache(variants=1)
    sizes = [(128, 128), (256, 256), (64, 64, 64)]
    stream = sv.request_stream(24, 40.0, seed=5, sizes=sizes)
    reqs = sv.gpu_requests(stream, cache)
    ex = sv.GpuExecutor(opt=dmcr.Opt(max_iter=2000, tol_derr=1e-4))
    srv = sv.Server(ex, budget_bytes=8 << 30, iters_per_tick=4, threads=4, asynchronous=asynchronous)
    done = srv.run(reqs)
    srv.close()
    s = sv.summary(done)
    print(s, flush=True)
    assert s["requests"] == 24 and s["converged"] == 24 and s["max_final_E"] <= 1e-4
