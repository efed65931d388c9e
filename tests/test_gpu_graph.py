"""The library allocates nothing, never synchronises inside dmcr_loss_grad and
records no memset, so a caller may capture an evaluation in a HIP graph (here via
torch.cuda.graph) and replay it.  Every replay must equal the eager result
bitwise, with eager evaluations and synchronisations between the replays.  One
case runs on the caller's stream only; the others fork side streams in the graph (the
levels of the pyramid), and in eager calls only for the largest batch."""
import numpy as np
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


# Eager calls fork side lanes from B C N >= 2^24 voxels; a captured call also
# forks them whenever it has levels to overlap, so the replays of the small
# multi-level cases run a different schedule than the eager calls they are
# compared with.  A recompute stays on its level's lane unless the batch is large
# and has one level.
@pytest.mark.parametrize("case", [((512, 512), 1, 1, 64, 1, 0), ((512, 512), 1, 3, 64, 1, 0),
                                  ((128, 128, 128), 2, 3, 32, 1, 0), ((128, 128, 128), 1, 3, 32, 2, 1),
                                  ((128, 128, 128), 2, 3, 32, 4, 0)],
                         ids=["2d512_one_stream", "2d512_levels_captured_lanes", "3d128_levels_captured_lanes",
                              "3d128_recompute_levels_captured_lanes",
                              "3d128_lanes_both"])
def test_captured_loss_grad_replays_bitwise(dm, case):
    shape, C, L, P, B, flags = case
    print("graph case", case, flush=True)
    spec = dm.make_spec(shape, C, L, P, flags=flags)
    K = dm.dmcr_descriptor_size(spec)
    gen = torch.Generator(device="cuda").manual_seed(5)
    phi = torch.rand((B, C) + shape, device="cuda", generator=gen)
    St = torch.rand((B, K), device="cuda", dtype=torch.float64, generator=gen) * 0.3
    E = torch.empty(B, dtype=torch.float64, device="cuda")
    g = torch.empty_like(phi)
    ws = dm.workspace(dm.dmcr_workspace_size(spec, B))

    def step():
        dm.dmcr_loss_grad(spec, phi, St, E, g, ws)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(3):
            step()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    E0, g0 = E.clone(), g.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(4):
        g.zero_()
        E.zero_()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(g, g0) and torch.equal(E, E0), r
        step()                      # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(g, g0) and torch.equal(E, E0), r
