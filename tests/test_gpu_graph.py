"""Iterations replayed from captured HIP graphs give the same results as plain launches
(every replay checked against a plain-launch run, with other eager work between the
replays), for plain, averaged-spinning and masked solves; plans whose low-rank scale
waits on the host do not use graphs."""
import numpy as np
import pytest
import torch

from synth import make_instance

pytestmark = pytest.mark.gpu

M, N = 128, 96
LADDER = [(1, 1), (4, 4), (8, 8), (16, 16), (32, 32), (M, N)]
KINDS = [0, 0, 0, 0, 0, 1]      # the last scale is the noise scale


@pytest.mark.parametrize("spin_count,masked", [(0, False), (3, False), (0, True)])
def test_graph_replays_match_plain_launches(lib, spin_count, masked):
    inst = make_instance(M, N, LADDER[:5], 0.05, noise=0.02, seed=31, keep_components=False)
    Y = torch.from_numpy(inst.Y).cuda()
    kw = dict(rho=1.0, iters=40, cycle_spin=True, seed=9, kinds=KINDS, spin_count=spin_count)
    a = lib.Solver(M, N, LADDER, **kw)
    b = lib.Solver(M, N, LADDER, **kw)
    assert a.set_graph(True) is True
    assert b.set_graph(False) is False
    if masked:
        mask = torch.from_numpy(np.random.default_rng(2).random((M, N)) < 0.7).cuda()
        a.set_mask(mask)
        b.set_mask(mask)
    ref, _ = b.solve(Y)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    for rep in range(3):
        got, info = a.solve(Y)
        torch.cuda.synchronize()
        assert info["iters"] == 40
        assert np.array_equal(got.cpu().numpy(), ref), rep
        # eager work between replays
        other, _ = b.solve(Y)
        (Y * 2.0).sum().item()
        torch.cuda.synchronize()
        assert np.array_equal(other.cpu().numpy(), ref)
    # new buffers: captured again
    Za = torch.empty((len(LADDER), M, N), device="cuda")
    Zb = torch.empty((len(LADDER), M, N), device="cuda")
    a.reset(Za)
    b.reset(Zb)
    a.step(Y, Za, 7)
    b.step(Y, Zb, 7)
    torch.cuda.synchronize()
    assert np.array_equal(Za.cpu().numpy(), Zb.cpu().numpy())
    a.close()
    b.close()


def test_host_waiting_plan_does_not_use_graphs(lib):
    s = lib.Solver(256, 256, [(1, 1), (16, 16), (256, 256)], iters=2)
    assert lib.TIERS[s.tier(2)] == "lowrank"
    assert s.set_graph(True) is False
    s.close()
