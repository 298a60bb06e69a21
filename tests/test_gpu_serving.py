"""Serving loop (continuous batching): results are the same alone and in the mix,
match the oracle's tolerance-stopped solve, and admission follows the HBM budget."""
import numpy as np
import pytest

import oracle as O
from synth import make_instance, geometric_ladder

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests():
    reqs = []
    for j, (M, N, L, rank) in enumerate([(128, 128, 4, 1), (256, 64, 4, 2), (128, 256, 5, 1),
                                         (64, 64, 4, 1), (256, 256, 5, 2)]):
        lad = geometric_ladder(M, N, L) if M == N else \
            [(1, 1), (4, 4), (16, 16), (M, N)]
        inst = make_instance(M, N, lad, 0.02, rank=rank, noise=0.01, seed=100 + j)
        reqs.append((j, inst))
    return reqs


def _run(lib, reqs, max_active, budget=32 << 30, tol=1e-4, cap=300):
    srv = lib.Server(max_active=max_active, hbm_budget=budget, num_streams=4)
    outs = {}
    order = []
    ys = {}
    for rid, inst in reqs:
        ys[rid] = torch.from_numpy(inst.Y).cuda()
        srv.submit(rid, ys[rid], inst.ladder, iters=cap, tol=tol)
    for _ in range(100000):
        for (rid, iters, resid, status, Z) in srv.step():
            assert status == 0
            outs[rid] = (iters, resid, Z.cpu().numpy().copy())
            order.append(rid)
        if len(outs) == len(reqs):
            break
    srv.close()
    return outs, order


def test_server_alone_equals_mix_and_oracle(lib):
    reqs = _requests()
    mix, _ = _run(lib, reqs, max_active=5)
    for rid, inst in reqs:
        alone, _ = _run(lib, [(rid, inst)], max_active=1)
        it_a, r_a, Z_a = alone[rid]
        it_m, r_m, Z_m = mix[rid]
        print(f"request {rid} {inst.Y.shape} L={len(inst.ladder)}: alone {it_a} it r={r_a:.3e}; "
              f"mix {it_m} it r={r_m:.3e}", flush=True)
        # the same iteration count and bitwise the same components: every kernel treats
        # a block the same way whatever else runs beside it
        assert it_a == it_m
        for i in range(len(inst.ladder)):
            assert np.array_equal(Z_a[i], Z_m[i]), (rid, i)
    # against the oracle's tolerance-stopped ADMM, for two of the requests
    for rid, inst in reqs[:2]:
        ref = O.admm(inst.Y, inst.ladder, rho=1.0, iters=300, tol=1e-4, check_every=1)
        it_m, r_m, Z_m = mix[rid]
        ny = np.linalg.norm(inst.Y)
        errs = [np.linalg.norm(Z_m[i] - ref["Z"][i]) / max(np.linalg.norm(ref["Z"][i]), 1e-3 * ny)
                for i in range(len(inst.ladder))]
        print(f"request {rid}: oracle {ref['iters']} it, gpu {it_m} it, errs "
              + " ".join(f"{e:.1e}" for e in errs), flush=True)
        assert abs(ref["iters"] - it_m) <= max(3, ref["iters"] // 50)
        assert max(errs) <= 1e-3


def test_server_budget_admits_in_fifo_order(lib):
    reqs = _requests()[:4]
    # one request at a time (max_active = 1): completion follows submission order
    _, order = _run(lib, reqs, max_active=1, tol=1e-3, cap=50)
    assert order == [rid for rid, _ in reqs]


def test_server_budget_defers_second_class(lib):
    """Admission by HBM footprint: with a budget of 1.5x the larger class footprint two
    shape classes never hold memory together. Requests A1, B1, A2 (A and B two shapes):
    A1 runs alone; B1 waits at the queue head, and A2 behind it (first come, first
    served), until A1 retires and its idle class is released; then B1 runs alone, then
    A2. Each result equals its solo run bit for bit."""
    lad_a = [(1, 1), (4, 4), (16, 16), (128, 128)]
    lad_b = [(1, 1), (4, 4), (16, 16), (256, 64)]
    reqs = [(0, make_instance(128, 128, lad_a, 0.02, rank=1, noise=0.01, seed=200)),
            (1, make_instance(256, 64, lad_b, 0.02, rank=1, noise=0.01, seed=201)),
            (2, make_instance(128, 128, lad_a, 0.02, rank=2, noise=0.01, seed=202))]
    fa = lib.Server.class_bytes(128, 128, lad_a, max_active=4)
    fb = lib.Server.class_bytes(256, 64, lad_b, max_active=4)
    budget = int(1.5 * max(fa, fb))
    print(f"class bytes A {fa} B {fb}, budget {budget}", flush=True)
    assert fa + fb > budget >= max(fa, fb)
    cap = 20
    srv = lib.Server(max_active=4, hbm_budget=budget, num_streams=4)
    ys, outs, order, trace = {}, {}, [], []
    for rid, inst in reqs:
        ys[rid] = torch.from_numpy(inst.Y).cuda()
        srv.submit(rid, ys[rid], inst.ladder, iters=cap, tol=0.0)
    for _ in range(100000):
        for (rid, iters, resid, status, Z) in srv.step():
            assert status == 0
            outs[rid] = (iters, Z.cpu().numpy().copy())
            order.append(rid)
        trace.append((srv.active, srv.queued, len(order)))
        if len(outs) == len(reqs):
            break
    srv.close()
    print(f"completion order {order}; {len(trace)} steps; first {trace[0]}", flush=True)
    assert order == [0, 1, 2]
    assert all(a <= 1 for a, _, _ in trace), "two classes were resident at once"
    assert trace[0] == (1, 2, 0)       # B1 and A2 wait while A1 runs
    # B1 is admitted only after A1 retired (its idle class released), A2 only after B1
    for a, q, d in trace:
        assert q == 2 - d or (a == 0 and q == 3 - d), (a, q, d)
    for rid, inst in reqs:
        solo, _ = _run(lib, [(rid, inst)], max_active=1, tol=0.0, cap=cap)
        assert outs[rid][0] == solo[rid][0] == cap
        for i in range(len(inst.ladder)):
            assert np.array_equal(outs[rid][1][i], solo[rid][2][i]), (rid, i)
