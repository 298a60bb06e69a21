"""The autotuner times the launch choices of a block size, records the fastest, and
later plans use it: the chosen tier is the one the solver reports, its block-wise SVT
matches the oracle, and a batch built afterwards equals its instances solved alone."""
import numpy as np
import pytest
import torch

import oracle as O
from synth import batch_instances

pytestmark = pytest.mark.gpu


def rel_err(got, ref, scale):
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-3 * scale))


@pytest.mark.parametrize("m,n", [(16, 16), (16, 4), (32, 32), (64, 64), (128, 128)])
def test_autotuned_choice_is_used_and_matches_oracle(lib, m, n):
    lib.autotune_clear()
    try:
        r = lib.autotune(m, n)
        print(f"autotune {m}x{n}: {r}", flush=True)
        assert r["candidates"] >= 1 and r["us_per_block"] > 0
        M, N = 4 * m, 6 * n
        rng = np.random.default_rng(m * 31 + n)
        V = (0.05 * rng.standard_normal((M, N))).astype(np.float32)
        for p in range(4):
            for q in range(0, 6, 2):
                V[p * m:(p + 1) * m, q * n:(q + 1) * n] += np.outer(
                    rng.standard_normal(m), rng.standard_normal(n)).astype(np.float32)
        s = lib.Solver(M, N, [(m, n)], iters=1)
        assert lib.TIERS[s.tier(0)] == r["tier"]
        shift = (int(rng.integers(0, m)), int(rng.integers(0, n)))
        tau = 0.5 * float(np.sqrt(m * n))
        ref = O.cycle_spun_bsvt(V.astype(np.float64), m, n, tau, shift)
        Z = s.bsvt(0, torch.from_numpy(V).cuda(), tau, shift)
        torch.cuda.synchronize()
        err = rel_err(Z.cpu().numpy(), ref, np.linalg.norm(V))
        print(f"  tier {r['tier']}: rel err {err:.2e}", flush=True)
        assert err <= 1e-4
        s.close()
    finally:
        lib.autotune_clear()


def test_autotuned_batch_equals_alone(lib):
    lib.autotune_clear()
    try:
        insts = batch_instances(6, seed=5)
        shapes = sorted({(m, n) for inst in insts for (m, n) in inst.ladder if m * n > 1})
        for (m, n) in shapes:
            lib.autotune(m, n)
        probs = [dict(M=inst.Y.shape[0], N=inst.Y.shape[1], ladder=inst.ladder, iters=20,
                      cycle_spin=True, seed=j) for j, inst in enumerate(insts)]
        b = lib.Batch(probs)
        Ys = [torch.from_numpy(inst.Y).cuda() for inst in insts]
        outs, _ = b.solve(Ys)
        torch.cuda.synchronize()
        for j, inst in enumerate(insts):
            Za, _ = lib.solve(Ys[j], inst.ladder, iters=20, cycle_spin=True, seed=j)
            torch.cuda.synchronize()
            ny = float(np.linalg.norm(inst.Y))
            err = max(rel_err(outs[j][i].cpu().numpy(), Za[i].cpu().numpy(), ny)
                      for i in range(len(inst.ladder)))
            assert torch.equal(outs[j], Za), (j, err)
        b.close()
    finally:
        lib.autotune_clear()
