"""Batched solves: many independent decompositions of uneven sizes and ladders run
through stacked launches; each instance must match its solve alone and the oracle."""
import numpy as np
import pytest

import oracle as O
from synth import batch_instances, make_instance, full_ladder

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _problems(insts, iters, cycle_spin=True, tol=0.0):
    return [{"M": inst.Y.shape[0], "N": inst.Y.shape[1], "ladder": inst.ladder, "iters": iters,
             "cycle_spin": cycle_spin, "seed": j, "tol": tol} for j, inst in enumerate(insts)]


def _rel(a, b, scale):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-3 * scale))


def test_batch_matches_alone_and_oracle(lib):
    insts = batch_instances(14, seed=3)
    probs = _problems(insts, 30)
    batch = lib.Batch(probs)
    ncls = batch.classes
    Ys = [torch.from_numpy(inst.Y).cuda() for inst in insts]
    outs, infos = batch.solve(Ys)
    torch.cuda.synchronize()
    print(f"{len(insts)} instances in {ncls} classes", flush=True)
    assert ncls < len(insts)
    worst = 0.0
    for j, inst in enumerate(insts):
        Za, _ = lib.solve(Ys[j], inst.ladder, iters=30, cycle_spin=True, seed=j)
        torch.cuda.synchronize()
        zb = outs[j].cpu().numpy()
        za = Za.cpu().numpy()
        ny = np.linalg.norm(inst.Y)
        err = max(_rel(zb[i], za[i], ny) for i in range(len(inst.ladder)))
        worst = max(worst, err)
        assert infos[j]["iters"] == 30
        # every kernel treats a block the same way whatever else runs beside it
        assert np.array_equal(zb, za), (j, inst.Y.shape, inst.ladder, err)
    print(f"batch vs alone: worst rel diff {worst:.2e}", flush=True)
    for j in (0, 5):
        inst = insts[j]
        ref = O.admm(inst.Y, inst.ladder, iters=30, cycle_spin=True, seed=j)
        zb = outs[j].double().cpu().numpy()
        ny = np.linalg.norm(inst.Y)
        errs = [_rel(zb[i], ref["Z"][i], ny) for i in range(len(inst.ladder))]
        print(f"instance {j} {inst.Y.shape} vs oracle: " + " ".join(f"{e:.1e}" for e in errs),
              flush=True)
        assert max(errs) <= 1e-3
    batch.close()


def test_batch_per_instance_tolerance(lib):
    insts = [make_instance(64, 64, full_ladder(64, 64, (1, 4, 16)), 0.02, noise=0.01, seed=s)
             for s in range(4)]
    probs = _problems(insts, 400, cycle_spin=False, tol=1e-2)
    batch = lib.Batch(probs)
    assert batch.classes == 1
    Ys = [torch.from_numpy(inst.Y).cuda() for inst in insts]
    outs, infos = batch.solve(Ys)
    for j, inst in enumerate(insts):
        ref = O.admm(inst.Y, inst.ladder, iters=400, tol=1e-2, check_every=1)
        assert ref["iters"] < 400
        print(f"instance {j}: batch {infos[j]['iters']} it r={infos[j]['primal_resid']:.3e}; "
              f"oracle {ref['iters']} it", flush=True)
        assert abs(infos[j]["iters"] - ref["iters"]) <= 2
        assert infos[j]["primal_resid"] <= 1e-2
        zb = outs[j].double().cpu().numpy()
        ny = np.linalg.norm(inst.Y)
        assert max(_rel(zb[i], ref["Z"][i], ny) for i in range(len(inst.ladder))) <= 1e-3
    batch.close()
