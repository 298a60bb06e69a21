"""The configurations the benchmark's metric is quoted on, against stored oracle
results (tests/golden/*.npz, written by make_goldens.py from the float64 oracle):
fixed iteration counts, every component within 1e-3 (relative Frobenius error with a
1e-3 ||Y||_F floor), through the C ABI, in the solver and in the serving loop."""
import numpy as np
import pytest

from tests.golden.goldens import CASES, case_instance, load_case, y_digest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _errs(Zg, Zref, Y):
    ny = np.linalg.norm(Y.astype(np.float64))
    return [np.linalg.norm(Zg[i] - Zref[i]) / max(np.linalg.norm(Zref[i]), 1e-3 * ny)
            for i in range(Zref.shape[0])]


def _case(name):
    Zref, meta = load_case(name)
    inst = case_instance(CASES[name])
    assert y_digest(inst.Y) == meta["y_digest"], "the seeded generator changed"
    return Zref, meta, inst


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("fork_mode", [0, 2, 3])
def test_solver_against_golden(lib, name, fork_mode):
    """fork_mode 2 forces the single fork after every stream pass, the schedule the
    8192^2 benchmark runs (its planes exceed 2^24 elements); 0 is the automatic choice
    (forks right after each scale's own pass on these planes); 3 runs the scales one
    after another on one stream (the benchmark's timing run of the SVD kernels)."""
    Zref, meta, inst = _case(name)
    print(f"case {name} {inst.Y.shape} ladder={inst.ladder} K={meta['iters']} "
          f"fork_mode={fork_mode}", flush=True)
    Yd = torch.from_numpy(inst.Y).cuda()
    Z, info = lib.solve(Yd, inst.ladder, rho=meta["rho"], iters=meta["iters"],
                        cycle_spin=meta["cycle_spin"], seed=meta["shift_seed"],
                        fork_mode=fork_mode)
    torch.cuda.synchronize()
    errs = _errs(Z.double().cpu().numpy(), Zref, inst.Y)
    print(f"  errs " + " ".join(f"{e:.2e}" for e in errs) + f"; resid gpu "
          f"{info['primal_resid']:.4e} oracle {meta['resid']:.4e}; live {info['live']} "
          f"certified {info['certified']}", flush=True)
    assert info["iters"] == meta["iters"]
    assert max(errs) <= 1e-3
    assert abs(info["primal_resid"] - meta["resid"]) <= 1e-3 * meta["resid"] + 1e-6


@pytest.mark.parametrize("name", [n for n in CASES if "serving_index" in CASES[n]])
def test_server_against_golden(lib, name):
    """The serving loop retires at tol or the cap; with tol = 0 and the cap at the
    case's iteration count it runs exactly that many iterations. Both stored requests
    are submitted together, each must match its golden."""
    cases = {n: _case(n) for n in CASES if "serving_index" in CASES[n]}
    srv = lib.Server(max_active=4, hbm_budget=32 << 30, num_streams=4)
    ys = {}
    for rid, (nm, (Zref, meta, inst)) in enumerate(cases.items()):
        ys[rid] = torch.from_numpy(inst.Y).cuda()
        srv.submit(rid, ys[rid], inst.ladder, iters=meta["iters"], tol=0.0)
    outs = {}
    for _ in range(100000):
        for (rid, iters, resid, status, Z) in srv.step():
            assert status == 0
            outs[rid] = (iters, resid, Z.double().cpu().numpy())
        if len(outs) == len(cases):
            break
    srv.close()
    for rid, (nm, (Zref, meta, inst)) in enumerate(cases.items()):
        if nm != name:
            continue
        iters, resid, Zg = outs[rid]
        errs = _errs(Zg, Zref, inst.Y)
        print(f"server {nm}: {iters} it, resid {resid:.4e} (oracle {meta['resid']:.4e}); errs "
              + " ".join(f"{e:.2e}" for e in errs), flush=True)
        assert iters == meta["iters"]
        assert max(errs) <= 1e-3


def test_schedules_agree_bitwise(lib):
    """The fork schedule only changes when each scale's work is issued and on which
    stream: every fork_mode gives the same bits (20 iterations of the 512^2 case)."""
    inst = case_instance(CASES["c2_512_k100"])
    Yd = torch.from_numpy(inst.Y).cuda()
    outs = []
    for fm in (0, 1, 2, 3):
        print(f"fork_mode {fm}", flush=True)
        Z, info = lib.solve(Yd, inst.ladder, rho=1.0, iters=20, cycle_spin=True, seed=1,
                            fork_mode=fm)
        torch.cuda.synchronize()
        outs.append(Z)
    for fm, Z in zip((1, 2, 3), outs[1:]):
        assert torch.equal(Z, outs[0]), f"fork_mode {fm} differs from fork_mode 0"
