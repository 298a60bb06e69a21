"""The serving workload's retirement tolerance at rho = 1 (Sec. 7 eq:admm): the plain
ADMM iteration does not bring the primal residual of a 128^2 serving request below
1e-4 within the 300-iteration cap, so served requests retire at the cap. This is a
property of the method at this rho, pinned here on the oracle alone."""
import oracle as O
from synth import make_instance, serving_trace


def test_oracle_r300_above_serving_tolerance():
    _, M, N, lad, rank, dseed = serving_trace(2, 1.0, seed=0)[1]
    assert (M, N) == (128, 128) and len(lad) == 4
    inst = make_instance(M, N, lad, 0.02, rank=rank, noise=0.01, seed=dseed,
                         keep_components=False)
    ref = O.admm(inst.Y, inst.ladder, rho=1.0, iters=300, tol=1e-4, check_every=1)
    print(f"request 1 {M}x{N} ladder {lad}: {ref['iters']} iterations, r = {ref['resid']:.3e}")
    assert ref["iters"] == 300
    assert ref["resid"] > 1e-4
