"""Stored oracle results of the large fixed-iteration parity cases (written by
make_goldens.py, which calls only the oracle): the case recipes and the loader that
rebuilds the components from their compact block-low-rank form."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from synth import make_instance, serving_trace

HERE = os.path.dirname(os.path.abspath(__file__))


def _serving_request(index: int):
    """Request `index` of the serving workload's Poisson trace (seed 0)."""
    _, M, N, lad, rank, dseed = serving_trace(index + 1, 1.0, seed=0)[index]
    return M, N, lad, rank, dseed


# name -> recipe. Inputs follow the synth recipe; lambda is the default of eq:lambda;
# rho = 1; a fixed iteration count with no tolerance stop.
CASES = {
    # 512^2, blocks 1/4/16/64/512, 3% rank-1 blocks + N(0, 0.01^2), 100 iterations of
    # random cycle spinning (shift seed 1)
    "c2_512_k100": dict(M=512, N=512, ladder=[[1, 1], [4, 4], [16, 16], [64, 64], [512, 512]],
                        density=0.03, rank=1, noise=0.01, data_seed=0, iters=100,
                        cycle_spin=True, shift_seed=1, rho=1.0),
    # the 8192^2 benchmark ladder (1/8/32/128/512), density and noise on a 2048^2
    # instance, 50 iterations with random cycle spinning
    "c5_2048_k50": dict(M=2048, N=2048,
                        ladder=[[1, 1], [8, 8], [32, 32], [128, 128], [512, 512]],
                        density=0.01, rank=1, noise=0.01, data_seed=0, iters=50,
                        cycle_spin=True, shift_seed=0, rho=1.0),
    # serving request 5: 2048^2, six scales 1/4/16/64/256/2048, rank-2 blocks at 2% +
    # N(0, 0.01^2), no cycle spinning, 30 iterations
    "c4_req5_2048_k30": dict(serving_index=5, density=0.02, noise=0.01, iters=30,
                             cycle_spin=False, shift_seed=0, rho=1.0),
    # serving request 2: 1024 x 256, five scales 1/4/16/64/(1024 x 256), rank 2
    "c4_req2_1024x256_k30": dict(serving_index=2, density=0.02, noise=0.01, iters=30,
                                 cycle_spin=False, shift_seed=0, rho=1.0),
}


def case_instance(spec: dict):
    if "serving_index" in spec:
        M, N, lad, rank, dseed = _serving_request(spec["serving_index"])
        return make_instance(M, N, lad, spec["density"], rank=rank, noise=spec["noise"],
                             seed=dseed, keep_components=False)
    return make_instance(spec["M"], spec["N"], [tuple(x) for x in spec["ladder"]],
                         spec["density"], rank=spec["rank"], noise=spec["noise"],
                         seed=spec["data_seed"], keep_components=False)


def y_digest(Y: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(Y, dtype=np.float32).tobytes()).hexdigest()[:16]


def golden_path(name: str) -> str:
    return os.path.join(HERE, name + ".npz")


def load_case(name: str):
    """(Z, meta): the stored components (L, M, N) float64 and the case record."""
    d = np.load(golden_path(name))
    meta = json.loads(bytes(d["meta"]).decode())
    ladder = [tuple(x) for x in meta["ladder"]]
    if "serving_index" in meta:
        M, N = _serving_request(meta["serving_index"])[:2]
    else:
        M, N = meta["M"], meta["N"]
    Z = np.zeros((len(ladder), M, N))
    for i, (m, n) in enumerate(ladder):
        if (m, n) == (1, 1):
            Z[i].ravel()[d[f"s{i}_idx"]] = d[f"s{i}_val"]
            continue
        P, Q = M // m, N // n
        A = np.zeros((P * Q, m, n))
        Us, Vs, ranks = d[f"s{i}_U"], d[f"s{i}_V"], d[f"s{i}_rank"]
        ou = ov = 0
        for b, r in zip(d[f"s{i}_blk"], ranks):
            r = int(r)
            U = Us[ou:ou + r * m].reshape(r, m)
            V = Vs[ov:ov + r * n].reshape(r, n)
            ou += r * m
            ov += r * n
            A[b] = U.T @ V
        A = A.reshape(P, Q, m, n).transpose(0, 2, 1, 3).reshape(M, N)
        sr, sc = (int(x) for x in d[f"s{i}_shift"])
        Z[i] = np.roll(A, (sr, sc), axis=(0, 1))   # Shift_{-s}: back to the matrix grid
    return Z, meta
