"""Write the stored expected values of the large fixed-iteration parity cases.

Every number stored here comes from the float64 oracle (oracle/) run on the seeded
synthetic input of synth/; nothing is read from the GPU library. Run from the
repository root:

    python tests/golden/make_goldens.py [case ...]      (default: every case)

Each case is an ADMM solve of eq:admm with a fixed iteration count (no tolerance
stop). Its components Z_i are exactly block-low-rank in the partition of the last
iteration's cycle-spin shift, so they are stored compactly and losslessly (to float64
rounding): the 1 x 1 scale as its nonzero entries, every other scale as, per nonzero
block of Shift_s(Z_i), the factors U diag(sigma) and V of its thin SVD (the oracle's
Jacobi SVD) truncated where sigma <= 1e-13 ||block||_F. `load_case` in goldens.py
rebuilds the components.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from synth import make_instance, serving_trace  # noqa: E402
from tests.golden.goldens import CASES, case_instance, golden_path, y_digest  # noqa: E402


def compress(Z: np.ndarray, ladder, shifts) -> dict:
    out = {}
    M, N = Z.shape[1:]
    for i, (m, n) in enumerate(ladder):
        Zi = Z[i]
        if (m, n) == (1, 1):
            idx = np.flatnonzero(Zi)
            out[f"s{i}_idx"] = idx.astype(np.int64)
            out[f"s{i}_val"] = Zi.ravel()[idx]
            continue
        A = O.shift(Zi, shifts[i])
        P, Q = M // m, N // n
        blocks = A.reshape(P, m, Q, n).transpose(0, 2, 1, 3).reshape(P * Q, m, n)
        norms = np.sqrt((blocks ** 2).sum(axis=(1, 2)))
        ids = np.flatnonzero(norms > 0)
        ranks, Us, Vs = [], [], []
        if len(ids):
            U, s, V = O.jacobi_svd(blocks[ids])
            for k, b in enumerate(ids):
                r = int((s[k] > 1e-13 * norms[b]).sum())
                ranks.append(r)
                Us.append((U[k][:, :r] * s[k][:r]).T.ravel())   # r rows of length m
                Vs.append(V[k][:, :r].T.ravel())                # r rows of length n
        out[f"s{i}_blk"] = ids.astype(np.int64)
        out[f"s{i}_rank"] = np.asarray(ranks, dtype=np.int64)
        out[f"s{i}_U"] = np.concatenate(Us) if Us else np.zeros(0)
        out[f"s{i}_V"] = np.concatenate(Vs) if Vs else np.zeros(0)
        out[f"s{i}_shift"] = np.asarray(shifts[i], dtype=np.int64)
    return out


def make(name: str) -> None:
    spec = CASES[name]
    inst = case_instance(spec)
    t0 = time.time()
    ref = O.admm(inst.Y, inst.ladder, rho=spec["rho"], iters=spec["iters"],
                 cycle_spin=spec["cycle_spin"], seed=spec["shift_seed"])
    dt = time.time() - t0
    K = spec["iters"]
    shifts = [O.cycle_shift(spec["shift_seed"], K - 1, i, m, n) if spec["cycle_spin"] else (0, 0)
              for i, (m, n) in enumerate(inst.ladder)]
    arrs = compress(ref["Z"], inst.ladder, shifts)
    meta = dict(spec)
    meta.update(ladder=[list(x) for x in inst.ladder], lam=ref["lam"], resid=ref["resid"],
                oracle_iters=ref["iters"], y_digest=y_digest(inst.Y),
                z_norms=[float(np.linalg.norm(ref["Z"][i])) for i in range(len(inst.ladder))],
                oracle_seconds=round(dt, 1))
    arrs["meta"] = np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8)
    path = golden_path(name)
    np.savez_compressed(path, **arrs)
    # the stored form must rebuild the oracle's components
    from tests.golden.goldens import load_case
    Zr, _ = load_case(name)
    for i in range(len(inst.ladder)):
        d = np.linalg.norm(Zr[i] - ref["Z"][i])
        assert d <= 1e-12 * max(np.linalg.norm(ref["Z"][i]), 1.0), (name, i, d)
    print(f"{name}: {os.path.getsize(path) / 1024:.0f} KiB, oracle {dt:.0f} s, "
          f"resid {ref['resid']:.4e}", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CASES)
    for nm in names:
        make(nm)
