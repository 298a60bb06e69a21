"""Pins for the FP64 oracle: facts fixed by the paper and by mathematics, independent
of the oracle's own formulas (closed forms, optimality conditions, brute force,
published generator outputs, exact invariances of the iteration)."""
import math
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from synth import make_instance

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_hex(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append(int(line, 16))
    return out


# ----------------------------------------------------------------- shift hash (Sec. 9)
def test_splitmix64_published_outputs():
    ref = _golden_hex("splitmix64_seed0.txt")
    state = 0
    for want in ref:
        state = (state + 0x9E3779B97F4A7C15) & O.MASK64
        assert O.splitmix64_mix(state) == want


def test_cycle_shift_counter_layout():
    # seed 0: counter 16k+i+1 = 1..4 for (k=0, i=0..3) gives the published stream.
    ref = _golden_hex("splitmix64_seed0.txt")
    for i, z in enumerate(ref):
        for (m, n) in [(4, 4), (8, 32), (512, 512), (7, 3), (1, 1)]:
            assert O.cycle_shift(0, 0, i, m, n) == ((z >> 32) % m, (z & 0xFFFFFFFF) % n)
    # (k=1, i=0) uses counter 17: 17 steps of the same stream
    state = 0
    for _ in range(17):
        state = (state + 0x9E3779B97F4A7C15) & O.MASK64
    z = O.splitmix64_mix(state)
    assert O.cycle_shift(0, 1, 0, 64, 64) == ((z >> 32) % 64, (z & 0xFFFFFFFF) % 64)


def test_shift_definition_bruteforce():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((5, 7))
    s = (3, 4)
    S = O.shift(A, s)
    for r in range(5):
        for c in range(7):
            assert S[r, c] == A[(r + 3) % 5, (c + 4) % 7]
    assert np.array_equal(O.unshift(S, s), A)


# ------------------------------------------------------------------ lambda (Sec. 4)
def test_lambda_special_cases():
    # full M x N block: sqrt(M) + sqrt(N) + sqrt(log(min(M, N)))
    assert math.isclose(O.default_lambda(64, 128, 64, 128),
                        8 + math.sqrt(128) + math.sqrt(math.log(64)), rel_tol=1e-15)
    # 1 x 1 blocks: 2 + sqrt(log(M N))
    assert math.isclose(O.default_lambda(512, 512, 1, 1), 2 + math.sqrt(math.log(512 * 512)),
                        rel_tol=1e-15)
    # noise-like MN x 1 reshape would give sqrt(MN) + 1 + 0
    assert math.isclose(O.default_lambda(1, 4096, 1, 4096), 1 + 64 + math.sqrt(math.log(1)),
                        rel_tol=1e-15)


# ------------------------------------------------------- Jacobi SVD (eq:svt's SVD)
@pytest.mark.parametrize("shape", [(12, 12), (40, 17), (17, 40), (1, 9), (9, 1), (64, 64),
                                   (3, 130)])
def test_jacobi_svd_reconstruction_and_orthogonality(shape):
    """B = U diag(s) V^T to 1e-13 ||B||, U and V with orthonormal columns, singular
    values equal to LAPACK's (a library routine, used here only as a checker)."""
    rng = np.random.default_rng(sum(shape))
    B = rng.standard_normal(shape) * np.exp(rng.uniform(-3, 3, size=(1, shape[1])))
    U, s, V = O.jacobi_svd(B)
    k = min(shape)
    assert U.shape == (shape[0], k) and V.shape == (shape[1], k) and s.shape == (k,)
    nb = np.linalg.norm(B)
    assert np.linalg.norm(U * s @ V.T - B) <= 1e-13 * nb
    assert np.abs(U.T @ U - np.eye(k)).max() <= 1e-13
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-13
    assert np.all(np.diff(s) <= 0) and s[-1] >= 0
    assert np.abs(s - np.linalg.svd(B, compute_uv=False)).max() <= 1e-13 * s[0]


def test_jacobi_svd_exact_cases():
    rng = np.random.default_rng(3)
    # diagonal (already orthogonal columns): no rotation, |d| sorted, one sweep
    d = np.array([0.5, -3.0, 0.0, 2.0, -1e-3])
    U, s, V, sw = O.jacobi_svd(np.diag(d), return_sweeps=True)
    assert sw == 1
    assert np.array_equal(s, np.sort(np.abs(d))[::-1])
    # rank one: sigma_1 = ||u|| ||v||, the rest zero to rounding
    u, v = rng.standard_normal(30), rng.standard_normal(20)
    s = O.jacobi_svd(np.outer(u, v))[1]
    assert abs(s[0] - np.linalg.norm(u) * np.linalg.norm(v)) <= 1e-13 * s[0]
    assert s[1:].max() <= 1e-13 * s[0]
    # orthogonal columns of chosen lengths: those lengths exactly (to rounding)
    Q = np.linalg.qr(rng.standard_normal((25, 6)))[0]
    lens = np.array([4.0, 1.0, 9.0, 0.25, 2.0, 7.0])
    s = O.jacobi_svd(Q * lens)[1]
    assert np.abs(s - np.sort(lens)[::-1]).max() <= 1e-13 * 9.0
    # zero block and zero columns: zero singular values with zero left vectors
    Z = np.zeros((6, 4))
    U, s, V = O.jacobi_svd(Z)
    assert np.all(s == 0) and np.all(U == 0)
    B = rng.standard_normal((8, 5))
    B[:, 2] = 0.0
    U, s, V = O.jacobi_svd(B)
    assert s[-1] == 0.0 and np.all(U[:, -1] == 0.0)
    assert np.linalg.norm(U * s @ V.T - B) <= 1e-13 * np.linalg.norm(B)


def test_jacobi_svd_batched_equals_single():
    rng = np.random.default_rng(5)
    B = rng.standard_normal((7, 10, 6))
    U, s, V = O.jacobi_svd(B)
    for b in range(7):
        u1, s1, v1 = O.jacobi_svd(B[b])
        assert np.array_equal(s[b], s1) and np.array_equal(U[b], u1) and np.array_equal(V[b], v1)


def test_jacobi_svd_sweep_cap_is_reported():
    rng = np.random.default_rng(9)
    with pytest.raises(RuntimeError):
        O.jacobi_svd(rng.standard_normal((30, 30)), max_sweeps=1)


# ------------------------------------------------------------------ SVT (eq:svt)
def _spec_norm(A):
    return math.sqrt(max(np.linalg.eigvalsh(A.T @ A).max(), 0.0))


def _nuc_norm(A):
    # eigenvalues of A^T A that are rounding noise around an exact zero are dropped
    ev = np.linalg.eigvalsh(A.T @ A)
    ev[ev < 1e-12 * max(ev.max(), 1e-300)] = 0.0
    return float(np.sqrt(ev).sum())


@pytest.mark.parametrize("shape", [(6, 6), (9, 4), (3, 11), (16, 16), (1, 7), (5, 1)])
@pytest.mark.parametrize("q", [0.1, 0.5, 0.9])
def test_svt_prox_optimality(shape, q):
    """Z = prox_{tau ||.||_*}(B) iff G = B - Z satisfies ||G||_2 <= tau and
    <G, Z> = tau ||Z||_* (subdifferential of the nuclear norm, Sec. 5.1)."""
    rng = np.random.default_rng(hash((shape, q)) % 2**32)
    B = rng.standard_normal(shape) * 3
    sv = np.sqrt(np.clip(np.linalg.eigvalsh(B.T @ B), 0, None))
    tau = float(np.quantile(sv, q)) + 1e-3
    Z = O.svt(B, tau)
    G = B - Z
    assert _spec_norm(G) <= tau * (1 + 1e-10)
    assert abs(float((G * Z).sum()) - tau * _nuc_norm(Z)) <= 1e-9 * max(1.0, tau * _nuc_norm(Z))


def test_svt_bruteforce_2x2():
    """Direct minimisation of 0.5||Z - V||^2 + tau ||Z||_* over 2x2 matrices, with the
    SVD-free identity ||Z||_* = sqrt(||Z||_F^2 + 2 |det Z|)."""
    rng = np.random.default_rng(7)
    for trial in range(12):
        V = rng.standard_normal((2, 2)) * 2
        tau = float(rng.uniform(0.1, 2.5))

        def f(z):
            Z = z.reshape(2, 2)
            nuc = math.sqrt(max((Z * Z).sum() + 2 * abs(np.linalg.det(Z)), 0.0))
            return 0.5 * ((Z - V) ** 2).sum() + tau * nuc

        best = None
        for x0 in [np.zeros(4), V.ravel(), 0.5 * V.ravel(), rng.standard_normal(4)]:
            res = minimize(f, x0, method="Nelder-Mead",
                           options={"xatol": 1e-12, "fatol": 1e-14, "maxiter": 40000,
                                    "maxfev": 40000})
            if best is None or res.fun < best.fun:
                best = res
        Z = O.svt(V, tau)
        assert f(Z.ravel()) <= best.fun + 1e-12
        assert np.abs(Z.ravel() - best.x).max() < 1e-5


def test_svt_rank1_closed_form():
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(7), rng.standard_normal(5)
    B = np.outer(u, v)
    sig = np.linalg.norm(u) * np.linalg.norm(v)
    for tau in [0.1 * sig, 0.7 * sig, 1.3 * sig]:
        want = max(1 - tau / sig, 0.0) * B
        assert np.allclose(O.svt(B, tau), want, atol=1e-12 * sig)


# ------------------------------------------------------------ BlockSVT (eq:bsvt)
def test_bsvt_1x1_is_soft_threshold():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((12, 10)) * 2
    tau = 0.8
    want = np.sign(A) * np.maximum(np.abs(A) - tau, 0)
    assert np.allclose(O.block_svt(A, 1, 1, tau), want, atol=1e-14)
    assert np.allclose(O.cycle_spun_bsvt(A, 1, 1, tau, (0, 0)), want, atol=1e-14)


@pytest.mark.parametrize("m,n,s", [(1, 10, (3, 0)), (1, 5, (2, 3)), (12, 1, (5, 0)),
                                   (4, 1, (3, 0))])
def test_bsvt_group_soft_threshold_with_wrap(m, n, s):
    """1 x n (and m x 1) blocks: joint soft-threshold v max(1 - tau/||v||, 0) per group,
    groups taken on the cyclically shifted grid (brute-force index loops)."""
    rng = np.random.default_rng(2)
    M, N = 12, 10
    A = rng.standard_normal((M, N))
    tau = 1.1
    want = np.zeros_like(A)
    for p in range(M // m):
        for q in range(N // n):
            idx = [((p * m + s[0] + r) % M, (q * n + s[1] + c) % N)
                   for r in range(m) for c in range(n)]
            v = np.array([A[i] for i in idx])
            g = max(1 - tau / np.linalg.norm(v), 0.0)
            for (i, val) in zip(idx, v):
                want[i] = g * val
    got = O.cycle_spun_bsvt(A, m, n, tau, s)
    assert np.allclose(got, want, atol=1e-13)


def test_bsvt_planted_rank1_blocks_wrapped():
    """Rank-1 blocks planted on the shifted grid are each scaled by (1 - tau/sigma_b)+,
    which only holds if gather/scatter wrap exactly as Shift_s prescribes."""
    rng = np.random.default_rng(4)
    M, N, m, n, s = 12, 18, 3, 6, (2, 5)
    A = np.zeros((M, N))
    want = np.zeros((M, N))
    tau = 2.0
    for p in range(M // m):
        for q in range(N // n):
            u, v = rng.standard_normal(m), rng.standard_normal(n)
            sig = np.linalg.norm(u) * np.linalg.norm(v)
            g = max(1 - tau / sig, 0.0)
            for r in range(m):
                for c in range(n):
                    pos = ((p * m + s[0] + r) % M, (q * n + s[1] + c) % N)
                    A[pos] = u[r] * v[c]
                    want[pos] = g * u[r] * v[c]
    assert np.allclose(O.cycle_spun_bsvt(A, m, n, tau, s), want, atol=1e-12)
    # the unshifted grid does not see rank-1 blocks: the result must differ
    assert not np.allclose(O.block_svt(A, m, n, tau), want, atol=1e-6)


def test_skip_bound_dominates_sigma_max():
    rng = np.random.default_rng(5)
    for shape in [(4, 4), (8, 8), (16, 3), (32, 32), (1, 9)]:
        for _ in range(20):
            B = rng.standard_normal(shape) * rng.uniform(0.01, 10)
            B[rng.random(shape) < 0.5] = 0
            smax = _spec_norm(B)
            assert O.skip_bound_sq(B) >= smax ** 2 * (1 - 1e-12)


# ------------------------------------------------------------------ ADMM (eq:admm)
def test_admm_single_scale_converges_to_Y():
    """L = 1: the only feasible point is X_1 = Y, so Z_1 -> Y."""
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((16, 16))
    out = O.admm(Y, [(4, 4)], rho=1.0, iters=400)
    assert np.linalg.norm(out["Z"][0] - Y) / np.linalg.norm(Y) < 1e-8


def test_admm_exact_rescaling():
    """eq:cvx is positively homogeneous and the BSVT threshold is lambda/rho, so the
    iterates for (cY, rho/c) are exactly c times those for (Y, rho) at every K."""
    inst = make_instance(32, 32, [(1, 1), (4, 4), (8, 8), (32, 32)], 0.05, noise=0.01, seed=3)
    c = 3.7
    a = O.admm(inst.Y, inst.ladder, rho=1.0, iters=25, cycle_spin=True, seed=11)
    b = O.admm(c * inst.Y.astype(np.float64), inst.ladder, rho=1.0 / c, iters=25,
               cycle_spin=True, seed=11)
    assert np.abs(b["Z"] - c * a["Z"]).max() <= 1e-10 * np.abs(c * a["Z"]).max()
    assert np.abs(b["U"] - c * a["U"]).max() <= 1e-10 * max(np.abs(c * a["U"]).max(), 1)


def test_admm_transpose_symmetry():
    inst = make_instance(24, 40, [(1, 1), (2, 4), (6, 8), (24, 40)], 0.1, seed=5)
    lam = [2.0, 3.0, 5.0, 9.0]
    a = O.admm(inst.Y, inst.ladder, lam=lam, iters=30)
    bt = O.admm(inst.Y.T.copy(), [(n, m) for (m, n) in inst.ladder], lam=lam, iters=30)
    assert np.allclose(bt["Z"], a["Z"].transpose(0, 2, 1), atol=1e-12)


def test_admm_grid_shift_equivariance():
    inst = make_instance(32, 32, [(1, 1), (4, 4), (8, 8)], 0.1, seed=8)
    a = O.admm(inst.Y, inst.ladder, iters=30)
    d = (8, 16)
    b = O.admm(np.roll(inst.Y, d, axis=(0, 1)), inst.ladder, iters=30)
    assert np.allclose(b["Z"], np.roll(a["Z"], d, axis=(1, 2)), atol=1e-12)


def test_admm_dual_residual():
    """The dual residual rho ||Z^k - Z^(k-1)|| / ||Y||: from Z^0 = 0 the first one is
    rho ||Z^1|| / ||Y||; it vanishes at the fixed point and scales with rho."""
    inst = make_instance(16, 16, [(1, 1), (4, 4), (16, 16)], 0.05, seed=0)
    Y = inst.Y.astype(np.float64)
    one = O.admm(Y, inst.ladder, rho=2.0, iters=1)
    assert math.isclose(one["dual"], 2.0 * np.linalg.norm(one["Z"]) / np.linalg.norm(Y),
                        rel_tol=1e-12)
    assert O.admm(Y, inst.ladder, rho=2.0, iters=5)["dual"] > 1e-3
    assert O.admm(Y, inst.ladder, rho=2.0, iters=1500)["dual"] < 1e-8


def test_admm_kkt_and_duality_gap():
    """At convergence (no cycle spinning) the ADMM fixed point solves eq:cvx:
    consensus sum Z_i = Y, all U_i equal, rho*U is dual feasible with the dual norm
    attained on scales carrying signal, and the primal-dual gap closes."""
    inst = make_instance(16, 16, [(1, 1), (4, 4), (16, 16)], 0.05, seed=0)
    Y = inst.Y.astype(np.float64)
    out = O.admm(Y, inst.ladder, rho=2.0, iters=1500)
    rep = O.kkt_report(Y, inst.ladder, out["lam"], 2.0, out["Z"], out["U"])
    assert out["resid"] < 1e-7
    assert rep["consensus"] < 1e-7
    assert rep["u_spread"] < 1e-9
    assert max(rep["dual_ratio"]) <= 1 + 1e-9
    for i in range(3):
        if np.abs(out["Z"][i]).max() > 1e-6:
            assert rep["dual_ratio"][i] > 1 - 1e-6
    assert abs(rep["gap"]) < 2e-7
    # early iterates are not optimal: the certificate is not trivially satisfied
    early = O.admm(Y, inst.ladder, rho=2.0, iters=20)
    rep0 = O.kkt_report(Y, inst.ladder, early["lam"], 2.0, early["Z"], early["U"])
    assert rep0["gap"] > 1e-4


@pytest.mark.parametrize("ladder,bar", [([(1, 1), (32, 32)], 5),
                                         ([(1, 1), (4, 4), (32, 32)], 4)])
def test_admm_recovers_sparse_multiscale_truth(ladder, bar):
    """Exact recovery on sparse incoherent instances (Thm 5.1; the Sec. 4 remark that
    the suggested lambda recovers matched models; low rank + sparse is the 2-scale
    case). Family: 32x32, density 0.01 (10 sparse entries, one rank-1 block per
    larger scale), no noise, seeds 0..4, stop at r <= 1e-6 (cap 4000). Success =
    every component within 1e-2 relative of the truth; `bar` successes required."""
    ok = 0
    for seed in range(5):
        inst = make_instance(32, 32, ladder, 0.01, seed=seed)
        out = O.admm(inst.Y, inst.ladder, rho=1.0, iters=4000, tol=1e-6, check_every=20)
        errs = [np.linalg.norm(out["Z"][i] - inst.components[i]) /
                max(np.linalg.norm(inst.components[i]), 1e-12) for i in range(len(ladder))]
        ok += max(errs) < 1e-2
    assert ok >= bar


def test_admm_tolerance_stop_and_history():
    inst = make_instance(16, 16, [(1, 1), (4, 4), (16, 16)], 0.1, seed=2)
    out = O.admm(inst.Y, inst.ladder, iters=500, tol=1e-2, check_every=5, history=True)
    assert out["iters"] % 5 == 0 and out["resid"] <= 1e-2 and out["iters"] < 500
    assert len(out["history"]) == out["iters"]
    assert all(h > 1e-2 for h in out["history"][4:out["iters"] - 1:5])


# ------------------------------------------------------------------ noise scale
@pytest.mark.parametrize("scale", [0.3, 3.0])
def test_noise_svt_prox_optimality(scale):
    """The noise scale's Z-step is the prox of tau ||.||_F (Sec. 2: SVT of the MN x 1
    reshape). Optimality: 0 in Z - V + tau dF(Z) with dF(0) the unit ball and
    dF(Z) = Z / ||Z||_F otherwise; checked on both sides of ||V||_F = tau."""
    rng = np.random.default_rng(11)
    V = scale * rng.standard_normal((12, 9))
    tau = 1.7
    Z = O.noise_svt(V, tau)
    nv = np.linalg.norm(V)
    if nv <= tau:
        assert np.abs(Z).max() == 0.0
    else:
        nz = np.linalg.norm(Z)
        assert nz > 0
        assert np.abs(Z - V + tau * Z / nz).max() < 1e-12
        # the prox is the minimiser: compare with perturbed candidates
        f = lambda X: 0.5 * ((X - V) ** 2).sum() + tau * np.linalg.norm(X)
        for _ in range(20):
            D = 1e-3 * rng.standard_normal(V.shape)
            assert f(Z) <= f(Z + D) + 1e-15


def test_noise_lambda_is_the_mn_by_1_block():
    """eq:lambda on the MN x 1 block: sqrt(MN) + 1 + sqrt(log 1) = sqrt(MN) + 1, the
    sqrt(MN) scaling Sec. 4 states for the noise matrix."""
    assert abs(O.scale_lambda(64, 48, 64, 48, O.KIND_NOISE) - (math.sqrt(64 * 48) + 1)) < 1e-12
    assert O.scale_lambda(64, 48, 8, 4) == O.default_lambda(64, 48, 8, 4)


def test_admm_noise_only_converges_to_Y():
    """With the noise scale alone the constraint X = Y decides: Z -> Y."""
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((16, 12))
    out = O.admm(Y, [(16, 12)], rho=1.0, iters=400, kinds=[O.KIND_NOISE])
    assert np.abs(out["Z"][0] - Y).max() < 1e-8


def test_admm_noisy_program_kkt_and_gap():
    """eq:noisy (Sec. 6): sparse + low rank + noise scale. At convergence the dual
    certificate Q = rho mean U_i meets every scale's dual norm bound (Frobenius for
    the noise scale) and the duality gap vanishes."""
    inst = make_instance(16, 16, [(1, 1), (16, 16)], 0.05, noise=0.05, seed=2)
    Y = inst.Y.astype(np.float64)
    ladder = [(1, 1), (16, 16), (16, 16)]
    kinds = [O.KIND_BLOCK, O.KIND_BLOCK, O.KIND_NOISE]
    lam = [O.scale_lambda(16, 16, m, n, k) for (m, n), k in zip(ladder, kinds)]
    lam[2] *= 0.25          # a noise weight that leaves both other scales active
    out = O.admm(Y, ladder, lam=lam, rho=1.0, iters=3000, kinds=kinds)
    rep = O.kkt_report(Y, ladder, lam, 1.0, out["Z"], out["U"], kinds=kinds)
    assert out["resid"] < 1e-7
    assert rep["u_spread"] < 1e-7
    assert max(rep["dual_ratio"]) <= 1 + 1e-7
    assert rep["dual_ratio"][2] > 1 - 1e-6          # the noise component is non-zero
    assert abs(rep["gap"]) < 1e-6


# ------------------------------------------------------------- masked consistency
def test_admm_full_mask_is_the_plain_iteration():
    """Sec. 10's masked data consistency with every entry observed is eq:admm."""
    inst = make_instance(16, 16, [(1, 1), (4, 4)], 0.1, noise=0.01, seed=1)
    a = O.admm(inst.Y, inst.ladder, iters=30, cycle_spin=True, seed=2)
    b = O.admm(inst.Y, inst.ladder, iters=30, cycle_spin=True, seed=2,
               mask=np.ones((16, 16), dtype=bool))
    assert np.array_equal(a["Z"], b["Z"])


def test_admm_masked_completion_recovers_low_rank():
    """One full-size scale with a mask is nuclear-norm matrix completion; a rank-2
    32 x 32 matrix with 60% of its entries observed at random is recovered exactly
    (to the iteration's precision), so the unobserved entries are filled in, which a
    consensus applied everywhere (or nowhere) would not do."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((32, 2)) @ rng.standard_normal((2, 32))
    mask = rng.random((32, 32)) < 0.6
    out = O.admm(A, [(32, 32)], rho=1.0, iters=3000, mask=mask)
    assert np.linalg.norm(out["Z"][0] - A) / np.linalg.norm(A) < 1e-8
    assert np.linalg.norm(np.where(mask, 0.0, A)) > 0.25 * np.linalg.norm(A)


def test_admm_masked_kkt_and_gap():
    """At convergence of the masked program the dual certificate lives on the observed
    entries, meets every dual-norm bound, and the duality gap vanishes. (Mask seed 1:
    some masks leave this small instance with a slowly converging iteration.)"""
    inst = make_instance(16, 16, [(1, 1), (4, 4), (16, 16)], 0.05, seed=0)
    Y = inst.Y.astype(np.float64)
    mask = np.random.default_rng(1).random((16, 16)) < 0.7
    out = O.admm(Y, inst.ladder, rho=2.0, iters=3000, mask=mask)
    rep = O.kkt_report(Y, inst.ladder, out["lam"], 2.0, out["Z"], out["U"], mask=mask)
    assert out["resid"] < 1e-7
    assert rep["consensus"] < 1e-7
    assert rep["off_support"] < 1e-12
    assert max(rep["dual_ratio"]) <= 1 + 1e-9
    assert abs(rep["gap"]) < 2e-7


# ------------------------------------------------------------ averaged spinning
def test_full_cycle_spinning_is_translation_equivariant():
    """Averaging over every shift (Sec. 9) makes the block-wise SVT translation
    invariant: T(Shift_t V) = Shift_t T(V) for any t, which a single partition is not."""
    rng = np.random.default_rng(4)
    V = rng.standard_normal((12, 16))
    m, n, tau = 4, 4, 0.9
    S = O.spin_shifts(0, 0, 0, m, n, m * n)
    assert len(S) == m * n and len(set(S)) == m * n
    T = lambda A: O.averaged_bsvt(A, m, n, tau, S)
    t = (3, 5)
    assert np.abs(T(O.shift(V, t)) - O.shift(T(V), t)).max() < 1e-12
    single = lambda A: O.cycle_spun_bsvt(A, m, n, tau, (0, 0))
    assert np.abs(single(O.shift(V, t)) - O.shift(single(V), t)).max() > 1e-3


def test_spin_count_one_is_random_cycle_spinning():
    inst = make_instance(32, 32, [(1, 1), (4, 4), (16, 16)], 0.05, noise=0.01, seed=3)
    a = O.admm(inst.Y, inst.ladder, iters=15, cycle_spin=True, seed=7)
    b = O.admm(inst.Y, inst.ladder, iters=15, cycle_spin=True, seed=7, spin_count=1)
    assert np.array_equal(a["Z"], b["Z"])
    # the first hashed shift of a spin set is the plain random shift
    assert O.spin_shifts(7, 3, 2, 16, 16, 4)[0] == O.cycle_shift(7, 3, 2, 16, 16)


def test_averaged_prox_is_nonexpansive():
    """Each Shift_{-s} BSVT Shift_s is a prox (firmly non-expansive), so their average
    is non-expansive: ||T(A) - T(B)|| <= ||A - B||."""
    rng = np.random.default_rng(6)
    S = O.spin_shifts(1, 0, 0, 8, 8, 5)
    for _ in range(5):
        A = rng.standard_normal((16, 24))
        B = A + 0.3 * rng.standard_normal((16, 24))
        TA = O.averaged_bsvt(A, 8, 8, 1.1, S)
        TB = O.averaged_bsvt(B, 8, 8, 1.1, S)
        assert np.linalg.norm(TA - TB) <= np.linalg.norm(A - B) + 1e-12


def test_averaged_bsvt_normalisation():
    """tau = 0 makes every shifted BlockSVT the identity, so the mean is the input; tau
    above every block norm makes it zero (checks the 1/|S| factor and the unshift)."""
    rng = np.random.default_rng(9)
    V = rng.standard_normal((16, 16))
    S = O.spin_shifts(2, 1, 1, 4, 8, 7)
    assert np.abs(O.averaged_bsvt(V, 4, 8, 0.0, S) - V).max() < 1e-12
    assert np.abs(O.averaged_bsvt(V, 4, 8, 1e3, S)).max() == 0.0


def test_spanning_axis_needs_one_shift():
    """A block that spans all rows (m = M): a cyclic row shift permutes rows inside each
    block, so the shifted BlockSVT does not change, and the reduced full set (column
    shifts only) is still translation equivariant in both axes."""
    rng = np.random.default_rng(10)
    V = rng.standard_normal((12, 16))
    M, N, m, n, tau = 12, 16, 12, 4, 1.3
    assert O.spin_extent(M, N, m, n) == (1, 4)
    for r in (1, 5, 11):
        a = O.cycle_spun_bsvt(V, m, n, tau, (r, 3))
        b = O.cycle_spun_bsvt(V, m, n, tau, (0, 3))
        assert np.abs(a - b).max() < 1e-12
    S = O.spin_shifts(0, 0, 0, m, n, 100, M, N)
    assert S == [(0, 0), (0, 1), (0, 2), (0, 3)]
    T = lambda A: O.averaged_bsvt(A, m, n, tau, S)
    for t in ((5, 3), (0, 7), (4, 0)):
        assert np.abs(T(O.shift(V, t)) - O.shift(T(V), t)).max() < 1e-12


# ------------------------------------------------------------- space-time blocks
def _brute_spacetime(A, H, W, ph, pw, bt, tau, s):
    """Space-time BlockSVT by index loops: gather each shifted (ph pw) x bt block pixel
    by pixel with wrap in y, x and t, threshold it with a library SVD, scatter back."""
    M, N = A.shape
    sy, sx = divmod(s[0], pw)
    Z = np.zeros_like(A)
    for py in range(H // ph):
        for px in range(W // pw):
            for pt in range(N // bt):
                rows, cols = [], []
                for dy in range(ph):
                    for dx in range(pw):
                        y = (py * ph + dy + sy) % H
                        x = (px * pw + dx + sx) % W
                        rows.append(y * W + x)
                for dt in range(bt):
                    cols.append((pt * bt + dt + s[1]) % N)
                B = A[np.ix_(rows, cols)]
                U, S, Vt = np.linalg.svd(B, full_matrices=False)
                Z[np.ix_(rows, cols)] = (U * np.maximum(S - tau, 0)) @ Vt
    return Z


@pytest.mark.parametrize("s", [(0, 0), (4, 1), (5, 3), (1, 2)])
def test_spacetime_bsvt_matches_index_loops(s):
    rng = np.random.default_rng(12)
    H, W, N, ph, pw, bt = 4, 6, 6, 2, 3, 2
    A = rng.standard_normal((H * W, N))
    tau = 0.8
    got = O.scale_bsvt(A, ph * pw, bt, tau, s, geo=(W, pw))
    ref = _brute_spacetime(A, H, W, ph, pw, bt, tau, s)
    assert np.abs(got - ref).max() < 1e-12
    # not the contiguous partition of the same block size
    assert np.abs(got - O.cycle_spun_bsvt(A, ph * pw, bt, tau, s)).max() > 1e-3


def test_spacetime_reduces_to_contiguous_partitions():
    """A patch one image row wide is the contiguous W x bt partition (a shift along x
    only permutes inside the block); the whole image is the M x bt partition."""
    rng = np.random.default_rng(13)
    H, W, N = 6, 8, 12
    A = rng.standard_normal((H * W, N))
    for s in [(0, 0), (5, 2), (3, 7)]:
        row = O.scale_bsvt(A, W, 4, 1.1, s, geo=(W, W))
        assert np.abs(row - O.cycle_spun_bsvt(A, W, 4, 1.1, (0, s[1]))).max() < 1e-12
        full = O.scale_bsvt(A, H * W, 3, 1.1, (s[0] * W, s[1]), geo=(W, W))
        assert np.abs(full - O.cycle_spun_bsvt(A, H * W, 3, 1.1, (0, s[1]))).max() < 1e-12


def test_spacetime_full_spinning_is_video_shift_equivariant():
    rng = np.random.default_rng(14)
    H, W, N, ph, pw, bt = 4, 4, 4, 2, 2, 2
    V = rng.standard_normal((H * W, N))
    S = O.spin_shifts(0, 0, 0, ph * pw, bt, 1000, H * W, N)
    assert len(S) == ph * pw * bt
    T = lambda A: O.averaged_bsvt(A, ph * pw, bt, 0.7, S, geo=(W, pw))
    t = (3 * pw + 1, 1)          # video shift (3, 1, 1)
    assert np.abs(T(O.st_shift(V, W, pw, t)) - O.st_shift(T(V), W, pw, t)).max() < 1e-12
    one = lambda A: O.scale_bsvt(A, ph * pw, bt, 0.7, (0, 0), geo=(W, pw))
    assert np.abs(one(O.st_shift(V, W, pw, t)) - O.st_shift(one(V), W, pw, t)).max() > 1e-3


def test_admm_spacetime_kkt_and_gap():
    """ADMM with space-time scales (2 x 2 x 2, space-only 4 x 4 patches over all frames,
    and the whole video) reaches the KKT conditions of eq:cvx with their dual norms."""
    H = W = 8
    N = 8
    rng = np.random.default_rng(15)
    Y = 0.05 * rng.standard_normal((H * W, N))
    Y[:, :] += np.outer(rng.standard_normal(H * W), rng.standard_normal(N)) * 0.3
    Y[9, 3] += 2.0
    # a rank-1 space-only blob on the 4 x 4 patch at (4, 4)
    pix = [(4 + dy) * W + 4 + dx for dy in range(4) for dx in range(4)]
    Y[pix, :] += 0.8 * np.outer(rng.standard_normal(16), rng.standard_normal(N))
    ladder = [(1, 1), (4, 2), (16, N), (H * W, N)]
    kinds = [0, O.KIND_SPATIAL, O.KIND_SPATIAL, 0]
    pws = [1, 2, 4, 1]
    out = O.admm(Y, ladder, rho=2.0, iters=2000, kinds=kinds, image_w=W, patch_w=pws)
    rep = O.kkt_report(Y, ladder, out["lam"], 2.0, out["Z"], out["U"], kinds=kinds,
                       image_w=W, patch_w=pws)
    assert out["resid"] < 1e-7
    assert rep["consensus"] < 1e-7
    assert max(rep["dual_ratio"]) <= 1 + 1e-9
    assert abs(rep["gap"]) < 2e-7
    assert np.abs(out["Z"][2]).max() > 0.1          # the space-time scale carries the blob
