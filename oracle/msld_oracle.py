"""Plain FP64 reference for the ADMM / block-wise SVT iteration (test infrastructure).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may use this
module. Each function cites the passage of the paper it follows. Notation follows
the paper: Y is M x N, scale i has m_i x n_i blocks, lambda_i its weight, rho the
ADMM parameter, X_i / Z_i / U_i the ADMM variables.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15          # SplitMix64 increment (Steele, Lea & Flood 2014)


# --------------------------------------------------------------------------- shifts
def splitmix64_mix(z: int) -> int:
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014; the
    'variant 13' 64-bit finaliser). Pure 64-bit integer arithmetic."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def cycle_shift(seed: int, k: int, i: int, m: int, n: int):
    """Random cycle-spin shift s = (s_r, s_c) of scale i at iteration k
    (Sec. 9, random cycle spinning: one random shift per Z-update).

    The paper does not say how shifts are drawn. Reading used here: shifts are
    residues modulo the block size (a shift by a whole block gives the same
    partition); one independent draw per (k, i), both 0-based, i < 16, from the
    counter-based SplitMix64 value z = mix(seed + gamma * (16 k + i + 1)) mod 2^64;
    s_r = (z >> 32) mod m, s_c = (z & 0xffffffff) mod n.
    """
    x = (int(seed) + _GAMMA * (16 * int(k) + int(i) + 1)) & MASK64
    z = splitmix64_mix(x)
    return (z >> 32) % int(m), (z & 0xFFFFFFFF) % int(n)


def shift(A: np.ndarray, s):
    """Shift_s of Sec. 9 with cyclic wrap: Shift_s(A)[r, c] = A[(r+s_r) mod M, (c+s_c) mod N]."""
    return np.roll(A, (-int(s[0]), -int(s[1])), axis=(0, 1))


def unshift(A: np.ndarray, s):
    """Shift_{-s}, the inverse of `shift`."""
    return np.roll(A, (int(s[0]), int(s[1])), axis=(0, 1))


# ------------------------------------------------------------------- regularisation
def default_lambda(M: int, N: int, m: int, n: int) -> float:
    """Boxed regularisation rule of Sec. 4 (eq:lambda), with constant 1 as in the
    experiments of Sec. 10 and the natural logarithm:
    lambda_i = sqrt(m_i) + sqrt(n_i) + sqrt(log(MN / max(m_i, n_i)))."""
    return math.sqrt(m) + math.sqrt(n) + math.sqrt(math.log(M * N / max(m, n)))


# ------------------------------------------------------------------- Jacobi SVD
_HERE = os.path.dirname(os.path.abspath(__file__))
_JACOBI_SRC = os.path.join(_HERE, "jacobi.c")
_JACOBI_LIB = os.path.join(_HERE, "libmsld_oracle.so")
_jacobi = None


def build_jacobi(force: bool = False) -> str:
    """Compile jacobi.c (plain C, float64, OpenMP) into libmsld_oracle.so next to it."""
    stale = (not os.path.exists(_JACOBI_LIB) or
             os.path.getmtime(_JACOBI_LIB) < os.path.getmtime(_JACOBI_SRC))
    if force or stale:
        tmp = _JACOBI_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        _JACOBI_SRC, "-lm", "-o", tmp], check=True)
        os.replace(tmp, _JACOBI_LIB)
    return _JACOBI_LIB


def _jacobi_lib():
    global _jacobi
    if _jacobi is None:
        lib = ctypes.CDLL(build_jacobi())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.msld_oracle_jacobi_svd.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp,
                                               dp, dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        lib.msld_oracle_jacobi_svd.restype = ctypes.c_int
        _jacobi = lib
    return _jacobi


def jacobi_svd(B: np.ndarray, max_sweeps: int = 100, return_sweeps: bool = False):
    """Thin SVD B = U diag(s) V^T by one-sided (Hestenes) Jacobi in float64 (jacobi.c):
    column pairs are rotated, round-robin order, until every pair is orthogonal to
    working precision; s_j = ||B v_j||. Works on (m, n) or a stack (..., m, n); a block
    with m < n goes through its transpose. Singular values come back in descending
    order; a zero singular value has a zero left vector. Raises if a block has not
    converged after max_sweeps sweeps."""
    B = np.asarray(B, dtype=np.float64)
    *lead, m, n = B.shape
    flip = m < n
    A = np.swapaxes(B, -1, -2) if flip else B
    mm, nn = (n, m) if flip else (m, n)
    A = np.ascontiguousarray(A.reshape(-1, mm, nn))
    nb = A.shape[0]
    U = np.empty((nb, mm, nn))
    s = np.empty((nb, nn))
    V = np.empty((nb, nn, nn))
    sw = np.zeros(nb, dtype=np.int32)
    if nb:
        dp = ctypes.POINTER(ctypes.c_double)
        rc = _jacobi_lib().msld_oracle_jacobi_svd(
            nb, mm, nn, A.ctypes.data_as(dp), U.ctypes.data_as(dp), s.ctypes.data_as(dp),
            V.ctypes.data_as(dp), sw.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
            int(max_sweeps))
        if rc < 0:
            raise RuntimeError("jacobi_svd: a block did not converge in %d sweeps" % max_sweeps)
    order = np.argsort(-s, axis=-1, kind="stable")
    s = np.take_along_axis(s, order, axis=-1)
    U = np.take_along_axis(U, order[:, None, :], axis=-1)
    V = np.take_along_axis(V, order[:, None, :], axis=-1)
    if flip:
        U, V = V, U
    k = min(m, n)
    U = U.reshape(*lead, m, k)
    V = V.reshape(*lead, n, k)
    s = s.reshape(*lead, k)
    if return_sweeps:
        return U, s, V, sw.reshape(lead)
    return U, s, V


# --------------------------------------------------------------------------- SVT
def svt(B: np.ndarray, tau: float) -> np.ndarray:
    """Singular value soft-threshold of Sec. 7 (eq:svt): U max(Sigma - tau, 0) V^T, with
    the singular triplets from the oracle's own Jacobi SVD. Works on a single matrix
    (m, n) or a stack (..., m, n)."""
    U, S, V = jacobi_svd(B)
    S = np.maximum(S - tau, 0.0)
    return np.matmul(U * S[..., None, :], np.swapaxes(V, -1, -2))


def _blocks(A: np.ndarray, m: int, n: int) -> np.ndarray:
    """All R_b(A) of the contiguous m x n partition (Sec. 2, block reshape operator),
    stacked as (M/m, N/n, m, n); block (p, q) is A[p m:(p+1) m, q n:(q+1) n]."""
    M, N = A.shape
    return A.reshape(M // m, m, N // n, n).transpose(0, 2, 1, 3)


def _unblocks(Bk: np.ndarray) -> np.ndarray:
    """sum_b R_b^T(B_b): embed every block back at its place (adjoint of R_b)."""
    P, Q, m, n = Bk.shape
    return Bk.transpose(0, 2, 1, 3).reshape(P * m, Q * n)


def block_svt(A: np.ndarray, m: int, n: int, tau: float) -> np.ndarray:
    """Block-wise SVT of Sec. 7 (eq:bsvt): sum_b R_b^T(SVT_tau(R_b(A))) over the
    contiguous m x n partition. Blocks are disjoint, so the sum is a placement."""
    M, N = A.shape
    if M % m or N % n:
        raise ValueError("block size must tile the matrix")
    Bk = _blocks(np.asarray(A, dtype=np.float64), m, n)
    P, Q = Bk.shape[:2]
    Zk = svt(Bk.reshape(P * Q, m, n), tau).reshape(P, Q, m, n)
    return _unblocks(Zk)


def cycle_spun_bsvt(A: np.ndarray, m: int, n: int, tau: float, s) -> np.ndarray:
    """Random cycle spinning of Sec. 9: Shift_{-s}(BSVT_tau(Shift_s(A)))."""
    return unshift(block_svt(shift(A, s), m, n, tau), s)


def spin_extent(M: int, N: int, m: int, n: int):
    """Distinct shifts per axis for cycle spinning of an m x n partition of an M x N
    matrix. A cyclic shift along an axis the block spans whole (m = M or n = N) only
    permutes rows or columns inside each block, which the block's SVT follows exactly,
    so that axis contributes a single shift (reading of Sec. 9)."""
    return (1 if m == M else m), (1 if n == N else n)


def spin_shifts(seed: int, k: int, i: int, m: int, n: int, count: int, M=None, N=None):
    """The shift set S of iteration k, scale i for averaged cycle spinning (Sec. 9).
    With count >= mr nc (mr x nc = spin_extent) it is every shift (s_r, s_c) in
    [0, mr) x [0, nc), in row-major order; otherwise `count` draws of the shift hash
    with seeds seed + j."""
    mr, nc = spin_extent(M if M is not None else -1, N if N is not None else -1, m, n)
    if count >= mr * nc:
        return [(r, c) for r in range(mr) for c in range(nc)]
    return [cycle_shift(seed + j, k, i, m, n) for j in range(count)]


def averaged_bsvt(A: np.ndarray, m: int, n: int, tau: float, shifts, geo=None) -> np.ndarray:
    """Cycle spinning of Sec. 9 as an average over a shift set S:
    (1/|S|) sum_{s in S} Shift_{-s}(BSVT_tau(Shift_s(A))) (geo: see scale_bsvt)."""
    acc = np.zeros(np.shape(A))
    for s in shifts:
        acc += scale_bsvt(A, m, n, tau, s, geo)
    return acc / len(shifts)


# ------------------------------------------------------------------ noise scale
# Sec. 2 (multi-scale low rank + noise): the noise matrix is one more scale whose
# reshape R_Z takes the whole M x N matrix to an MN x 1 vector; the block-wise nuclear
# norm of that scale is then the Frobenius norm (Sec. 3, remark after eq:cvx).
KIND_BLOCK = 0       # block-wise nuclear norm over an m_i x n_i partition
KIND_NOISE = 1       # nuclear norm of the MN x 1 reshape (Frobenius norm)


def noise_svt(A: np.ndarray, tau: float) -> np.ndarray:
    """SVT of eq:svt applied to the MN x 1 reshape R_Z(A), placed back by R_Z^T."""
    A = np.asarray(A, dtype=np.float64)
    return svt(A.reshape(-1, 1), tau).reshape(A.shape)


# -------------------------------------------------------------- space-time blocks
# Sec. 2 (general block reshape R_b) and the video / DCE experiments of Sec. 10: the
# rows of Y are the pixels of an H x W image in row-major order (row y W + x) and the
# columns are frames. A space-time block is a ph x pw pixel patch over bt consecutive
# frames, reshaped to a (ph pw) x bt matrix (row dy pw + dx of the block is pixel
# (y0 + dy, x0 + dx)); a patch spanning every frame (bt = N) is the space-only
# decimation of the face experiment. Shift_s is the cyclic shift of the video in
# (y, x, t).
KIND_SPATIAL = 2     # block-wise nuclear norm over the space-time partition


def st_shift(A: np.ndarray, W: int, pw: int, s):
    """Shift_s of Sec. 9 on the video: V[y, x, t] <- V[(y+sy) mod H, (x+sx) mod W,
    (t+st) mod N]. Reading: the patch shift (sy, sx) is drawn as one residue
    s_r mod (ph pw) with sy = s_r div pw, sx = s_r mod pw; st = s_c."""
    M, N = A.shape
    sy, sx = divmod(int(s[0]), pw)
    V = np.asarray(A).reshape(M // W, W, N)
    return np.roll(V, (-sy, -sx, -int(s[1])), axis=(0, 1, 2)).reshape(M, N)


def st_unshift(A: np.ndarray, W: int, pw: int, s):
    """Shift_{-s}, the inverse of `st_shift`."""
    M, N = A.shape
    sy, sx = divmod(int(s[0]), pw)
    V = np.asarray(A).reshape(M // W, W, N)
    return np.roll(V, (sy, sx, int(s[1])), axis=(0, 1, 2)).reshape(M, N)


def _st_blocks(A: np.ndarray, W: int, ph: int, pw: int, bt: int) -> np.ndarray:
    """All R_b(A) of the space-time partition, stacked as (nblocks, ph pw, bt)."""
    M, N = A.shape
    H = M // W
    if H * W != M or H % ph or W % pw or N % bt:
        raise ValueError("patch and frame block must tile the video")
    T = np.asarray(A, dtype=np.float64).reshape(H // ph, ph, W // pw, pw, N // bt, bt)
    return T.transpose(0, 2, 4, 1, 3, 5).reshape(-1, ph * pw, bt)


def _st_unblocks(Bk: np.ndarray, M: int, N: int, W: int, ph: int, pw: int, bt: int):
    """sum_b R_b^T(B_b) for the space-time partition (adjoint of `_st_blocks`)."""
    H = M // W
    T = Bk.reshape(H // ph, W // pw, N // bt, ph, pw, bt).transpose(0, 3, 1, 4, 2, 5)
    return T.reshape(M, N)


def spacetime_bsvt(A: np.ndarray, W: int, ph: int, pw: int, bt: int, tau: float):
    """eq:bsvt over the space-time partition: every (ph pw) x bt block thresholded."""
    M, N = A.shape
    Bk = _st_blocks(A, W, ph, pw, bt)
    return _st_unblocks(svt(Bk, tau), M, N, W, ph, pw, bt)


def scale_bsvt(A: np.ndarray, m: int, n: int, tau: float, s, geo=None) -> np.ndarray:
    """Shift_{-s}(BSVT_tau(Shift_s(A))) of one scale: the contiguous m x n partition
    (geo None) or the space-time partition geo = (W, pw) with ph = m / pw, bt = n."""
    if geo is None:
        return cycle_spun_bsvt(A, m, n, tau, s)
    W, pw = geo
    return st_unshift(spacetime_bsvt(st_shift(A, W, pw, s), W, m // pw, pw, n, tau), W, pw, s)


def scale_lambda(M: int, N: int, m: int, n: int, kind: int = KIND_BLOCK) -> float:
    """eq:lambda for scale i; the noise scale's block is MN x 1 (Sec. 4 notes its
    lambda ~ sqrt(MN))."""
    if kind == KIND_NOISE:
        return default_lambda(M, N, M * N, 1)
    return default_lambda(M, N, m, n)


# --------------------------------------------------------------------------- ADMM
def admm(Y, ladder, lam=None, rho=1.0, iters=100, cycle_spin=False, seed=0,
         tol=0.0, check_every=1, history=False, kinds=None, mask=None, spin_count=1,
         image_w=None, patch_w=None):
    """ADMM of Sec. 7 (eq:admm) for eq:cvx, with the random cycle spinning of Sec. 9.

    Per iteration k, in the paper's order:
        X_i <- (Z_i - U_i) + (Y - sum_j (Z_j - U_j)) / L
        Z_i <- Shift_{-s}(BSVT_{lambda_i/rho}(Shift_s(X_i + U_i)))   (s = 0 without spinning)
        U_i <- U_i - (Z_i - X_i)
    kinds[i] == KIND_NOISE makes scale i the noise scale of Sec. 2 (its Z-step is the
    SVT of the MN x 1 reshape, which no shift changes; its block size must be M x N).
    spin_count > 1 (with cycle_spin) averages each block scale's Z-step over the shift
    set spin_shifts(seed, k, i, m, n, spin_count, M, N) of Sec. 9 (every distinct shift
    when spin_count covers them); scales with a single distinct shift (1 x 1, the
    whole matrix) and noise scales keep the plain iteration.
    kinds[i] == KIND_SPATIAL makes scale i a space-time partition (rows = pixels of an
    image of width image_w, ladder entry (ph pw, bt), patch width patch_w[i]).
    mask (M x N, true = observed) applies the data consistency of the collaborative
    filtering experiment of Sec. 10: the X-update above only on observed entries,
    X_i = Z_i - U_i on the others; the residual is then relative to ||P_obs(Y)||_F.
    Readings where the paper is silent: Z_i = U_i = 0 at start; the returned
    components are Z_i (exactly block-low-rank); primal residual
    r_k = sqrt(sum_i ||X_i - Z_i||_F^2) / ||Y||_F with the new Z_i; when tol > 0 the
    loop stops after iteration k if (k+1) % check_every == 0 and r_k <= tol. The dual
    residual rho ||Z^k - Z^(k-1)||_F / ||Y||_F of the last iteration is reported only.
    """
    Y = np.asarray(Y, dtype=np.float64)
    M, N = Y.shape
    ladder = [(int(m), int(n)) for (m, n) in ladder]
    L = len(ladder)
    kinds = [KIND_BLOCK] * L if kinds is None else [int(x) for x in kinds]
    if lam is None:
        lam = [scale_lambda(M, N, m, n, kinds[i]) for i, (m, n) in enumerate(ladder)]
    lam = [float(x) for x in lam]
    Z = np.zeros((L, M, N))
    U = np.zeros((L, M, N))
    X = np.zeros((L, M, N))
    obs = None if mask is None else np.asarray(mask, dtype=bool)
    if obs is not None:
        Y = np.where(obs, Y, 0.0)          # unobserved entries carry no data
    ny = np.linalg.norm(Y)
    ny = ny if ny > 0 else 1.0
    hist = []
    r = float("nan")
    dual = float("nan")
    k_done = 0
    geos = [(int(image_w), int(patch_w[i])) if kinds[i] == KIND_SPATIAL else None
            for i in range(L)]
    for k in range(int(iters)):
        Zprev = Z.copy()
        S = (Z - U).sum(axis=0)
        for i in range(L):
            if obs is None:
                X[i] = (Z[i] - U[i]) + (Y - S) / L
            else:
                X[i] = np.where(obs, (Z[i] - U[i]) + (Y - S) / L, Z[i] - U[i])
        for i, (m, n) in enumerate(ladder):
            if kinds[i] == KIND_NOISE:
                Z[i] = noise_svt(X[i] + U[i], lam[i] / rho)
                continue
            mr, nc = spin_extent(M, N, m, n)
            if cycle_spin and spin_count > 1 and mr * nc > 1:
                S = spin_shifts(seed, k, i, m, n, int(spin_count), M, N)
                Z[i] = averaged_bsvt(X[i] + U[i], m, n, lam[i] / rho, S, geos[i])
                continue
            s = cycle_shift(seed, k, i, m, n) if cycle_spin else (0, 0)
            Z[i] = scale_bsvt(X[i] + U[i], m, n, lam[i] / rho, s, geos[i])
        U = U - (Z - X)
        r = float(np.sqrt(((X - Z) ** 2).sum()) / ny)
        dual = float(rho * np.sqrt(((Z - Zprev) ** 2).sum()) / ny)
        k_done = k + 1
        if history:
            hist.append(r)
        if tol > 0 and k_done % int(check_every) == 0 and r <= tol:
            break
    return {"Z": Z, "X": X, "U": U, "iters": k_done, "resid": r, "dual": dual,
            "history": hist, "lam": lam}


# --------------------------------------------------------------------- diagnostics
def block_nuclear_norm(A, m, n) -> float:
    """||A||_(i) of Sec. 3: sum over blocks of the nuclear norm of R_b(A)."""
    Bk = _blocks(np.asarray(A, dtype=np.float64), m, n)
    P, Q = Bk.shape[:2]
    return float(np.linalg.svd(Bk.reshape(P * Q, m, n), compute_uv=False).sum())


def block_dual_norm(A, m, n) -> float:
    """||A||*_(i) of Sec. 3: max over blocks of the largest singular value of R_b(A)."""
    Bk = _blocks(np.asarray(A, dtype=np.float64), m, n)
    P, Q = Bk.shape[:2]
    return float(np.linalg.svd(Bk.reshape(P * Q, m, n), compute_uv=False).max())


def scale_norm(A, m, n, kind=KIND_BLOCK, geo=None) -> float:
    """The norm of scale i in eq:cvx (Frobenius for the noise scale; geo = (W, pw)
    for a space-time scale)."""
    if kind == KIND_NOISE:
        return float(np.linalg.norm(A))
    if geo is not None:
        Bk = _st_blocks(A, geo[0], m // geo[1], geo[1], n)
        return float(np.linalg.svd(Bk, compute_uv=False).sum())
    return block_nuclear_norm(A, m, n)


def scale_dual_norm(A, m, n, kind=KIND_BLOCK, geo=None) -> float:
    """Its dual norm (Sec. 3); the Frobenius norm is self-dual."""
    if kind == KIND_NOISE:
        return float(np.linalg.norm(A))
    if geo is not None:
        Bk = _st_blocks(A, geo[0], m // geo[1], geo[1], n)
        return float(np.linalg.svd(Bk, compute_uv=False).max())
    return block_dual_norm(A, m, n)


def kkt_report(Y, ladder, lam, rho, Z, U, kinds=None, mask=None, image_w=None, patch_w=None):
    """Optimality diagnostics for eq:cvx from an ADMM state (no cycle spinning).

    Dual certificate: at a fixed point all U_i coincide and Q = rho * mean_i U_i
    satisfies Q in lambda_i * subdifferential of ||Z_i||_(i) (the condition of
    Thm A.3 with the dual norm of Sec. 3). For any Q with ||Q||*_(i) <= lambda_i,
    <Q, Y> lower-bounds the optimum (weak duality), so Q is scaled into that set.
    The primal value is taken at the feasible point Z_i + (Y - sum_j Z_j)/L. With a
    mask the constraint holds on observed entries only: Q must vanish elsewhere
    ("off_support") and the feasible point corrects observed entries only.
    """
    Y = np.asarray(Y, dtype=np.float64)
    L = len(ladder)
    kinds = [KIND_BLOCK] * L if kinds is None else list(kinds)
    geos = [(int(image_w), int(patch_w[i])) if kinds[i] == KIND_SPATIAL else None
            for i in range(L)]
    obs = np.ones(Y.shape, dtype=bool) if mask is None else np.asarray(mask, dtype=bool)
    Y = np.where(obs, Y, 0.0)
    Ubar = np.mean(U, axis=0)
    Q = rho * Ubar
    ratios = [scale_dual_norm(Q, m, n, kinds[i], geos[i]) / lam[i]
              for i, (m, n) in enumerate(ladder)]
    Qs = Q / max(1.0, max(ratios))
    dual = float((Qs * Y).sum())
    Zf = Z + np.where(obs, Y - Z.sum(axis=0), 0.0) / L
    primal = float(sum(lam[i] * scale_norm(Zf[i], m, n, kinds[i], geos[i])
                       for i, (m, n) in enumerate(ladder)))
    spread = float(max(np.linalg.norm(U[i] - Ubar) for i in range(L)) /
                   max(np.linalg.norm(Ubar), 1e-300))
    return {"primal": primal, "dual": dual,
            "gap": (primal - dual) / max(abs(primal), 1e-300),
            "dual_ratio": ratios, "u_spread": spread,
            "consensus": float(np.linalg.norm(np.where(obs, Y - Z.sum(axis=0), 0.0)) /
                               max(np.linalg.norm(Y), 1e-300)),
            "off_support": float(np.abs(np.where(obs, 0.0, Q)).max(initial=0.0))}


def skip_bound_sq(B) -> float:
    """Square of the upper bound on the largest singular value used to skip SVDs
    (Sec. 8). The printed formula has an unbound index; reading used here:
    sigma_max(B)^2 <= max_r sum_k |B_rk| (sum_j |B_jk|), the maximum row sum of
    |B||B|^T, which bounds the spectral radius of B B^T."""
    A = np.abs(np.asarray(B, dtype=np.float64))
    return float((A @ A.sum(axis=0)).max())
