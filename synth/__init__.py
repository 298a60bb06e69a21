"""Seeded synthetic inputs for multi-scale low-rank decomposition.

This module is shared by the tests, the benchmark and the oracle harness. It holds
only random draws and the signal model (Sec. 2: Y is a sum of block-wise low-rank
components plus optional Gaussian noise); it contains none of the solver's
arithmetic (no thresholding, no ADMM, no regularisation defaults).

Recipe (one definition used everywhere):
  * rng = numpy.random.default_rng(seed) (PCG64).
  * For each scale i in ladder order, with block size m_i x n_i and
    P_i = (M/m_i)(N/n_i) contiguous blocks in row-major block order:
      k_i = max(1, round(density * P_i)) distinct block ids drawn by
      rng.choice(P_i, k_i, replace=False), then sorted;
      per rank r: u ~ N(0,1)^{k_i x m_i x r}, v ~ N(0,1)^{k_i x n_i x r} (drawn in
      that order); block = u @ v^T.
  * noise: sigma * N(0,1)^{M x N}, drawn last, added after the components.
  * Y = float32(sum of components + noise); components are returned in fp64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = ["Instance", "make_instance", "full_ladder", "geometric_ladder",
           "batch_instances", "serving_trace"]


@dataclass
class Instance:
    Y: np.ndarray                     # (M, N) float32
    ladder: list                      # [(m_i, n_i)]
    components: np.ndarray | None     # (L, M, N) float64 ground truth, or None
    active: list = field(default_factory=list)   # per scale: sorted active block ids
    seed: int = 0
    density: float = 0.0
    rank: int = 1
    noise: float = 0.0

    @property
    def shape(self):
        return self.Y.shape


def _check_ladder(M, N, ladder):
    for (m, n) in ladder:
        if m <= 0 or n <= 0 or M % m or N % n:
            raise ValueError(f"block {m}x{n} does not tile {M}x{N}")


def make_instance(M, N, ladder, density, rank=1, noise=0.0, seed=0,
                  keep_components=True, ranks=None) -> Instance:
    """Draw Y = sum_i X_i + noise following the module recipe.

    `ranks` (optional, per scale) overrides `rank` scale by scale.
    `keep_components=False` skips storing the (L, M, N) fp64 ground truth, which
    matters for 8192 x 8192 inputs.
    """
    ladder = [(int(m), int(n)) for (m, n) in ladder]
    _check_ladder(M, N, ladder)
    rng = np.random.default_rng(seed)
    L = len(ladder)
    acc = np.zeros((M, N), dtype=np.float64)
    comps = np.zeros((L, M, N), dtype=np.float64) if keep_components else None
    active = []
    for i, (m, n) in enumerate(ladder):
        r = int(ranks[i]) if ranks is not None else int(rank)
        P, Q = M // m, N // n
        nb = P * Q
        k = max(1, int(round(density * nb)))
        ids = np.sort(rng.choice(nb, size=k, replace=False))
        u = rng.standard_normal((k, m, r))
        v = rng.standard_normal((k, n, r))
        blocks = np.matmul(u, np.transpose(v, (0, 2, 1)))      # (k, m, n)
        tgt = acc if comps is None else comps[i]
        view = tgt.reshape(P, m, Q, n)                          # view, no copy
        p, q = ids // Q, ids % Q
        view[p, :, q, :] += blocks
        if comps is not None:
            acc += comps[i]
        active.append(ids)
    if noise > 0:
        acc += noise * rng.standard_normal((M, N))
    Y = acc.astype(np.float32)
    return Instance(Y=Y, ladder=ladder, components=comps, active=active,
                    seed=seed, density=density, rank=rank, noise=noise)


def full_ladder(M, N, small):
    """Ladder of square blocks `small` followed by the full M x N block."""
    return [(b, b) for b in small] + [(M, N)]


def geometric_ladder(M, N, L):
    """Ratio-4 ladder 1, 4, 16, ... of L-1 square scales, then the full block."""
    out = []
    b = 1
    for _ in range(L - 1):
        out.append((b, b))
        b *= 4
    out.append((M, N))
    _check_ladder(M, N, out)
    return out


def batch_instances(count, seed=0, density=0.02, noise=0.01):
    """Independent instances of mixed sizes and ladders (one batched launch).

    Shapes are drawn uniformly from {64^2, 128^2, 256^2, 128x512}; ladders from
    {1,4,16,full} and {1,8,32,full}; rank-1 block ground truth.
    Instance j uses data seed (seed * 1_000_003 + j).
    """
    shapes = [(64, 64), (128, 128), (256, 256), (128, 512)]
    smalls = [(1, 4, 16), (1, 8, 32)]
    rng = np.random.default_rng(seed)
    si = rng.integers(0, len(shapes), size=count)
    li = rng.integers(0, len(smalls), size=count)
    out = []
    for j in range(count):
        M, N = shapes[si[j]]
        lad = full_ladder(M, N, smalls[li[j]])
        out.append(make_instance(M, N, lad, density, rank=1, noise=noise,
                                 seed=seed * 1_000_003 + j, keep_components=False))
    return out


def serving_trace(count, rate, seed=0, density=0.02, noise=0.01):
    """Poisson arrival trace of decomposition requests.

    Returns a list of (arrival_time_s, M, N, ladder, rank, data_seed). Shapes are
    uniform over {128^2, 512^2, 1024x256, 2048^2}; L uniform over {4, 5, 6} with a
    ratio-4 ladder ending in the full block (truncated where a block would not
    tile the matrix); rank 1 or 2 with equal probability.
    """
    shapes = [(128, 128), (512, 512), (1024, 256), (2048, 2048)]
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(count):
        t += rng.exponential(1.0 / rate)
        M, N = shapes[rng.integers(0, len(shapes))]
        L = int(rng.integers(4, 7))
        lad = []
        b = 1
        while len(lad) < L - 1 and b <= min(M, N) // 4 and M % b == 0 and N % b == 0:
            lad.append((b, b))
            b *= 4
        lad.append((M, N))
        rank = int(rng.integers(1, 3))
        out.append((t, M, N, lad, rank, seed * 1_000_003 + j))
    return out


def completion_instance(M=1682, N=943, groups=23, observed=0.063, seed=0, noise=0.3):
    """Stand-in for a ratings matrix (items x users, users grouped along the columns):
    a global rank-2 term, one rank-1 term per user group of N / groups columns, noise,
    and a uniformly random set of observed entries (fraction `observed`).

    Returns (Y float32 with unobserved entries set to 0, mask bool, truth float64)."""
    if N % groups:
        raise ValueError("groups must divide N")
    rng = np.random.default_rng(seed)
    T = rng.standard_normal((M, 2)) @ rng.standard_normal((2, N))
    w = N // groups
    for g in range(groups):
        T[:, g * w:(g + 1) * w] += np.outer(rng.standard_normal(M), rng.standard_normal(w))
    Y = T + noise * rng.standard_normal((M, N))
    mask = rng.random((M, N)) < observed
    return np.where(mask, Y, 0.0).astype(np.float32), mask, T


def video_instance(H=144, W=176, T=192, objects=6, radius=6.0, seed=0, noise=0.01):
    """Stand-in for a surveillance video as a (H W) x T matrix (pixel y W + x per row,
    one frame per column): a static background image whose brightness drifts slowly
    (rank 1), `objects` Gaussian blobs of the given radius moving on straight lines
    with wrap (local in space and time), and noise.

    Returns Y as float32."""
    rng = np.random.default_rng(seed)
    bg = 0.5 + 0.5 * rng.random((H, W))
    t = np.arange(T)
    gain = 1.0 + 0.1 * np.sin(2 * np.pi * t / T)
    V = bg[:, :, None] * gain[None, None, :]
    yy, xx = np.mgrid[0:H, 0:W]
    for _ in range(objects):
        y0, x0 = rng.random() * H, rng.random() * W
        vy, vx = rng.uniform(-1.0, 1.0, size=2)
        amp = rng.uniform(0.3, 0.8)
        for f in range(T):
            cy, cx = (y0 + vy * f) % H, (x0 + vx * f) % W
            dy = np.minimum(np.abs(yy - cy), H - np.abs(yy - cy))
            dx = np.minimum(np.abs(xx - cx), W - np.abs(xx - cx))
            V[:, :, f] += amp * np.exp(-(dy ** 2 + dx ** 2) / (2 * radius ** 2))
    Y = V.reshape(H * W, T) + noise * rng.standard_normal((H * W, T))
    return Y.astype(np.float32)


def spacetime_instance(H, W, T, blobs, rank=2, spikes=0.001, noise=0.01, seed=0):
    """Stand-in for an image series as a (H W) x T matrix (pixel y W + x per row, one
    frame or lighting condition per column): a global rank-`rank` term with positive
    factors, rank-1 space-time blobs (`blobs` = list of (ph, pw, bt, count, amp): `count`
    blobs on random ph x pw pixel patches over bt consecutive columns, not aligned to any
    grid), sparse spikes at a fraction `spikes` of the entries, and noise. Used for the
    face illumination (space-only blobs, bt = T) and DCE (contrast curves over time)
    workloads of the paper, whose data are not available.

    Returns Y as float32."""
    rng = np.random.default_rng(seed)
    M = H * W
    Y = (rng.random((M, rank)) + 0.5) @ (rng.random((rank, T)) + 0.5) / rank
    for (ph, pw, bt, count, amp) in blobs:
        for _ in range(count):
            y0, x0 = int(rng.integers(0, H - ph + 1)), int(rng.integers(0, W - pw + 1))
            t0 = int(rng.integers(0, T - bt + 1))
            pix = [(y0 + dy) * W + x0 + dx for dy in range(ph) for dx in range(pw)]
            Y[np.ix_(pix, range(t0, t0 + bt))] += amp * np.outer(rng.standard_normal(ph * pw),
                                                                rng.standard_normal(bt))
    k = int(spikes * M * T)
    if k:
        Y.flat[rng.choice(M * T, k, replace=False)] += rng.choice([-3.0, 3.0], k)
    Y += noise * rng.standard_normal((M, T))
    return Y.astype(np.float32)


def lcm_blocks(ladder):
    a, b = 1, 1
    for (m, n) in ladder:
        a = a * m // math.gcd(a, m)
        b = b * n // math.gcd(b, n)
    return a, b
