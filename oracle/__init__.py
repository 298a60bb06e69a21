"""FP64 CPU oracle for multi-scale low-rank decomposition.

TEST INFRASTRUCTURE ONLY. Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never touches it, and
this package never touches the product path: the two share no code, only the
seeded inputs of the ``synth`` module.

Everything here is float64, written step by step from the paper (Ong & Lustig,
"Beyond Low Rank + Sparse: Multi-scale Low Rank Matrix Decomposition"): plain numpy
for the iteration, and the oracle's own one-sided Jacobi SVD in plain C
(jacobi.c, compiled with gcc into libmsld_oracle.so on first use) inside singular
value thresholding. LAPACK (numpy.linalg.svd) appears only in the optimality
diagnostics (block nuclear and dual norms of kkt_report), which check results and
produce none.

Parity status per function (what independent facts pin it; see tests/):
  jacobi_svd          pinned: reconstruction to 1e-13 ||B||, orthonormal U and V,
                      singular values against LAPACK's, exact diagonal / rank-1 /
                      orthogonal-column cases, the transposed (m < n) route.
  cycle_shift         pinned: SplitMix64 published output for seed 0, and the
                      block-wise identities of the shifted operator.
  default_lambda      pinned: the special cases of the boxed lambda formula.
  svt                 pinned: prox optimality conditions (subdifferential of the
                      nuclear norm), brute-force 2x2 minimisation, rank-1 and
                      1xN / Nx1 closed forms.
  block_svt,          pinned: 1x1 soft-threshold and 1xN group closed forms,
  cycle_spun_bsvt     rank-1 planted blocks under wrapped shifts.
  admm                pinned: KKT conditions and a vanishing duality gap at
                      convergence, scaling / transpose invariances, trivial
                      ladders, ground-truth recovery on sparse instances.
  noise_svt,          pinned: prox optimality of the Frobenius norm (zero inside
  scale_lambda        the ball, the subgradient condition outside), the lambda
                      special case of the MN x 1 block, and the noisy program's
                      KKT conditions / duality gap through admm(kinds=...).
  admm(mask=...)      pinned: a full mask is the plain iteration; one masked
                      full-size scale recovers a low-rank matrix from 60% of its
                      entries (nuclear-norm completion); KKT with the dual
                      certificate supported on the observed entries.
  spin_shifts,        pinned: averaging over every shift makes the Z-step exactly
  spin_extent,        translation equivariant (it is not for a single shift), also
  averaged_bsvt       with the reduced set of a block that spans an axis; a shift
                      along such an axis leaves the shifted BlockSVT unchanged; one
                      hashed shift is the random cycle spinning of the plain
                      iteration; tau = 0 gives the input back (the 1/|S| factor);
                      the average of proxes stays non-expansive.
  st_shift,           pinned: brute-force index loops over the video (patch pixels
  spacetime_bsvt,     with wrap in y, x, t) give the same thresholded blocks; a patch
  scale_bsvt          one image row wide equals the contiguous W x bt partition; the
                      whole image equals the contiguous M x bt partition; equivariance
                      under video shifts after averaging over every shift; ADMM with
                      space-time scales reaches the KKT conditions of eq:cvx.
"""
from .msld_oracle import (  # noqa: F401
    MASK64, splitmix64_mix, jacobi_svd, build_jacobi, cycle_shift, default_lambda, shift, unshift, svt,
    block_svt, cycle_spun_bsvt, admm, block_nuclear_norm, block_dual_norm,
    kkt_report, skip_bound_sq, KIND_BLOCK, KIND_NOISE, noise_svt, scale_lambda,
    scale_norm, scale_dual_norm, spin_shifts, spin_extent, averaged_bsvt,
    KIND_SPATIAL, st_shift, st_unshift, spacetime_bsvt, scale_bsvt,
)
