"""The allocation-free BlockSVT entry point (msld_bsvt_noalloc) against the handle-based
one (msld_bsvt on a handle without the low-rank paths) through the C ABI: bitwise the
same on two calls in a row, the second smaller; and against the oracle's SVT."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _field(M, N, m, n, seed):
    """Blocks of low rank and various sizes plus small noise, so that the bound test
    keeps some blocks and skips others."""
    rng = np.random.default_rng(seed)
    V = 0.05 * rng.standard_normal((M, N))
    for _ in range(max(1, (M // m) * (N // n) // 4)):
        r, c = rng.integers(0, M - m + 1), rng.integers(0, N - n + 1)
        V[r:r + m, c:c + n] += rng.uniform(0.2, 3.0) * np.outer(rng.standard_normal(m),
                                                                 rng.standard_normal(n))
    return V.astype(np.float32)


@pytest.mark.parametrize("cases", [
    # register tier: 8 x 8 blocks, then a smaller matrix
    [(512, 384, 8, 8, (3, 5), 1.3, 1), (128, 64, 8, 8, (7, 2), 0.9, 2)],
    # LDS tier: 32 x 32 and 16 x 64 blocks, then smaller
    [(256, 256, 32, 32, (11, 30), 2.5, 3), (64, 128, 16, 64, (5, 63), 1.7, 4)],
])
def test_noalloc_equals_bsvt_twice(lib, cases):
    for (M, N, m, n, shift, tau, seed) in cases:
        print(f"noalloc bsvt {M}x{N} blocks {m}x{n} shift {shift} tau {tau}", flush=True)
        V = _field(M, N, m, n, seed)
        Vd = torch.from_numpy(V).cuda()
        ref = lib.bsvt(Vd, m, n, tau, shift, lowrank_min=-1)
        out = lib.bsvt_noalloc(Vd, m, n, tau, shift)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        # and the oracle's SVT of the shifted partition (relative Frobenius <= 1e-4)
        Zo = O.cycle_spun_bsvt(V.astype(np.float64), m, n, tau, shift)
        err = np.linalg.norm(out.double().cpu().numpy() - Zo) / max(np.linalg.norm(Zo),
                                                                    1e-3 * np.linalg.norm(V))
        print(f"  equal to msld_bsvt; oracle rel err {err:.2e}; nonzero "
              f"{int((out != 0).sum())} of {M * N}", flush=True)
        assert err <= 1e-4
        assert (out != 0).any() and (out == 0).any()


def test_noalloc_in_place_and_limits(lib):
    V = _field(128, 128, 16, 16, 9)
    Vd = torch.from_numpy(V).cuda()
    ref = lib.bsvt(Vd, 16, 16, 1.1, (2, 3), lowrank_min=-1)
    inplace = Vd.clone()
    lib.bsvt_noalloc(inplace, 16, 16, 1.1, (2, 3), out=inplace)
    torch.cuda.synchronize()
    assert torch.equal(inplace, ref)
    # 1 x 1 blocks and a workspace beyond the fixed array are refused before any work
    with pytest.raises(lib.MsldError) as ei:
        lib.bsvt_noalloc(Vd, 1, 1, 1.0)
    assert ei.value.status == -1
    big = torch.zeros((4096, 4096), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.MsldError) as ei:
        lib.bsvt_noalloc(big, 8, 8, 1.0)
    assert ei.value.status == -6
    # the output buffer was not touched by the refused calls
    assert torch.equal(inplace, ref)
