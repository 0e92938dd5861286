"""rsrr_moments_noalloc (no device allocation: points and coefficient table in the
library's static per-GPU scratch array) against rsrr_moments on the same inputs,
through the C ABI: bitwise equal (the same kernels on the same table) and within
1e-13 of the oracle; two calls in a row, the second smaller, so the shared array's
leftover contents from the first call cannot leak into the second; a size beyond
the array is refused before anything is enqueued."""
import numpy as np
import pytest

import workloads as W
from oracle import rsrr_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1605_07951_amd import rsrr
    rsrr.lib()
    return rsrr


def _case(R, ctx, n, N, L, K, seed):
    nep, C, U = W.cfg_qep(n=n, N=N, L=L, seed=seed)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, N)
    S, _, _ = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=0)
    rho = max(C.a, C.b)
    return S, z, C.gamma, rho, (C.a + C.b) / (2 * rho)


def test_noalloc_moments_equal_the_allocating_call(R):
    ctx = R.rsrr_create(0)
    try:
        for (n, N, L, K, seed) in [(200, 32, 16, 8, 1), (120, 16, 4, 7, 2)]:
            S, z, g, rho, cap = _case(R, ctx, n, N, L, K, seed)
            ref = R.rsrr_moments(ctx, S, n, z, L, K, g, rho, cap)
            M = torch.full((K * L, n), complex(np.nan, np.nan), dtype=torch.complex128, device=S.device)
            R.rsrr_moments_noalloc(ctx, S, n, z, L, K, g, rho, cap, M)
            torch.cuda.synchronize()
            assert torch.equal(M, ref)
            Mo = O.moments(R.from_colmajor(S, n), z, L, K, g, rho, cap)
            Mh = R.from_colmajor(M, n)
            assert np.linalg.norm(Mh - Mo) <= 1e-13 * np.linalg.norm(Mo)
        # beyond the scratch array: refused, nothing written
        S, z, g, rho, cap = _case(R, ctx, 64, 300, 1, 300, 3)
        M = torch.zeros((300, 64), dtype=torch.complex128, device=S.device)
        with pytest.raises(R.RsrrError) as e:
            R.rsrr_moments_noalloc(ctx, S, 64, z, 1, 300, g, rho, cap, M)
        assert e.value.code == R.RSRR_ELIMIT
        assert torch.count_nonzero(M).item() == 0
    finally:
        ctx.close()
