"""GPU parity of rsrr_moments (the moment matrix M = S Z of Sec. 4.1) against the
oracle: M from the same S within 1e-13 (relative Frobenius), and the moment variant
of SS-RR (Steps 3-5 on M) with eigenvalues within 1e-9 of the oracle's and of the
closed form inside the contour."""
import numpy as np
import pytest

import workloads as W
from oracle import pins as P
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


@pytest.fixture(scope="module")
def ctx(R):
    return R.rsrr_create(0)


def _match(got, ref):
    return max(np.min(np.abs(ref - g)) / max(1.0, abs(g)) for g in got) if len(got) else 0.0


@pytest.mark.parametrize("shape", [(37, 5, 3, 1), (37, 5, 3, 5), (120, 16, 4, 7), (200, 32, 16, 8)])
def test_moments_match_oracle_on_the_same_S(R, ctx, shape):
    n, N, L, K = shape
    nep, C, U = W.cfg_qep(n=n, N=N, L=L)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, N)
    S, _, _ = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=0)
    rho = max(C.a, C.b)
    cap = (C.a + C.b) / (2 * rho)
    M = R.rsrr_moments(ctx, S, n, z, L, K, C.gamma, rho, cap)
    Sh = R.from_colmajor(S, n)
    Mo = O.moments(Sh, z, L, K, C.gamma, rho, cap)
    Mh = R.from_colmajor(M, n)
    assert np.linalg.norm(Mh - Mo) <= 1e-13 * np.linalg.norm(Mo)


def test_moment_variant_of_ssrr(R, ctx):
    nep, C, U = W.cfg_qep(n=200, N=32, L=16)
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, _, _ = R.rsrr_sample(ctx, dnep, z, U, prec=1)
    rho = max(C.a, C.b)
    M = R.rsrr_moments(ctx, S, 200, z, 16, 8, C.gamma, rho, (C.a + C.b) / (2 * rho))
    Q, k, _ = R.rsrr_basis(ctx, M, 200, 1e-14)
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, rho)
    out = R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b, NQ=300)
    ro = O.rsrr_moment(O.Problem(nep), C, U, K=8, NQ=300)
    assert k == ro["k"]
    ins = O.level(out["lam"], C.gamma, C.a, C.b) < 0.98
    oin = ro["lam"][ro["level"] < 0.98]
    assert ins.sum() == oin.size == 32
    assert _match(out["lam"][ins], oin) < 1e-9 and _match(oin, out["lam"][ins]) < 1e-9
    assert _match(out["lam"][ins], P.qep_roots(nep.extra["c"], nep.extra["k"])) < 1e-9
