"""GPU parity of rsrr_two_stage (Sec. 5.4 and Sec. 6) against the oracle's two-stage RSRR:
the added points equal the oracle's (1e-8 relative), the stage-2 eigenvalues inside
the contour match the oracle and the closed form within 1e-9, and the eigen-residuals
match the oracle's (they are set by the stage-2 subspace)."""
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


def _match(got, ref):
    return max(np.min(np.abs(ref - g)) / max(1.0, abs(g)) for g in got) if len(got) else 0.0


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("shape", [(60, 6, 4), (100, 8, 4)])
def test_two_stage_matches_oracle(R, prec, shape):
    n, N1, L = shape
    nep, C, U = W.cfg_qep(n=n, N=N1, L=L)
    prob = O.Problem(nep)
    r1, r2, znew = O.two_stage(prob, C, U, NQ=300)
    ctx = R.rsrr_create(0)
    out = R.rsrr_two_stage(ctx, R.DeviceNEP(nep), C.gamma, C.a, C.b, N1, U, prec=prec, NQ=300, max_new=32,
                           max_eigs=128)
    ctx.close()
    assert out["n_new"] == znew.size
    assert _match(out["z_new"], znew) < 1e-8 and _match(znew, out["z_new"]) < 1e-8
    ex = P.qep_roots(nep.extra["c"], nep.extra["k"])
    lv = O.level(out["lam"], C.gamma, C.a, C.b)
    ins = lv < 0.98
    oin = r2["lam"][r2["level"] < 0.98]
    assert ins.sum() == oin.size
    assert _match(out["lam"][ins], oin) < 1e-9 and _match(oin, out["lam"][ins]) < 1e-9
    assert _match(out["lam"][ins], ex) < 1e-9
    for i in np.where(ins)[0]:
        ro = O.residual(prob, out["lam"][i], out["V"][:, i])
        assert abs(ro - out["resid"][i]) <= 1e-3 * ro + 1e-15
        j = int(np.argmin(np.abs(r2["lam"] - out["lam"][i])))
        assert ro <= 2.0 * r2["res"][j] + 1e-14
    assert out["resid1_max"] > 1e3 * out["resid"][ins].max()
