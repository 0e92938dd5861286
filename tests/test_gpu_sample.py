"""GPU parity of rsrr_sample (RSRR Step 2, eq. hatS) against the CPU FP64 oracle.

Each block X_k = T(z_k)^-1 U of the HIP result is compared with the oracle's
LAPACK solve on the same seeded inputs.  Bar: relative Frobenius error of
every block <= 1e-10 (both precisions: the mixed path refines to FP64
backward error), and the FP64 residual that the library reports agrees with
one the oracle computes on the CPU.
"""
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


@pytest.fixture(scope="module")
def ctx(R):
    return R.rsrr_create(0)


def _blocks(S_dev, n, L, N, R):
    S = R.from_colmajor(S_dev, n)
    return [S[:, k * L:(k + 1) * L] for k in range(N)]


def _check_parity(R, ctx, nep, z, U, prec, tol=1e-10):
    prob = O.Problem(nep)
    dnep = R.DeviceNEP(nep)
    S, info, code = R.rsrr_sample(ctx, dnep, z, U, prec=prec)
    torch.cuda.synchronize()
    n, L = U.shape
    Xs = _blocks(S, n, L, len(z), R)
    worst = 0.0
    for k, zk in enumerate(z):
        Xo = O.solve_point(prob.T(zk), U)
        err = np.linalg.norm(Xs[k] - Xo) / np.linalg.norm(Xo)
        worst = max(worst, err)
        res = np.linalg.norm(U - prob.T(zk) @ Xs[k], axis=0) / np.linalg.norm(U, axis=0)
        assert res.max() <= 1e-10, (k, res.max())
        assert info[k]["resid"] <= 1e-10
        # the two FP64 residuals differ only by rounding (order eps * kappa)
        assert abs(info[k]["resid"] - res.max()) <= max(0.05 * res.max(), 1e-13)
    assert worst <= tol, worst
    return info


@pytest.mark.parametrize("prec", [0, 1])
def test_sample_qep_cfg0_reading(R, ctx, prec):
    """Rotated diagonal QEP n=200, N=32, L=16 on the ellipse centred 5i (semi-axes 4, 1)."""
    nep, C, U = W.cfg_qep()
    z, _ = O.ellipse(C.gamma, C.a, C.b, C.N)
    info = _check_parity(R, ctx, nep, z, U, prec)
    if prec == 1:
        assert all(i["fallback"] == 0 for i in info)
        assert max(i["ir_iters"] for i in info) <= 6


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 130, 257])
@pytest.mark.parametrize("prec", [0, 1])
def test_sample_ragged_sizes(R, ctx, n, prec):
    """Tile and panel edges: n not a multiple of the 64-column panel or the GEMM tiles."""
    nep = W.rotated_diagonal_qep(n, 100 + n)
    U = W.probes(n, 5, 7)
    z, _ = O.ellipse(1.0j, 3.0, 2.0, 6)
    _check_parity(R, ctx, nep, z, U, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_sample_delay(R, ctx, prec):
    """Delay Laplacian 16x16 (n=256), circle (-20, 15) of the throughput run, N=12, L=8."""
    nep = W.delay_laplacian(16)
    U = W.probes(nep.n, 8, 1000)
    z, _ = O.ellipse(-20.0, 15.0, 15.0, 12)
    _check_parity(R, ctx, nep, z, U, prec)


@pytest.mark.parametrize("prec", [0, 1])
def test_sample_helmholtz(R, ctx, prec):
    """Helmholtz sphere n=300 on the ellipse (3.8; 1.4, 0.3), N=8, L=6."""
    nep = W.helmholtz_sphere(300)
    U = W.probes(300, 6, 2000)
    z, _ = O.ellipse(3.8, 1.4, 0.3, 8)
    _check_parity(R, ctx, nep, z, U, prec)


def test_sample_pivoting_needed(R, ctx):
    """A matrix whose leading entries are tiny forces row interchanges at every panel."""
    rng = np.random.default_rng(5)
    n = 150
    A0 = W.complex_gaussian(rng, (n, n))
    A0[np.arange(n), np.arange(n)] = 1e-12
    nep = W.SeparableNEP("piv", [A0, np.eye(n, dtype=complex)], [W.term(1, 0), W.term(1e-9, 1)])
    U = W.probes(n, 4, 3)
    z = np.array([0.1 + 0.2j, -0.3j])
    for prec in (0, 1):
        _check_parity(R, ctx, nep, z, U, prec, tol=1e-9)


def test_sample_exactly_singular_point(R, ctx):
    """T(2) = diag(z^2 - 4, ...) has an exact zero pivot: ESINGULAR with getrf's info."""
    n = 40
    k = np.linspace(1.0, 9.0, n)
    k[17] = -4.0
    nep = W.SeparableNEP("sing", [np.diag(k).astype(complex), np.eye(n, dtype=complex)],
                         [W.term(1, 0), W.term(1, 2)])
    U = W.probes(n, 3, 9)
    dnep = R.DeviceNEP(nep)
    for prec in (0, 1):
        S, info, code = R.rsrr_sample(ctx, dnep, np.array([2.0 + 0j, 1.0 + 1j]), U, prec=prec,
                                      ok=(R.RSRR_ESINGULAR,))
        assert code == R.RSRR_ESINGULAR
        assert info[0]["info"] > 0 and info[1]["info"] == 0
        assert info[1]["resid"] <= 1e-10


def test_sample_nan_input(R, ctx):
    n = 20
    A0 = np.eye(n, dtype=complex)
    A0[3, 5] = np.nan
    nep = W.SeparableNEP("nan", [A0], [W.term(1, 0)])
    dnep = R.DeviceNEP(nep)
    S, info, code = R.rsrr_sample(ctx, dnep, np.array([0.5 + 0j]), W.probes(n, 2, 1), prec=1, ok=(R.RSRR_ENAN,))
    assert code == R.RSRR_ENAN and info[0]["info"] < 0


def test_sample_argument_errors(R, ctx):
    nep = W.rotated_diagonal_qep(10, 1)
    dnep = R.DeviceNEP(nep)
    U = W.probes(10, 2, 1)
    with pytest.raises(R.RsrrError) as e:
        R.rsrr_sample(ctx, dnep, np.array([0.5 + 0j]), U, prec=7)
    assert e.value.code == -8


def test_sample_empty_and_degenerate_arguments(R, ctx):
    """Empty inputs are argument errors (nothing enqueued): no points, no probe columns,
    leading dimensions below n; the basis of a one-column S keeps one direction."""
    import ctypes as C
    nep = W.rotated_diagonal_qep(10, 1)
    dnep = R.DeviceNEP(nep)
    U, ldu = R.colmajor(W.probes(10, 2, 1))
    S = torch.zeros((2, 10), dtype=torch.complex128, device="cuda")
    z = (C.c_double * 2)(0.5, 0.0)
    L = R.lib()
    args = lambda N, Lc, lu, ls: (ctx.h, C.byref(dnep.desc), N, z, U.data_ptr(), Lc, lu, 1, S.data_ptr(), ls, None)
    assert L.rsrr_sample(*args(0, 2, 10, 10)) == -3
    assert L.rsrr_sample(*args(1, 0, 10, 10)) == -6
    assert L.rsrr_sample(*args(1, 2, 9, 10)) == -7
    assert L.rsrr_sample(*args(1, 2, 10, 9)) == -10
    Sd, _, _ = R.rsrr_sample(ctx, dnep, np.array([0.5 + 0j]), W.probes(10, 1, 3))
    Q, k, sig = R.rsrr_basis(ctx, Sd, 10, 1e-14)
    assert k == 1 and abs(np.linalg.norm(R.from_colmajor(Q[:1], 10)) - 1) < 1e-14
