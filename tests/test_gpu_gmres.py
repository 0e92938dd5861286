"""GPU parity of rsrr_sample_gmres: resolvent sampling (RSRR Step 2, eq. hatS)
with flexible GMRES preconditioned by complex FP32 LU factors of T at
reference points, against the CPU FP64 oracle.

GMRES stops at a relative residual tol, so the oracle's direct solve is
matched up to the perturbation bound of a residual: for each column,
||x - x*|| / ||x*|| <= kappa_2(T(z_k)) ||u - T x|| / ||u||.  Bars (written
below): every point converged; the FP64 relative residual of every column,
recomputed on the CPU with the oracle's own T(z_k), is at most 1.5 tol and
agrees with the one the library reports; every column's distance to the
oracle's solve is at most 2 kappa_2 times its residual (kappa_2 from an SVD
on the CPU) plus 1e-13.
"""
import os

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


def _check(R, nep, z, U, S_dev, infos, tol, kappa=True):
    prob = O.Problem(nep)
    n, L = U.shape
    S = R.from_colmajor(S_dev, n)
    worst = 0.0
    for k, zk in enumerate(z):
        T = prob.T(zk)
        X = S[:, k * L:(k + 1) * L]
        res = np.linalg.norm(U - T @ X, axis=0) / np.linalg.norm(U, axis=0)
        assert infos[k]["converged"] == 1, (k, infos[k])
        assert res.max() <= 1.5 * tol, (k, res.max())
        # the library's own FP64 residual agrees with the oracle's recomputation
        assert abs(infos[k]["resid"] - res.max()) <= 0.05 * tol + 0.05 * res.max(), (k, infos[k]["resid"], res.max())
        if kappa:
            Xo = O.solve_point(T, U)
            kap = np.linalg.cond(T)
            err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
            assert np.all(err <= 2.0 * kap * res + 1e-13), (k, err.max(), kap, res.max())
            worst = max(worst, float((err / (kap * res + 1e-300)).max()))
    return worst


def _run(R, ctx, nep, z, U, zref, ref=None, tol=1e-10, restart=32, max_iters=300, ok=None, flags=0):
    dn = R.DeviceNEP(nep)
    Ud, _ = R.colmajor(U)
    kw = {} if ok is None else {"ok": ok}
    S, infos, code = R.rsrr_sample_gmres(ctx, dn, z, Ud, zref, ref=ref, tol=tol, restart=restart,
                                         max_iters=max_iters, flags=flags, **kw)
    torch.cuda.synchronize()
    return S, infos, code


def test_gmres_helmholtz_one_reference(R, ctx):
    nep, C, U = W.cfg_helmholtz(n=512, N=16, L=2, seed=2100)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma])
    assert code == R.RSRR_OK
    assert all(i["ref"] == 0 for i in infos)
    assert all(2 <= i["iters"] <= 60 for i in infos), [i["iters"] for i in infos]
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_delay_nearest_of_four_references(R, ctx):
    nep, C, U = W.cfg_delay(nx=16, ny=32, N=12, L=3, seed=1100)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    zref, _ = R.rsrr_contour(C.gamma, 0.5 * C.a, 0.5 * C.b, 4)
    S, infos, code = _run(R, ctx, nep, z, U, zref)
    assert code == R.RSRR_OK
    near = [int(np.argmin(np.abs(zref - zk))) for zk in z]
    assert [i["ref"] for i in infos] == near
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_qep_own_factors_converge_at_once(R, ctx):
    """With each point's own factors as preconditioner the FP64 iteration needs only a few steps."""
    nep, C, U = W.cfg_qep(n=200, N=10, L=4, seed=7)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, z, ref=list(range(len(z))))
    assert code == R.RSRR_OK
    assert all(i["iters"] <= 4 for i in infos), [i["iters"] for i in infos]
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_unequal_reference_groups_and_order(R, ctx):
    """References of different group sizes, assigned out of point order (grouped solves per reference)."""
    nep, C, U = W.cfg_qep(n=160, N=7, L=2, seed=11)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    zref = np.array([z[0], z[3], z[5]])
    ref = [2, 0, 0, 1, 2, 2, 0]
    S, infos, code = _run(R, ctx, nep, z, U, zref, ref=ref)
    assert code == R.RSRR_OK
    assert [i["ref"] for i in infos] == ref
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_inverse_preconditioner_unequal_groups(R, ctx):
    """Enough points per reference to apply the factors as explicit inverses, groups of 8, 5 and 3."""
    nep, C, U = W.cfg_helmholtz(n=256, N=16, L=2, seed=2600)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    zref, _ = R.rsrr_contour(C.gamma, 0.5 * C.a, 0.5 * C.b, 3)
    ref = [0] * 8 + [1] * 5 + [2] * 3
    ref = ref[5:] + ref[:5]
    S, infos, code = _run(R, ctx, nep, z, U, zref, ref=ref)
    assert code == R.RSRR_OK
    assert [i["ref"] for i in infos] == ref
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_split_products_with_ragged_slices(R, ctx):
    """n = 300: the split preconditioner product ends in a partial K slice (300 = 4*64 + 44)."""
    nep, C, U = W.cfg_helmholtz(n=300, N=8, L=2, seed=2700)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma])
    assert code == R.RSRR_OK
    _check(R, nep, z, U, S, infos, 1e-10)


@pytest.mark.parametrize("L", [2, 5, 20])
def test_gmres_helmholtz_matrix_free_operator(R, ctx, L):
    """Entries generated inside every application (no stored matrices): the same bars, and the
    iterate agrees with the one from the assembled matrices (same entry formula, same order)."""
    nep, C, U = W.cfg_helmholtz(n=320, N=6, L=L, seed=2800)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma], flags=R.RSRR_GMRES_MATRIX_FREE)
    assert code == R.RSRR_OK
    assert all(i["matrix_free"] == 1 for i in infos)
    _check(R, nep, z, U, S, infos, 1e-10)
    S2, infos2, _ = _run(R, ctx, nep, z, U, [C.gamma])
    assert all(i["matrix_free"] == 0 for i in infos2)
    a, b = R.from_colmajor(S, 320), R.from_colmajor(S2, 320)
    assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    assert all(abs(x["iters"] - y["iters"]) <= 1 for x, y in zip(infos, infos2))


def test_gmres_short_restart_cycles(R, ctx):
    nep, C, U = W.cfg_helmholtz(n=384, N=6, L=2, seed=2200)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma], restart=4, max_iters=400)
    assert code == R.RSRR_OK
    assert max(i["restarts"] for i in infos) >= 1
    _check(R, nep, z, U, S, infos, 1e-10)


def test_gmres_helmholtz_many_probes_gemm_operator(R, ctx):
    """L > 16 takes the batched GEMM operator instead of the skinny kernel."""
    nep, C, U = W.cfg_helmholtz(n=256, N=4, L=20, seed=2300)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma], tol=1e-11)
    assert code == R.RSRR_OK
    _check(R, nep, z, U, S, infos, 1e-11)


def test_gmres_zero_probe_column(R, ctx):
    nep, C, U = W.cfg_delay(nx=8, ny=16, N=5, L=3, seed=1200)
    U = U.copy()
    U[:, 1] = 0.0
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    dn = R.DeviceNEP(nep)
    Ud, _ = R.colmajor(U)
    S, infos, code = R.rsrr_sample_gmres(ctx, dn, z, Ud, [C.gamma])
    torch.cuda.synchronize()
    assert code == R.RSRR_OK
    Sh = R.from_colmajor(S, nep.n)
    for k in range(len(z)):
        assert np.all(Sh[:, k * 3 + 1] == 0)
    prob = O.Problem(nep)
    for k, zk in enumerate(z):
        X = Sh[:, k * 3:(k + 1) * 3]
        T = prob.T(zk)
        for c in (0, 2):
            assert np.linalg.norm(U[:, c] - T @ X[:, c]) / np.linalg.norm(U[:, c]) <= 1.5e-10


def test_gmres_reports_non_convergence(R, ctx):
    nep, C, U = W.cfg_helmholtz(n=256, N=3, L=2, seed=2400)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx, nep, z, U, [C.gamma], tol=1e-12, restart=2, max_iters=2,
                          ok=(R.RSRR_OK, R.RSRR_ENOTCONV))
    assert code == R.RSRR_ENOTCONV
    assert any(i["converged"] == 0 for i in infos)
    for i in infos:
        assert i["iters"] <= 2
        assert (i["converged"] == 1) == (i["resid"] <= 1e-12)
    assert torch.isfinite(torch.view_as_real(S)).all()


def test_gmres_argument_errors(R, ctx):
    import ctypes as C_
    nep, C, U = W.cfg_helmholtz(n=64, N=2, L=1, seed=1)
    dn = R.DeviceNEP(nep)
    Ud, _ = R.colmajor(U)
    S = torch.empty((2, 64), dtype=torch.complex128, device="cuda")
    z = np.array([3.0 + 0.1j, 4.0 - 0.1j])
    zr = np.array([3.8 + 0j])
    zp = z.view(np.float64).ctypes.data_as(C_.POINTER(C_.c_double))
    rp = zr.view(np.float64).ctypes.data_as(C_.POINTER(C_.c_double))
    f = R.lib().rsrr_sample_gmres
    good = dict(N=2, nref=1, ref=None, L=1, ldu=64, tol=1e-10, restart=8, it=50, flags=0, lds=64)

    def call(**kw):
        a = dict(good, **kw)
        return f(ctx.h, C_.byref(dn.desc), a["N"], kw.get("zp", zp), a["nref"], kw.get("rp", rp), a["ref"],
                 kw.get("U", Ud.data_ptr()), a["L"], a["ldu"], a["tol"], a["restart"], a["it"], a["flags"],
                 kw.get("S", S.data_ptr()), a["lds"], None)

    nullp = C_.cast(None, C_.POINTER(C_.c_double))
    assert f(None, None, 1, None, 1, None, None, None, 1, 1, 1e-10, 8, 10, 0, None, 1, None) == -1
    assert call(N=0) == -3
    assert call(zp=nullp) == -4
    assert call(nref=0) == -5
    assert call(rp=nullp) == -6
    assert call(ref=(C_.c_int * 2)(0, 1)) == -7
    assert call(U=None) == -8
    assert call(L=0) == -9
    assert call(ldu=63) == -10
    assert call(tol=0.0) == -11
    assert call(tol=1.0) == -11
    assert call(restart=0) == -12
    assert call(restart=65) == -12
    assert call(it=0) == -13
    assert call(flags=2) == -14
    assert call(S=None) == -15
    assert call(lds=63) == -16
    assert call() == R.RSRR_OK
    assert call(flags=R.RSRR_GMRES_MATRIX_FREE) == R.RSRR_OK


def test_gmres_chunked_by_memory_budget(R):
    """A small workspace budget (read when a context is created) splits the points into chunks of
    three; the result meets the same bars."""
    os.environ["RSRR_WS_BUDGET_MB"] = "5"
    try:
        ctx2 = R.rsrr_create(0)
    finally:
        del os.environ["RSRR_WS_BUDGET_MB"]
    nep, C, U = W.cfg_helmholtz(n=256, N=10, L=2, seed=2500)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, infos, code = _run(R, ctx2, nep, z, U, [C.gamma])
    assert code == R.RSRR_OK
    _check(R, nep, z, U, S, infos, 1e-10)
    ctx2.close()
