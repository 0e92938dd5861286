"""GPU parity at the benchmark's full sizes, in the launch configuration bench.py
times.  The oracle cannot redo whole runs of this size in seconds, so it
recomputes sampled outputs one by one (points of S, eigenpairs) and every
output is checked against properties that hold at any size (solve residuals,
eigen-residuals recomputed on the CPU).  Bars as in the small-size tests:
sampled blocks within 1e-10 (relative Frobenius) of the oracle's solve,
residuals <= 1e-10."""
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


def _sampled_parity(R, prob, S, z, U, ks, tol=1e-10):
    n, L = U.shape
    Sh = R.from_colmajor(S, n)
    for k in ks:
        Xo = O.solve_point(prob.T(z[k]), U)
        X = Sh[:, k * L:(k + 1) * L]
        assert np.linalg.norm(X - Xo) <= tol * np.linalg.norm(Xo), k


@pytest.fixture(scope="module")
def headline(R, ctx):
    """Helmholtz sphere n=4096, N=64, L=64, mixed precision: the default bench step."""
    nep, C, U = W.cfg_helmholtz()
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, info, code = R.rsrr_sample(ctx, dnep, z, U, prec=1)
    torch.cuda.synchronize()
    return nep, C, U, dnep, z, S, info, code


def test_headline_sampled_points_match_oracle(R, headline):
    nep, C, U, dnep, z, S, info, code = headline
    assert code == R.RSRR_OK
    assert all(i["resid"] <= 1e-10 and i["fallback"] == 0 and i["info"] == 0 for i in info)
    _sampled_parity(R, O.Problem(nep), S, z, U, ks=[0, 45])


def test_headline_eigenpairs(R, ctx, headline):
    """Steps 3-5 on the headline S; eigen-residuals recomputed on the CPU, and the eigenvalues
    near the zeros of the spherical Bessel functions j_0 (pi) and j_1 (4.4934, threefold) that
    the single-layer operator of the unit sphere has inside this contour."""
    nep, C, U, dnep, z, S, info, code = headline
    Q, k, sig = R.rsrr_basis(ctx, S.clone(), nep.points.shape[0], 1e-14)
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, max(C.a, C.b))
    out = R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b)
    ins = O.level(out["lam"], C.gamma, C.a, C.b) < 1
    lam = np.sort_complex(out["lam"][ins])
    assert lam.size == 4
    assert abs(lam[0] - np.pi) < 1e-2
    assert np.all(np.abs(lam[1:] - 4.4934) < 1e-2)
    prob = O.Problem(nep)
    for i in np.where(ins)[0]:
        r = O.residual(prob, out["lam"][i], out["V"][:, i])
        assert r <= 1e-10
        assert abs(r - out["resid"][i]) <= 0.05 * r + 1e-16


def test_largest_size_sampled_point(R, ctx):
    """n = 8192 (the largest serving size), two points, both precisions."""
    nep = W.helmholtz_sphere(8192)
    U = W.probes(8192, 8, 2001)
    z, _ = R.rsrr_contour(3.8, 1.4, 0.3, 2)
    prob = O.Problem(nep)
    for prec in (0, 1):
        S, info, code = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=prec)
        assert code == R.RSRR_OK and all(i["resid"] <= 1e-10 for i in info)
        _sampled_parity(R, prob, S, z, U, ks=[1])


@pytest.mark.parametrize("prec", [0, 1])
def test_delay_throughput_config_sampled(R, ctx, prec):
    """Delay Laplacian 32x32 (n=1024), circle (-20, 15), N=48, L=32."""
    nep, C, U = W.cfg_delay(nx=32, N=48, L=32, parity=False)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, info, code = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=prec)
    assert code == R.RSRR_OK and all(i["resid"] <= 1e-10 for i in info)
    _sampled_parity(R, O.Problem(nep), S, z, U, ks=[0, 17, 47])


def test_ragged_batch_config_sampled(R):
    """The 256-instance ragged batch (n ~ U{64..1024}, N=24, L=8) replayed from its hipGraph;
    five instances (smallest, largest and three others) checked point by point."""
    sizes = [int(n) for n in W.cfg_batched_sizes(count=256)]
    z, _ = R.rsrr_contour(5j, 4.0, 1.0, 24)
    items, neps = [], []
    for i, n in enumerate(sizes):
        nep = W.rotated_diagonal_qep(n, 3000 + i)
        U = W.probes(n, 8, 30000 + i)
        items.append(R.BatchItem(R.DeviceNEP(nep), z, U))
        neps.append((nep, U))
    ctx = R.rsrr_create(0)
    R.rsrr_sample_batched(ctx, items, flags=R.RSRR_BATCH_GRAPH)   # capture
    for it in items:
        it.S.zero_()
    infos, code = R.rsrr_sample_batched(ctx, items, flags=R.RSRR_BATCH_GRAPH)  # replay
    torch.cuda.synchronize()
    assert code == R.RSRR_OK
    assert all(p["resid"] <= 1e-10 and p["fallback"] == 0 for inf in infos for p in inf)
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 100, 200})
    for i in pick:
        nep, U = neps[i]
        _sampled_parity(R, O.Problem(nep), items[i].S, z, U, ks=[0, 11, 23])
    ctx.close()


def test_gmres_full_size_sampled_points(R, ctx):
    """The GMRES workload bench.py times: Helmholtz sphere n=4096 on the headline ellipse, N=64,
    L=2, one reference factorisation at the centre, tol 1e-10.  Every point converged; at sampled
    points the residual recomputed with the oracle's T is <= 1.5 tol, and the distance to the
    oracle's solve is within 2 kappa times it.  kappa: LAPACK's 1-norm estimate (zgecon) on the
    oracle's LU; T is complex symmetric, so kappa_2 <= kappa_1."""
    import scipy.linalg as sl
    from scipy.linalg import lapack
    nep, C, U = W.cfg_helmholtz(n=4096, N=64, L=2)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    Ud, _ = R.colmajor(U)
    S, info, code = R.rsrr_sample_gmres(ctx, R.DeviceNEP(nep), z, Ud, [C.gamma], tol=1e-10, restart=32)
    torch.cuda.synchronize()
    assert code == R.RSRR_OK
    assert all(i["converged"] == 1 and i["resid"] <= 1e-10 for i in info)
    prob = O.Problem(nep)
    Sh = R.from_colmajor(S, 4096)
    for k in (0, 45):
        T = prob.T(z[k])
        assert np.allclose(T, T.T)
        X = Sh[:, 2 * k:2 * k + 2]
        res = np.linalg.norm(U - T @ X, axis=0) / np.linalg.norm(U, axis=0)
        assert res.max() <= 1.5e-10
        lu, piv = sl.lu_factor(T)
        Xo = sl.lu_solve((lu, piv), U)
        rcond, inf = lapack.zgecon(lu, np.linalg.norm(T, 1), norm="1")
        assert inf == 0
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert np.all(err <= 2.0 * res / rcond + 1e-13), (k, err, res, 1 / rcond)
