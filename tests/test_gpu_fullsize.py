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


def test_sparse_gmres_full_size_sampled_points(R, ctx):
    """The sparse workload bench.py times (--workload gmres --gmres-nep sparse --N 32 --L 8): the
    delay Laplacian on a 20^3 grid (n = 8000) with its matrices in CSR, 32 points on the circle
    (-4, 0.75), 8 probes, one reference factorisation at the centre, the operator applied from
    the sparse rows.  Every point converged; at sampled points the residual recomputed with the
    oracle's dense T is <= 1.5 tol and the distance to the oracle's solve is within 2 kappa
    times it (T is complex symmetric: kappa_2 <= kappa_1, LAPACK's estimate)."""
    import scipy.linalg as sl
    from scipy.linalg import lapack
    nep, C, U = W.cfg_sparse(dims=(20, 20, 20), N=32, L=8)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    Ud, _ = R.colmajor(U)
    S, info, code = R.rsrr_sample_gmres(ctx, R.DeviceNEP(nep), z, Ud, [C.gamma], tol=1e-10, restart=32)
    torch.cuda.synchronize()
    assert code == R.RSRR_OK
    assert all(i["converged"] == 1 and i["resid"] <= 1e-10 for i in info)
    prob = O.Problem(nep)
    n, L = U.shape
    Sh = R.from_colmajor(S, n)
    for k in (3, 20):
        T = prob.T(z[k])
        assert np.array_equal(T, T.T)
        X = Sh[:, k * L:(k + 1) * L]
        res = np.linalg.norm(U - T @ X, axis=0) / np.linalg.norm(U, axis=0)
        assert res.max() <= 1.5e-10
        lu, piv = sl.lu_factor(T)
        Xo = sl.lu_solve((lu, piv), U)
        rcond, inf = lapack.zgecon(lu, np.linalg.norm(T, 1), norm="1")
        assert inf == 0
        err = np.linalg.norm(X - Xo, axis=0) / np.linalg.norm(Xo, axis=0)
        assert np.all(err <= 2.0 * res / rcond + 1e-13), (k, err, res, 1 / rcond)


def _clusters(lo, tol_rel=1e-3):
    out, seen = [], np.zeros(lo.size, bool)
    for i in range(lo.size):
        if seen[i]:
            continue
        cl = np.where(np.abs(lo - lo[i]) <= tol_rel * max(1.0, abs(lo[i])))[0]
        seen[cl] = True
        out.append(cl)
    return out


def test_headline_eigenpairs_match_the_oracle(R, ctx, headline):
    """Helmholtz n = 4096, N = 64, L = 64 (mixed precision, the bench's launch), Steps 3-5 against
    the oracle's RSRR on the same inputs (tests/golden/helmholtz_n4096_N64_L64.json, written by
    make_helmholtz_n4096.py from oracle/ only): eigenvalues inside within 1e-9 (relative), the
    gap count, k within the rounding band at delta (reading: counts near delta*sigma_1 may move),
    singular values of S within 1e-13 sigma_1 where the sketch resolved them, eigenvector cosines
    (per cluster of eigenvalues within 1e-3) >= 1 - 1e-9, residuals <= 1e-10."""
    import json
    import os
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    g = json.load(open(os.path.join(here, "helmholtz_n4096_N64_L64.json")))
    Vo = np.load(os.path.join(here, "helmholtz_n4096_N64_L64_V.npz"))["V"]
    lo = np.array([complex(a, b) for a, b in g["lam_inside"]])
    nep, C, U, dnep, z, S, info, code = headline
    n = nep.points.shape[0]
    Q, k, sig = R.rsrr_basis(ctx, S.clone(), n, 1e-14)
    so = np.array(g["sigma_S_leading"])
    assert abs(k - g["k"]) <= 8
    r = min(int(np.sum(sig > 0)), k - 8)
    assert np.max(np.abs(sig[:r] - so[:r])) <= 1e-13 * so[0]
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, max(C.a, C.b))
    out = R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b)
    assert out["nbar"] == g["nbar"]
    ins = O.level(out["lam"], C.gamma, C.a, C.b) < 1
    lam, V = out["lam"][ins], out["V"][:, ins]
    assert lam.size == lo.size == 4
    assert _match_rel(lam, lo) < 1e-9 and _match_rel(lo, lam) < 1e-9
    for cl in _clusters(lo):
        gsel = np.array([int(np.argmin(np.abs(lam - lo[i]))) for i in cl])
        assert np.unique(gsel).size == cl.size
        qa = np.linalg.qr(V[:, gsel])[0]
        qb = np.linalg.qr(Vo[:, cl])[0]
        cos = np.linalg.svd(qa.conj().T @ qb, compute_uv=False).min()
        assert cos >= 1 - 1e-9, (lo[cl], 1 - cos)
    assert out["resid"][ins].max() <= 1e-10


def _match_rel(got, ref):
    return max(np.min(np.abs(ref - x)) / max(1.0, abs(x)) for x in got)


def test_delay_parity_config_32x32(R, ctx):
    """Config 1' at its stated size: delay Laplacian 32 x 32 (n = 1024), parity circle (-4, 0.75),
    N = 48, L = 32, mixed precision; the three eigenvalues inside against Lambert W to 1e-9 and
    eigen-residuals recomputed on the CPU."""
    from oracle import pins as P
    nep, C, U = W.cfg_delay(nx=32, N=48, L=32)
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, info, code = R.rsrr_sample(ctx, dnep, z, U, prec=1)
    assert code == R.RSRR_OK and all(i["resid"] <= 1e-10 for i in info)
    Q, k, _ = R.rsrr_basis(ctx, S, 1024, 1e-14)
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, max(C.a, C.b))
    out = R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b)
    ex = P.delay_eigs(W.laplacian_modes(32, 32))
    exin = ex[O.level(ex, C.gamma, C.a, C.b) < 1]
    ins = O.level(out["lam"], C.gamma, C.a, C.b) < 0.98
    assert exin.size == 3 and ins.sum() == 3
    assert _match_rel(out["lam"][ins], exin) < 1e-9 and _match_rel(exin, out["lam"][ins]) < 1e-9
    prob = O.Problem(nep)
    for i in np.where(ins)[0]:
        assert O.residual(prob, out["lam"][i], out["V"][:, i]) <= 1e-10


def test_sketch_narrower_than_S_matches_full_svd(R, ctx):
    """Helmholtz n = 2048, N = 48, L = 32: NL = 1536 is wider than the first sketch (1024
    columns).  Singular values of the normalised S within 1e-13 sigma_1 of the oracle's full SVD
    where resolved, k within the rounding band, and the leading subspace (to the largest gap)
    within 100x Wedin's bound of the oracle's."""
    nep, C, U = W.cfg_helmholtz(n=2048, N=48, L=32)
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, info, code = R.rsrr_sample(ctx, dnep, z, U, prec=1)
    assert code == R.RSRR_OK
    Sh = R.from_colmajor(S, 2048)
    Q, k, sig = R.rsrr_basis(ctx, S, 2048, 1e-14)
    Qo, sigo, ko = O.basis(O.normalize(Sh), 1e-14)
    assert abs(k - ko) <= 8
    r = min(int(np.sum(sig > 0)), k - 8)
    assert np.max(np.abs(sig[:r] - sigo[:r])) <= 1e-13 * sigo[0]
    # leading subspace up to the largest relative gap among sigma > 1e-6 sigma_1, against 100x
    # Wedin's bound eps sigma_1 / gap (the subspace is fixed only to that accuracy)
    cand = np.where(sigo[:k] > 1e-6 * sigo[0])[0]
    j = int(cand[np.argmax(sigo[cand] / sigo[cand + 1])])
    bound = 100 * 2.22e-16 * sigo[0] / (sigo[j] - sigo[j + 1])
    Qh = R.from_colmajor(Q[:k], 2048)
    A = Qo[:, :j + 1]
    assert np.linalg.norm(A - Qh @ (Qh.conj().T @ A), 2) <= max(bound, 1e-13)
