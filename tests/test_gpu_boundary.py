"""GPU tests of the boundary's contracts beyond the plain parity runs.

* rsrr_solve forms the reduced matrix of eq. A from every retained singular
  triplet (nbar of them, eq. gap) and only then returns the max_eigs of lowest
  elliptic level: with max_eigs < nbar the returned eigenvalues are those of
  the full run and of the oracle (1e-9), with RSRR_WARN_MORE and the truncation
  flag; a reduced problem larger than the old 256 limit (300 eigenvalues
  inside) is solved; one beyond 1024 is refused with RSRR_ELIMIT.
* rsrr_options: ir_max_iters = 0 sends every point of the complex FP32 path to
  the FP64 fallback (flagged, results equal to the oracle's); an
  ill-conditioned T (kappa ~ 1e8, beyond what FP32 factors can refine) falls
  back by itself; a narrow first range sketch in rsrr_basis (16 columns,
  doubling) gives the oracle's singular values and subspace.
"""
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


@pytest.fixture()
def ctx(R):
    c = R.rsrr_create(0)
    yield c
    c.close()


def _match(got, ref):
    return max(np.min(np.abs(ref - g)) / max(1.0, abs(g)) for g in got)


def _steps_3_to_5(R, ctx, dnep, S, C, max_eigs, NQ=500, KQ=2):
    n = dnep.n
    Q, k, _ = R.rsrr_basis(ctx, S, n, 1e-14)
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, max(C.a, C.b))
    return R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b, NQ=NQ, KQ=KQ, max_eigs=max_eigs)


def test_solve_max_eigs_below_count_returns_lowest_levels(R, ctx):
    """QEP n = 200 (centre 5i): nbar eigenpairs in all; max_eigs = 8 returns the 8 of lowest
    elliptic level, each equal to the full run's and the oracle's to 1e-9."""
    nep, C, U = W.cfg_qep()
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, _, _ = R.rsrr_sample(ctx, dnep, z, U)
    S2 = S.clone()
    full = _steps_3_to_5(R, ctx, dnep, S, C, max_eigs=512)
    cut = _steps_3_to_5(R, ctx, dnep, S2, C, max_eigs=8)
    nbar = full["nbar"]
    assert full["status"] == R.RSRR_OK and not full["truncated"] and full["lam"].size == nbar > 8
    assert cut["status"] == R.RSRR_WARN_MORE and cut["truncated"] and cut["nbar"] == nbar
    assert cut["lam"].size == 8
    lev_full = np.sort(O.level(full["lam"], C.gamma, C.a, C.b))
    lev_cut = O.level(cut["lam"], C.gamma, C.a, C.b)
    assert np.all(np.diff(lev_cut) >= 0)                      # increasing level
    assert np.allclose(lev_cut, lev_full[:8], rtol=0, atol=1e-9)
    assert _match(cut["lam"], full["lam"]) < 1e-9
    prob = O.Problem(nep)
    ro = O.rsrr(prob, C, U)
    assert _match(cut["lam"], ro["lam"]) < 1e-9
    assert _match(cut["lam"], P.qep_roots(nep.extra["c"], nep.extra["k"])) < 1e-9
    assert cut["resid"].max() <= 1e-10
    for i in range(8):
        assert O.residual(prob, cut["lam"][i], cut["V"][:, i]) <= 1e-10


def _diag_nep(lam):
    A = [np.diag(-lam).astype(complex), np.eye(lam.size, dtype=complex)]
    return W.SeparableNEP("diag", A, [W.term(1.0, 0), W.term(1.0, 1)])


def _diag_case(n, inside, seed):
    rng = np.random.default_rng(seed)
    r_in = 0.8 * np.sqrt(rng.uniform(0, 1, inside))
    r_out = rng.uniform(1.25, 2.0, n - inside)
    ph = rng.uniform(0, 2 * np.pi, n)
    return np.concatenate([r_in, r_out]) * np.exp(1j * ph)


def test_solve_reduced_problem_past_256(R, ctx):
    """T(z) = diag(z - l_i), n = 400, 300 eigenvalues inside the unit circle: rsrr_solve with Q = I
    forms and solves the 300 x 300 reduced matrix; all 300 eigenvalues match the l_i and the
    oracle's SS-FULL to 1e-9."""
    n, inside = 400, 300
    lam = _diag_case(n, inside, 11)
    nep = _diag_nep(lam)
    dnep = R.DeviceNEP(nep)
    Q, _ = R.colmajor(np.eye(n, dtype=complex))
    AQ, terms = R.rsrr_project(ctx, dnep, Q, n, 0.0, 1.0)
    out = R.rsrr_solve(ctx, dnep, Q, n, AQ, terms, 0j, 1.0, 1.0, NQ=200, KQ=1, max_eigs=n)
    assert out["nbar"] == inside and out["lam"].size == inside and out["status"] == R.RSRR_OK
    assert _match(out["lam"], lam[:inside]) < 1e-9 and _match(lam[:inside], out["lam"]) < 1e-9
    ro = O.ss_full(lambda zz: O.T_separable(nep.A, nep.terms, zz), n, 0j, 1.0, 1.0, NQ=200, KQ=1)
    assert ro["nbar"] == inside
    assert _match(out["lam"], ro["lam"]) < 1e-9
    assert out["resid"].max() <= 1e-10


def test_solve_refuses_more_than_1024(R, ctx):
    n, inside = 1100, 1040
    lam = _diag_case(n, inside, 12)
    dnep = R.DeviceNEP(_diag_nep(lam))
    Q, _ = R.colmajor(np.eye(n, dtype=complex))
    AQ, terms = R.rsrr_project(ctx, dnep, Q, n, 0.0, 1.0)
    with pytest.raises(R.RsrrError) as e:
        R.rsrr_solve(ctx, dnep, Q, n, AQ, terms, 0j, 1.0, 1.0, NQ=200, KQ=1, max_eigs=8)
    assert e.value.code == R.RSRR_ELIMIT


def test_options_round_trip_and_range_checks(R, ctx):
    o = R.rsrr_set_options(ctx, ir_max_iters=0, basis_sketch_max=16, fallback_resid=1e-11)
    assert (o.ir_max_iters, o.basis_sketch_max, o.fallback_resid) == (0, 16, 1e-11)
    assert o.ir_max_iters_batched == 3 and o.delta == 1e-14
    for bad in ({"ir_max_iters": -1}, {"ir_max_iters_batched": 17}, {"basis_sketch_max": 4}, {"ir_tol": 0.0},
                {"fallback_resid": 1.0}, {"delta": 0.0}, {"tol_gap": -1.0}):
        with pytest.raises(R.RsrrError):
            R.rsrr_set_options(ctx, **bad)
    o = R.rsrr_get_options(ctx)
    assert o.ir_max_iters == 0 and o.basis_sketch_max == 16      # a refused call changes nothing


def test_ir_max_iters_zero_sends_every_point_to_fp64(R, ctx):
    nep, C, U = W.cfg_qep(n=200, N=8, L=16)
    R.rsrr_set_options(ctx, ir_max_iters=0)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, info, code = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=R.RSRR_PREC_C64_IR)
    assert code == R.RSRR_WARN_FALLBACK
    assert all(i["fallback"] == 1 and i["ir_iters"] == 0 for i in info)
    assert max(i["resid"] for i in info) <= 1e-10
    So = O.sample(O.Problem(nep), z, U)
    Sh = R.from_colmajor(S, 200)
    assert np.linalg.norm(Sh - So) <= 1e-10 * np.linalg.norm(So)


def test_ill_conditioned_point_falls_back(R, ctx):
    """T(z) = A0 + z I with A0 = G diag(d) G^H, d from 1 down to 1e-8: at z = 0, kappa = 1e8 and
    complex FP32 factors cannot refine it; the point is redone in FP64.  Its solve has FP64
    backward error and the oracle's forward error within kappa * 1e-14."""
    n = 128
    rng = np.random.default_rng(5)
    G = W.haar_unitary(rng, n)
    d = np.logspace(0, -8, n)
    A0 = (G * d[None, :]) @ G.conj().T
    nep = W.SeparableNEP("illcond", [A0, np.eye(n, dtype=complex)], [W.term(1.0, 0), W.term(1.0, 1)])
    U = W.probes(n, 4, 6)
    z = np.array([0j, 0.5 + 0.5j])
    S, info, code = R.rsrr_sample(ctx, R.DeviceNEP(nep), z, U, prec=R.RSRR_PREC_C64_IR)
    assert code == R.RSRR_WARN_FALLBACK
    assert info[0]["fallback"] == 1 and info[1]["fallback"] == 0
    Sh = R.from_colmajor(S, n)
    prob = O.Problem(nep)
    So = O.sample(prob, z, U)
    X, Xo = Sh[:, :4], So[:, :4]
    assert np.linalg.norm(X - Xo) <= 1e8 * 1e-14 * np.linalg.norm(Xo)
    T = prob.T(0j)
    be = np.linalg.norm(U - T @ X, axis=0) / (np.linalg.norm(T, 2) * np.linalg.norm(X, axis=0))
    assert be.max() <= 1e-14
    assert np.linalg.norm(Sh[:, 4:] - So[:, 4:]) <= 1e-10 * np.linalg.norm(So[:, 4:])


def test_narrow_sketch_basis_matches_full_svd(R, ctx):
    """basis_sketch_max = 16 on a 300 x 512 Helmholtz S: the sketch doubles to the range of S;
    singular values within 1e-13 sigma_1 of the oracle's full SVD where resolved, k equal, and the
    leading subspace within 1e-10 of the oracle's; the whole method's eigenvalues match to 1e-9."""
    nep, C, U = W.cfg_helmholtz(n=300, N=16, L=32)
    dnep = R.DeviceNEP(nep)
    z, _ = R.rsrr_contour(C.gamma, C.a, C.b, C.N)
    S, _, _ = R.rsrr_sample(ctx, dnep, z, U)
    Sh = R.from_colmajor(S, 300)
    R.rsrr_set_options(ctx, basis_sketch_max=16)
    Q, k, sig = R.rsrr_basis(ctx, S, 300, 1e-14)
    Qo, sigo, ko = O.basis(O.normalize(Sh), 1e-14)
    r = int(np.sum(sig > 0))
    assert r >= ko - 2 and abs(k - ko) <= 2
    assert np.max(np.abs(sig[:r] - sigo[:r])) <= 1e-13 * sigo[0]
    Qh = R.from_colmajor(Q[:k], 300)
    lead = int(np.sum(sigo > 1e-8 * sigo[0]))
    A = Qo[:, :lead]
    assert np.linalg.norm(A - Qh @ (Qh.conj().T @ A), 2) <= 1e-10
    AQ, terms = R.rsrr_project(ctx, dnep, Q, k, C.gamma, max(C.a, C.b))
    out = R.rsrr_solve(ctx, dnep, Q, k, AQ, terms, C.gamma, C.a, C.b, NQ=200)
    ro = O.rsrr(O.Problem(nep), C, U, NQ=200, S=Sh)
    ins = O.level(out["lam"], C.gamma, C.a, C.b) < 0.98
    oin = ro["lam"][ro["level"] < 0.98]
    assert ins.sum() == oin.size == 4
    assert _match(out["lam"][ins], oin) < 1e-9 and _match(oin, out["lam"][ins]) < 1e-9
