"""Pins of the CPU FP64 oracle against closed forms, textbook reductions and brute force.

Every oracle step has at least one check here that a plausible slip (a
dropped term, a wrong sign or index, a transposed operand) would fail; the
last group plants such slips in the oracle and checks that a pin catches them.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import pins as P
from oracle import rsrr_oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------- Step 1 ----

def test_ellipse_quadrature_identities():
    """Trapezoid nodes/weights of eq. ellip-contour-xw: sum w/(z - z0) = i inside, 0 outside; sum w z^m = 0."""
    z, w = O.ellipse(0.3 + 0.2j, 2.0, 0.7, 128)
    assert abs(np.sum(w / (z - (0.5 + 0.15j))) - 1j) < 1e-12
    assert abs(np.sum(w / (z - (6.0 + 0.0j)))) < 1e-12
    for m in range(0, 20):
        assert abs(np.sum(w * (z - 0.3 - 0.2j) ** m)) < 1e-12 * 2.0 ** m
    # node placement: alpha_j = 2 pi (j + 1/2)/N on the ellipse
    assert np.allclose(O.level(z, 0.3 + 0.2j, 2.0, 0.7), 1.0)
    assert abs(z[0] - (0.3 + 0.2j + 2.0 * math.cos(math.pi / 128) + 0.7j * math.sin(math.pi / 128))) < 1e-15


def test_coefficient_terms_closed_values():
    t = W.term(2.0, 2, z0=1.0, tau=0.5, s=3.0, q=1)
    assert abs(O.coef(t, 2.0) - (2.0 * 1.0 * math.exp(-1.0) / (-1.0))) < 1e-15
    t2 = W.term(-1.0, 1)
    assert O.coef(t2, 3.0 + 1j) == -(3.0 + 1j)
    # derivative against a central difference on a smooth term
    for t in (W.term(1.5, 3, z0=0.2, tau=0.3, s=2.0, q=2), W.term(-1.0, 1), W.term(1.0, 0, tau=1.0)):
        z0, h = 0.7 + 0.4j, 1e-5
        fd = (O.coef(t, z0 + h) - O.coef(t, z0 - h)) / (2 * h)
        assert abs(fd - O.coef_deriv(t, z0)) < 1e-8 * max(1.0, abs(fd))


# --------------------------------------------------------------- T(z) ------

def test_qep_assembly_matches_rotated_diagonal():
    nep = W.rotated_diagonal_qep(12, 5)
    Q, c, k = nep.extra["Q"], nep.extra["c"], nep.extra["k"]
    for z in (0.3 + 2j, -1.0 + 0.5j):
        ref = Q.conj().T @ np.diag(z * z + c * z + k) @ Q
        assert np.allclose(O.T_separable(nep.A, nep.terms, z), ref, atol=1e-12, rtol=0)


def test_helmholtz_single_layer_of_constant_density():
    """On the unit sphere, int e^{ikr}/(4 pi r) dS(y) = e^{ik} sin(k)/k; the Nystrom row sums approach it."""
    n = 2048
    nep = W.helmholtz_sphere(n)
    prob = O.Problem(nep)
    for kz in (1.0, 3.8, 2.5 + 0.2j):
        T = prob.T(kz)
        approx = T.sum(axis=1)
        exact = np.exp(1j * kz) * np.sin(kz) / kz
        assert np.max(np.abs(approx - exact)) < 3e-2 * abs(exact) + 5e-3
        assert np.allclose(T, T.T)  # complex symmetric


def _self_patch_ratio(T, z, w):
    """Largest |T_ii - D(z)| over the diagonal in units of |z|^2 a^3 / 12, where
    D(z) = (e^{i z a} - 1)/(2 i z) is the single-layer integral of e^{i z r}/(4 pi r)
    over a flat disk of radius a = sqrt(w/pi) about its centre (the self patch of the
    Nystrom rule), and |z|^2 a^3 / 12 is the size of its first term past second order."""
    a = math.sqrt(w / math.pi)
    disk = (np.exp(1j * z * a) - 1.0) / (2j * z)
    return float(np.max(np.abs(np.diag(T) - disk)) / (abs(z) ** 2 * a ** 3 / 12.0))


def test_helmholtz_self_patch_is_the_disk_integral():
    """The diagonal sqrt(w/pi)/2 + i z w/(4 pi) is the disk integral (e^{iza} - 1)/(2iz) up to
    its third-order term -z^2 a^3/12: both terms of the diagonal are fixed by it."""
    for n in (1024, 2048):
        nep = W.helmholtz_sphere(n)
        for z in (1.0, 3.8, 2.5 + 0.2j, 4.9 - 0.1j):
            T = O.T_helmholtz(nep.points[:16], nep.w, z)
            assert _self_patch_ratio(T, z, nep.w) < 1.25


def test_helmholtz_derivative_is_the_difference_quotient():
    """dT/dz against a central difference of T (step 1e-5): off the diagonal and on it."""
    nep = W.helmholtz_sphere(300)
    for z in (3.8, 2.5 + 0.2j):
        h = 1e-5
        fd = (O.T_helmholtz(nep.points, nep.w, z + h) - O.T_helmholtz(nep.points, nep.w, z - h)) / (2 * h)
        D = O.dT_helmholtz(nep.points, nep.w, z)
        assert np.max(np.abs(fd - D)) <= 1e-8 * np.max(np.abs(D))
        assert np.max(np.abs(np.diag(fd) - np.diag(D))) <= 1e-8 * np.max(np.abs(np.diag(D)))


def test_helmholtz_argument_count_inside_the_headline_ellipse():
    """Argument principle with T and dT/dz: the ellipse (3.8; 1.4, 0.3) holds 4 eigenvalues of the
    sphere's single-layer matrix (pi, and the l = 1 triple near 4.493 split by the lattice)."""
    nep = W.helmholtz_sphere(256)
    prob = O.Problem(nep)
    cnt = P.argument_count(prob.T, prob.dT, 3.8, 1.4, 0.3, M=128)
    assert abs(cnt - 4) < 1e-6


# --------------------------------------------------------------- Step 2 ----

def test_sample_matches_high_precision_solve():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    nep = W.rotated_diagonal_qep(6, 11)
    prob = O.Problem(nep)
    U = W.probes(6, 2, 3)
    z = np.array([0.4 + 3.1j, -0.2 + 1.0j])
    S = O.sample(prob, z, U)
    for kk, zk in enumerate(z):
        T = prob.T(zk)
        Tm = mpmath.matrix([[mpmath.mpc(T[i, j].real, T[i, j].imag) for j in range(6)] for i in range(6)])
        for c in range(2):
            b = mpmath.matrix([mpmath.mpc(U[i, c].real, U[i, c].imag) for i in range(6)])
            x = mpmath.lu_solve(Tm, b)
            xe = np.array([complex(x[i]) for i in range(6)])
            assert np.linalg.norm(S[:, 2 * kk + c] - xe) <= 1e-12 * np.linalg.norm(xe)


# --------------------------------------------------------------- Step 3 ----

def test_basis_recovers_planted_rank_and_singular_values():
    rng = np.random.default_rng(7)
    n, p, r = 60, 90, 17
    Ua = np.linalg.qr(W.complex_gaussian(rng, (n, r)))[0]
    Vb = np.linalg.qr(W.complex_gaussian(rng, (p, r)))[0]
    s = np.logspace(0, -12, r)
    S = (Ua * s[None, :]) @ Vb.conj().T
    Q, sig, k = O.basis(S, 1e-14)
    assert k == r
    assert np.allclose(sig[:r], s, rtol=1e-8, atol=1e-15)
    assert np.allclose(Q.conj().T @ Q, np.eye(k), atol=1e-12)
    # same span as the planted factor (directions with sigma >= 1e-3 are fixed to ~eps/sigma)
    lead = Ua[:, s >= 1e-3]
    assert np.linalg.norm(lead - Q @ (Q.conj().T @ lead)) < 1e-11


def test_normalize_keeps_span_and_unit_norms():
    rng = np.random.default_rng(8)
    S = W.complex_gaussian(rng, (20, 8)) * np.logspace(0, 6, 8)[None, :]
    Sn = O.normalize(S)
    assert np.allclose(np.linalg.norm(Sn, axis=0), 1.0)
    Q = np.linalg.qr(S)[0]
    assert np.linalg.norm(Sn - Q @ (Q.conj().T @ Sn)) < 1e-12


# --------------------------------------------------------------- Step 4-5 --

def test_ss_full_on_diagonal_nep_with_known_roots():
    """T(z) = diag(z - l_i): SS-FULL must return exactly the l_i inside the ellipse."""
    lam = np.array([0.2 + 0.1j, -0.5 + 0.3j, 0.9 - 0.2j, 3.0 + 0j, -2.5j, 0.0 + 0.05j])
    A = [np.diag(-lam).astype(complex), np.eye(lam.size, dtype=complex)]
    terms = [W.term(1.0, 0), W.term(1.0, 1)]
    TQ = lambda z: O.T_separable(A, terms, z)
    res = O.ss_full(TQ, lam.size, 0.1 + 0.0j, 1.5, 1.0, NQ=200, KQ=2)
    inside = lam[O.level(lam, 0.1, 1.5, 1.0) < 1]
    got = res["lam"]
    assert res["nbar"] == inside.size and not res["warn_gap"]
    for l in inside:
        assert np.min(np.abs(got - l)) < 1e-12
    # eigenvectors are the unit vectors of the matching coordinate
    for i, l in enumerate(got):
        j = int(np.argmin(np.abs(lam - l)))
        assert abs(abs(res["G"][j, i]) - 1.0) < 1e-10


def _match(got, ref):
    return max(np.min(np.abs(ref - g)) / max(1.0, abs(g)) for g in got)


@pytest.mark.slow
def test_rsrr_qep_closed_form_cfg0_reading():
    """Rotated diagonal QEP, n=200, N=32, L=16, centre 5i: eigenvalues vs roots of z^2 + c z + k."""
    nep, C, U = W.cfg_qep()
    prob = O.Problem(nep)
    r = O.rsrr(prob, C, U)
    ex = P.qep_roots(nep.extra["c"], nep.extra["k"])
    inside = r["level"] < 0.98
    assert inside.sum() >= 30
    assert _match(r["lam"][inside], ex) < 1e-9
    assert r["res"][inside].max() < 1e-10
    assert r["k"] == 200  # N*L = 512 > n: full rank
    # every exact root strictly inside (with margin) was found
    exin = ex[O.level(ex, C.gamma, C.a, C.b) < 0.98]
    assert _match(exin, r["lam"]) < 1e-9
    # eigenvectors are Q^H e_i
    Q = nep.extra["Q"]
    for i in np.where(inside)[0]:
        j = int(np.argmin(np.abs(ex - r["lam"][i]))) % 200
        v = Q.conj().T[:, j]
        assert abs(np.vdot(v, r["V"][:, i])) > 1 - 1e-9


def test_rsrr_qep_literal_contour_is_empty():
    """Centre 5 + 0i holds none of the roots: the gap rule does not find a reliable count."""
    nep, C, U = W.cfg_qep(n=40, N=16, L=4, literal=True)
    prob = O.Problem(nep)
    ex = P.qep_roots(nep.extra["c"], nep.extra["k"])
    assert np.all(O.level(ex, C.gamma, C.a, C.b) > 1)
    cnt = P.argument_count(prob.T, prob.dT, C.gamma, C.a, C.b, M=256)
    assert abs(cnt) < 1e-6
    r = O.rsrr(prob, C, U, NQ=200)
    assert np.sum(r["level"] < 0.98) == 0 or r["ss"]["warn_gap"]


@pytest.mark.slow
def test_rsrr_delay_lambert_w():
    """Delay Laplacian (16x16), circle (-4, 0.75): the three eigenvalues mu + W(0.5 e^-mu)."""
    nep, C, U = W.cfg_delay(nx=16, N=48, L=32)
    prob = O.Problem(nep)
    r = O.rsrr(prob, C, U)
    ex = P.delay_eigs(W.laplacian_modes(16, 16))
    exin = ex[O.level(ex, C.gamma, C.a, C.b) < 1]
    assert exin.size == 3
    inside = r["level"] < 0.98
    assert inside.sum() == 3
    assert _match(r["lam"][inside], exin) < 1e-9
    assert r["res"][inside].max() < 1e-10
    cnt = P.argument_count(prob.T, prob.dT, C.gamma, C.a, C.b, M=256)
    assert abs(cnt - 3) < 1e-6


def test_lambert_w_closed_form_solves_the_delay_equation():
    for mu in (-19.7, -49.3, -300.0):
        for br in (-2, 0, 1):
            lam = P._delay_branch(mu, 0.5, br)
            f = -lam + mu + 0.5 * np.exp(-lam) if lam.real > -700 else None
            if f is not None:
                assert abs(f) < 1e-9 * max(1.0, abs(lam))


def test_rsrr_tiny_nonnormal_against_det_newton():
    """n=5 non-normal QEP + delay mix: RSRR eigenvalues inside == brute-force det T roots inside."""
    rng = np.random.default_rng(21)
    n = 5
    A = [W.complex_gaussian(rng, (n, n)) for _ in range(3)]
    terms = [W.term(1.0, 0), W.term(1.0, 1), W.term(0.3, 0, tau=1.0)]
    nep = W.SeparableNEP("tiny", A, terms)
    prob = O.Problem(nep)
    C = W.Contour(0.0 + 0.0j, 1.6, 1.2, 40)
    seeds = [complex(x, y) for x in np.linspace(-2.4, 2.4, 13) for y in np.linspace(-1.8, 1.8, 10)]
    roots = P.det_newton_roots(prob.T, prob.dT, seeds)
    lv = O.level(roots, C.gamma, C.a, C.b)
    assert np.all(np.abs(lv - 1) > 0.05), "a root too close to the contour for this seed"
    rin = roots[lv < 1]
    cnt = P.argument_count(prob.T, prob.dT, C.gamma, C.a, C.b, M=512)
    assert abs(cnt - rin.size) < 1e-6
    U = W.probes(n, 3, 4)
    r = O.rsrr(prob, C, U, NQ=300)
    got = r["lam"][r["level"] < 1]
    assert got.size == rin.size
    assert _match(got, rin) < 1e-9 and _match(rin, got) < 1e-9


def test_companion_linearisation_agrees_for_random_qep():
    rng = np.random.default_rng(9)
    n = 10
    A0, A1 = W.complex_gaussian(rng, (n, n)), W.complex_gaussian(rng, (n, n))
    A2 = np.eye(n, dtype=complex)
    ev = P.companion_eigs(A0, A1, A2)
    nep = W.SeparableNEP("q", [A0, A1, A2], [W.term(1, 0), W.term(1, 1), W.term(1, 2)])
    prob = O.Problem(nep)
    C = W.Contour(0.2 + 0.1j, 1.3, 1.1, 48)
    lv = O.level(ev, C.gamma, C.a, C.b)
    if np.any(np.abs(lv - 1) < 0.05):
        pytest.skip("eigenvalue on the contour for this seed")
    r = O.rsrr(prob, C, W.probes(n, 4, 5), NQ=300)
    got = r["lam"][r["level"] < 1]
    ref = ev[lv < 1]
    assert got.size == ref.size
    assert _match(got, ref) < 1e-9


def test_residual_of_exact_and_perturbed_pairs():
    nep = W.rotated_diagonal_qep(30, 2)
    prob = O.Problem(nep)
    c, k, Q = nep.extra["c"], nep.extra["k"], nep.extra["Q"]
    lam = (-c[3] + np.sqrt(c[3] ** 2 - 4 * k[3] + 0j)) / 2
    v = Q.conj().T[:, 3]
    assert O.residual(prob, lam, v) < 1e-15
    assert O.residual(prob, lam * (1 + 1e-6), v) > 1e-9


# ------------------------------------------------------ paper golden value --

@pytest.mark.slow
def test_loaded_string_count_matches_paper():
    """Example 1: 32 eigenvalues in [3, 10000] for n = 400 (printed count)."""
    g = json.load(open(os.path.join(HERE, "golden", "loaded_string.json")))
    nep = W.loaded_string(g["n"])
    prob = O.Problem(nep)
    a = g["contour"]["a"]
    C = W.Contour(g["contour"]["gamma"] + 0j, a, a * g["contour"]["b_over_a"], 64)
    U = W.probes(g["n"], 2, 77)
    r = O.rsrr(prob, C, U, NQ=500)
    lam = r["lam"]
    sel = (lam.real >= g["interval"][0]) & (lam.real <= g["interval"][1]) & (r["level"] < 1) & (r["res"] < 1e-10)
    assert int(sel.sum()) == g["count"]
    assert np.max(np.abs(lam[sel].imag)) < 1e-6 * np.max(np.abs(lam[sel]))


# --------------------------------------------------------- planted slips ---

def test_planted_slips_are_caught(monkeypatch):
    """Mistakes planted in the oracle (on the CPU) make a pin fail."""
    nep = W.rotated_diagonal_qep(12, 5)
    Q, c, k = nep.extra["Q"], nep.extra["c"], nep.extra["k"]
    z = 0.3 + 2j
    ref = Q.conj().T @ np.diag(z * z + c * z + k) @ Q

    # a dropped term in the assembly
    T = O.T_separable(nep.A[:2], nep.terms[:2], z)
    assert not np.allclose(T, ref, atol=1e-12)
    # a transposed operand
    T = O.T_separable([A.T for A in nep.A], nep.terms, z)
    assert not np.allclose(T, ref, atol=1e-12)
    # a wrong sign in the trapezoid weight
    zz, ww = O.ellipse(0.3 + 0.2j, 2.0, 0.7, 64)
    assert abs(np.sum((-ww.conj()) / (zz - (0.5 + 0.1j))) - 1j) > 1e-3
    # an off-by-one Hankel shift in SS-FULL moves the eigenvalues
    lam = np.array([0.2 + 0.1j, -0.5 + 0.3j])
    A = [np.diag(-lam).astype(complex), np.eye(2, dtype=complex)]
    terms = [W.term(1.0, 0), W.term(1.0, 1)]
    orig_block = np.block

    def shifted_block(rows):
        if len(rows) == 2 and len(rows[0]) == 2:
            rows = [[rows[1][0], rows[1][1]], [rows[1][1], rows[1][1]]]
        return orig_block(rows)
    monkeypatch.setattr(O.np, "block", shifted_block)
    res = O.ss_full(lambda zz_: O.T_separable(A, terms, zz_), 2, 0.0, 1.5, 1.0, NQ=100, KQ=2)
    monkeypatch.undo()
    bad = res["lam"]
    assert bad.size == 0 or _match(bad, lam) > 1e-6 or res["warn_gap"]


def _moments_closed_form(lam, U, z, gamma, rho, capacity, K):
    """eq. fa1 for T(z) = diag(z - l_m): with mu = (l - gamma)/rho and l(x) = prod_j (x - zeta_j),
    sum_i omega_i zeta_i^alpha / (z_i - l_m) = -C^(N-1) mu_m^alpha / (rho l(mu_m)) for alpha <= N-1."""
    zeta = (np.asarray(z) - gamma) / rho
    mu = (lam - gamma) / rho
    node_poly = np.array([np.prod(m - zeta) for m in mu])
    L = U.shape[1]
    M = np.zeros((lam.size, K * L), dtype=np.complex128)
    for a in range(K):
        f = -capacity ** (zeta.size - 1) * mu ** a / (rho * node_poly)
        M[:, a * L:(a + 1) * L] = f[:, None] * U
    return M


def _diag_moment_case():
    lam = np.array([0.2 + 0.1j, -0.5 + 0.3j, 0.9 - 0.2j, 3.0 + 0j, -2.5j, 0.05j, 1.7 + 0.6j])
    A = [np.diag(-lam).astype(complex), np.eye(lam.size, dtype=complex)]
    nep = W.SeparableNEP("diag", A, [W.term(1.0, 0), W.term(1.0, 1)])
    C = W.Contour(0.3 + 0.1j, 1.5, 0.8, 12)
    U = W.probes(lam.size, 3, 31)
    z, _ = O.ellipse(C.gamma, C.a, C.b, C.N)
    S = O.sample(O.Problem(nep), z, U)
    rho = max(C.a, C.b)
    return lam, U, z, S, C.gamma, rho, (C.a + C.b) / (2 * rho), C.N


def test_moments_match_the_closed_form_of_a_diagonal_nep():
    """Sec. 4.1, eq. Malpha with the capacity-scaled weights of eq. bary-wt: every moment order
    alpha = 0..N-1 against the closed form that eq. fa1 gives for T(z) = diag(z - l_m)."""
    lam, U, z, S, gamma, rho, cap, N = _diag_moment_case()
    M = O.moments(S, z, U.shape[1], N, gamma, rho, cap)
    ref = _moments_closed_form(lam, U, z, gamma, rho, cap, N)
    assert np.linalg.norm(M - ref) <= 1e-12 * np.linalg.norm(ref)


def test_planted_moment_and_self_patch_slips_are_caught(monkeypatch):
    """A moment order off by one (zeta^(alpha+1) for zeta^alpha, planted through the weights),
    a dropped or sign-flipped self-patch term i z w/(4 pi), and a conjugated phase in the
    off-diagonal kernel each fail a pin."""
    lam, U, z, S, gamma, rho, cap, N = _diag_moment_case()
    ref = _moments_closed_form(lam, U, z, gamma, rho, cap, N)
    orig = O.barycentric_weights
    monkeypatch.setattr(O, "barycentric_weights", lambda zz, capacity=1.0: orig(zz, capacity) * np.asarray(zz))
    bad = O.moments(S, z, U.shape[1], N, gamma, rho, cap)
    monkeypatch.undo()
    assert np.linalg.norm(bad - ref) > 1e-3 * np.linalg.norm(ref)

    nep = W.helmholtz_sphere(2048)
    w = nep.w
    for zz in (3.8, 2.5 + 0.2j):
        T = O.T_helmholtz(nep.points[:16], w, zz)
        term = 1j * zz * w / (4.0 * math.pi)
        dropped = T - np.diag(np.full(16, term))
        flipped = T - np.diag(np.full(16, 2 * term))
        assert _self_patch_ratio(dropped, zz, w) > 5.0
        assert _self_patch_ratio(flipped, zz, w) > 5.0
    prob = O.Problem(nep)
    T = prob.T(3.8)
    conj = T.real - 1j * T.imag
    np.fill_diagonal(conj, np.diag(T))
    exact = np.exp(1j * 3.8) * np.sin(3.8) / 3.8
    assert np.max(np.abs(conj.sum(axis=1) - exact)) > 3e-2 * abs(exact) + 5e-3


def test_distinct_inside_keeps_first_of_close_estimates():
    lam = np.array([1.0 + 0.1j, 1.0 + 0.1j + 5e-7, 3.0 + 0j, 0.2 - 0.05j, 1.0 + 0.1j + 2e-6])
    got = O.distinct_inside(lam, 1.0 + 0j, 1.5, 0.5)  # 3.0 lies outside (level 1.78)
    assert np.allclose(got, [1.0 + 0.1j, 0.2 - 0.05j, 1.0 + 0.1j + 2e-6])


def test_two_stage_points_at_estimates_sharpen_the_eigenvalues():
    """Sec. 5.4 and Sec. 6: stage 1 on six contour points is rough; adding its estimates inside as
    sampling points gives every eigenvalue inside to 1e-9 of the closed form and cuts the
    eigen-residuals by orders of magnitude."""
    nep, C, U = W.cfg_qep(n=60, N=6, L=4)
    prob = O.Problem(nep)
    ex = P.qep_roots(nep.extra["c"], nep.extra["k"])
    r1, r2, znew = O.two_stage(prob, C, U, NQ=300)
    exin = ex[O.level(ex, C.gamma, C.a, C.b) < 0.98]
    in1, in2 = r1["level"] < 0.98, r2["level"] < 0.98
    assert exin.size == 5 and in2.sum() == 5
    assert _match(r1["lam"][in1], ex) > 1e-3              # stage 1 is rough
    assert _match(r2["lam"][in2], ex) < 1e-9 and _match(exin, r2["lam"]) < 1e-9
    assert r2["res"][in2].max() < 1e-4 * r1["res"][in1].max()
    # the new points are the stage-1 estimates inside, and S keeps the stage-1 columns
    assert znew.size == np.sum(r1["level"] < 1)
    assert np.array_equal(r2["S"][:, :C.N * 4], r1["S"])


def test_barycentric_weights_take_leading_coefficients():
    """eq. bary-wt / eq. fa1: sum_i omega_i p(z_i) is the leading coefficient of the degree N-1
    interpolant, so sum_i omega_i z_i^a = 0 for a < N-1 and 1 for a = N-1; scaling every
    factor by 1/C multiplies the weights by C^(N-1)."""
    rng = np.random.default_rng(0)
    z = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    w = O.barycentric_weights(z)
    for a in range(8):
        assert abs(np.sum(w * z ** a)) < 1e-12
    assert abs(np.sum(w * z ** 8) - 1) < 1e-12
    wc = O.barycentric_weights(z, capacity=2.5)
    assert np.allclose(wc, w * 2.5 ** 8, rtol=1e-12)


def test_chebyshev_weights_are_the_simplified_barycentric_weights():
    for N in (5, 12, 40):
        r = O.barycentric_weights(O.chebyshev_points(N)) / O.chebyshev_weights(N)
        assert np.allclose(r, r[0], rtol=1e-11)


def test_moment_scheme_span_and_robustness():
    """M = S Z (eq. MS) lies in span(S) (eq. ms).  With K L = 128 columns the moment scheme
    finds the QEP roots inside; with K = 4 (64 columns for 32 eigenvalues) it does not,
    while the sampling scheme on the same S does (the paper's robustness argument)."""
    nep, C, U = W.cfg_qep(n=200, N=32, L=16)
    prob = O.Problem(nep)
    ex = P.qep_roots(nep.extra["c"], nep.extra["k"])
    rm = O.rsrr_moment(prob, C, U, K=8, NQ=300)
    M, S = rm["M"], rm["S_sampled"]
    Qs, _, ks = O.basis(O.normalize(S), 1e-14)
    assert np.linalg.norm(M - Qs @ (Qs.conj().T @ M)) <= 1e-10 * np.linalg.norm(M)
    ins = rm["level"] < 0.98
    assert ins.sum() == 32 and _match(rm["lam"][ins], ex) < 1e-9
    assert rm["k"] <= 8 * 16
    r4 = O.rsrr_moment(prob, C, U, K=4, NQ=300)
    rs = O.rsrr(prob, C, U, NQ=300, S=S)
    i4, i_s = r4["level"] < 0.98, rs["level"] < 0.98
    assert _match(r4["lam"][i4], ex) > 1e-6
    assert _match(rs["lam"][i_s], ex) < 1e-9


def test_real_sampling_on_chebyshev_points_finds_the_string_eigenvalues():
    """Real sampling (Sec. 5.1, Example 1): Chebyshev points of the interval [3, 10000] and
    real probes make S real; SS-RR on it finds the 32 eigenvalues of the loaded string in
    the interval (the paper's count) with residuals below 1e-10."""
    g = json.load(open(os.path.join(HERE, "golden", "loaded_string.json")))
    nep = W.loaded_string(g["n"])
    prob = O.Problem(nep)
    lo, hi = g["interval"]
    z = W.interval_points(lo, hi, 48)
    assert np.all(z.imag == 0) and np.allclose(np.sort(z.real), np.sort((lo + hi) / 2 + (hi - lo) / 2 * O.chebyshev_points(48)))
    U = W.real_probes(g["n"], 2, 78)
    S = O.sample(prob, z, U)
    assert np.max(np.abs(S.imag)) == 0.0
    a = g["contour"]["a"]
    C = W.Contour(g["contour"]["gamma"] + 0j, a, a * g["contour"]["b_over_a"], 64)
    r = O.rsrr(prob, C, U, NQ=500, S=S)
    lam = r["lam"]
    sel = (lam.real >= lo) & (lam.real <= hi) & (r["level"] < 1) & (r["res"] < 1e-10)
    assert int(sel.sum()) == g["count"]


# -------------------------------------------------------- sparse storage ----

def _random_csr(seed, n=40):
    """A CSR matrix with unsorted columns and repeated (row, column) pairs."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 8, n)
    indptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    indices = rng.integers(0, n // 4, indptr[-1]).astype(np.int32)
    data = W.complex_gaussian(rng, indptr[-1])
    return indptr, indices, data


def test_csr_dense_sums_repeated_entries_like_scipy():
    """csr_dense against SciPy's own CSR-to-dense conversion (which sums repeats)."""
    from scipy import sparse
    ip, ix, d = _random_csr(77)
    n = ip.size - 1
    rows = np.repeat(np.arange(n), np.diff(ip))
    assert np.unique(np.stack([rows, ix]), axis=1).shape[1] < ix.size  # repeats are present
    ref = sparse.csr_matrix((d, ix, ip), shape=(n, n)).toarray()
    got = O.csr_dense(ip, ix, d, n)
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
    # a slip: later repeats overwrite instead of adding
    slip = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for e in range(ip[i], ip[i + 1]):
            slip[i, ix[e]] = d[e]
    assert np.abs(slip - ref).max() > 1e-3


def test_sparse_delay_nep_is_the_dense_one():
    """The CSR generators give the matrices of the dense delay NEP (SciPy conversion), and the
    oracle's T(z) of the two forms agree."""
    from scipy import sparse
    sp, de = W.delay_laplacian_sparse((16, 32)), W.delay_laplacian(16, 32)
    for (ip, ix, d), A in zip(sp.csr, de.A):
        B = sparse.csr_matrix((d, ix, ip), shape=A.shape).toarray()
        assert np.abs(B - A).max() <= 1e-12 * np.abs(A).max()
    ps, pd = O.Problem(sp), O.Problem(de)
    for z in (-4.2 + 0.3j, -3.5 - 0.1j):
        assert np.abs(ps.T(z) - pd.T(z)).max() <= 1e-12 * np.abs(pd.T(z)).max()
        assert np.abs(ps.dT(z) - pd.dT(z)).max() <= 1e-12 * np.abs(pd.dT(z)).max()


def test_laplacian_3d_csr_spectrum_closed_form():
    """7-point Dirichlet Laplacian on a 6 x 5 x 4 grid: symmetric, with the eigenvalues
    sum_d -(4/h_d^2) sin^2(p pi h_d / 2)."""
    from scipy import sparse
    ip, ix, d = W.laplacian_csr((6, 5, 4))
    A = sparse.csr_matrix((d, ix, ip), shape=(120, 120)).toarray().real
    assert np.array_equal(A, A.T)
    ex = np.sort(W.laplacian_modes_nd((6, 5, 4)))
    assert np.abs(np.linalg.eigvalsh(A) - ex).max() <= 1e-10 * np.abs(ex).max()
    assert np.all(np.diff(ip) <= 7) and np.all(np.diff(ip) >= 4)
