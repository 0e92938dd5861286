"""Plain, slow CPU FP64 oracle of the RSRR method (Xiao, Zhang, Huang, Sakurai).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP
library: it evaluates T(z) itself, solves with LAPACK through SciPy, takes the
SVD from NumPy and follows the paper's steps in the paper's order.

Steps and the passages they follow
----------------------------------
* ``ellipse``          Sec. 5.1, eq. ellip-contour and eq. ellip-contour-xw
                       (nodes z_i = phi(alpha_j), trapezoid weights phi'/N).
* ``coef``             the separable form T(z) = sum_j f_j(z) A_j of Sec. 2.1.
* ``T_separable``, ``T_helmholtz``
                       T(z) for the two families (eq. QEP / eq. REP-string /
                       the delay form; the single-layer kernel of eq. nyes).
* ``csr_dense``        the dense matrix of a compressed-sparse-row matrix (the
                       storage of the finite-element models of Sec. 4.3 and
                       Sec. 6); a sparse NEP is the separable form with its
                       A_j given that way and is evaluated densely here.
* ``sample``           RSRR Step 2 and eq. hatS: S = [T(z_0)^-1 U, ...].
                       This is a plain definition (the unique solution of
                       each linear system), computed by zgetrf/zgetrs.
* ``normalize``        Sec. 4.2: columns of S scaled to one norm before the SVD.
* ``basis``            RSRR Step 3: truncated SVD S ~ Q Sigma V^H keeping the
                       singular values larger than delta*sigma_1 (delta 1e-14,
                       Sec. 4.3).
* ``project``          RSRR Step 4 / eq. Ts-NEP: T_Q(z) = Q^H T(z) Q.
* ``ss_full``          Sec. 3.3 (SS-RI with U dropped, i.e. SS-FULL): moments
                       eq. Aalpha-rat with F = T_Q^-1, block Hankel pencils
                       eq. HH, truncated SVD eq. svdH with the gap rule eq. gap,
                       the reduced matrix eq. A and the lift eq. eigens.
* ``rsrr``             the five steps of Sec. 4.3 chained together.
* ``barycentric_weights``, ``chebyshev_points``, ``chebyshev_weights``
                       eq. bary-wt (with each factor divided by a capacity C, the
                       scaling Sec. 3.3 suggests against under- and overflow),
                       eq. Chebyshev-pts and eq. Chebyshev-wts.
* ``moments``          the resolvent moment scheme, Sec. 4.1: M_alpha =
                       sum_i omega_i zeta_i^alpha T(z_i)^-1 U (eq. Malpha) for
                       alpha < K, collected as M = [M_0 ... M_{K-1}] (eq. M-pr),
                       i.e. M = S Z (eq. MS).
* ``rsrr_moment``      SS-RR with M in place of S (the variant Sec. 4.3 describes
                       in its closing remark).
* ``two_stage``        the two-stage strategy of Sec. 5.4 (Example 2, the gun
                       cavity) and Sec. 6 (Example 3): RSRR on a few contour points, then the
                       distinct eigenvalue estimates inside the contour become
                       extra sampling points; the first-stage columns of S are
                       kept and RSRR runs again on all of them.
* ``residual``         the relative residual of an eigenpair (Sec. 3.3 and
                       Sec. 5.1: ||T(lambda) v||_2 / ||v||_2), here further
                       divided by ||T(lambda)||_1.

Readings of passages that are silent or garbled
-----------------------------------------------
* Moments use the shifted and scaled variable zeta = (z - gamma)/rho with
  rho = max(a, b) instead of the raw z^alpha of eq. Aalpha-rat; the pencil
  eigenvalues mu map back as lambda = gamma + rho*mu.  A shift and a scale
  of the variable leave the spans and the pencil eigenvalues unchanged, and
  avoid the overflow the paper warns about for the weights (Sec. 3.3).
* The trapezoid weight is phi'(alpha_j)/N for node j; the 1/(2 pi i) factor
  is omitted because a common factor cancels in the pencil (Sec. 3.3).
* Eigenpairs: (lambda, M W0 Sigma0^-1 b) for SS-RI and (lambda, Q g) for RSRR
  (the printed "(v, ...)" and "(lambda, S g)" are taken as typos).
* Gap edge cases: a zero sigma_{j+1} makes the ratio infinite and selects j;
  g_max below tol_gap returns the best-effort count with ``warn_gap=True``.
* The eigenvalues of the reduced matrix are all returned with their elliptic
  level |((z-gamma)/a).real|^2 + |((z-gamma)/b).imag|^2 ... (see ``level``);
  callers decide which are inside.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import scipy.linalg as sla

EPS = np.finfo(np.float64).eps


# ---------------------------------------------------------------------------
# Step 1: contour, nodes and weights
# ---------------------------------------------------------------------------

def ellipse(gamma, a, b, N):
    """Nodes and trapezoid weights on phi(t) = gamma + a cos t + i b sin t (Sec. 5.1).

    alpha_j = 2 pi (j + 1/2) / N, z_j = phi(alpha_j), w_j = phi'(alpha_j) / N.
    """
    j = np.arange(N, dtype=np.float64)
    alpha = 2.0 * math.pi * (j + 0.5) / N
    z = complex(gamma) + a * np.cos(alpha) + 1j * b * np.sin(alpha)
    w = (-a * np.sin(alpha) + 1j * b * np.cos(alpha)) / N
    return z.astype(np.complex128), w.astype(np.complex128)


def level(z, gamma, a, b):
    """Elliptic level of z: < 1 strictly inside the ellipse, 1 on it."""
    d = np.asarray(z) - gamma
    return (d.real / a) ** 2 + (d.imag / b) ** 2


# ---------------------------------------------------------------------------
# T(z) for the separable and the Helmholtz families
# ---------------------------------------------------------------------------

def coef(t, z):
    """f(z) = c (z - z0)^p exp(-tau z) / (z - s)^q for one term dict."""
    z = complex(z)
    v = t["c"] * (z - t["z0"]) ** t["p"]
    if t["tau"] != 0.0:
        v *= cmath.exp(-t["tau"] * z)
    if t["q"] != 0:
        v /= (z - t["s"]) ** t["q"]
    return v


def coef_deriv(t, z):
    """Derivative f'(z) of one term, by the product rule."""
    z = complex(z)
    f = coef(t, z)
    if f == 0:
        # only possible for c == 0 or a root of (z - z0)^p; differentiate directly
        if t["c"] == 0:
            return 0j
        p = t["p"]
        if p == 1:
            v = t["c"]
            if t["tau"] != 0.0:
                v *= cmath.exp(-t["tau"] * z)
            if t["q"] != 0:
                v /= (z - t["s"]) ** t["q"]
            return v
        return 0j
    logd = 0j
    if t["p"] != 0:
        logd += t["p"] / (z - t["z0"])
    logd += -t["tau"]
    if t["q"] != 0:
        logd += -t["q"] / (z - t["s"])
    return f * logd


def T_separable(A, terms, z):
    """T(z) = sum_j f_j(z) A_j."""
    T = np.zeros_like(A[0])
    for Aj, t in zip(A, terms):
        T += coef(t, z) * Aj
    return T


def dT_separable(A, terms, z):
    """T'(z) = sum_j f_j'(z) A_j."""
    T = np.zeros_like(A[0])
    for Aj, t in zip(A, terms):
        T += coef_deriv(t, z) * Aj
    return T


def csr_dense(indptr, indices, data, n):
    """The dense n x n matrix of a compressed-sparse-row matrix: row i holds the
    entries indptr[i] .. indptr[i+1]-1, entry e at column indices[e] with value
    data[e]; a repeated (row, column) pair is summed."""
    A = np.zeros((n, n), dtype=np.complex128)
    for i in range(n):
        for e in range(int(indptr[i]), int(indptr[i + 1])):
            A[i, int(indices[e])] += data[e]
    return A


def _distances(points):
    diff = points[:, None, :] - points[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=2))


def T_helmholtz(points, w, z, r=None):
    """Single-layer Helmholtz Nystrom matrix on a point set (kernel of eq. nyes).

    T_ij = w exp(i z r_ij) / (4 pi r_ij) for i != j and
    T_ii = sqrt(w/pi)/2 + i z w / (4 pi).
    """
    if r is None:
        r = _distances(points)
    n = points.shape[0]
    z = complex(z)
    with np.errstate(divide="ignore", invalid="ignore"):
        T = w * np.exp(1j * z * r) / (4.0 * math.pi * r)
    T[np.arange(n), np.arange(n)] = math.sqrt(w / math.pi) / 2.0 + 1j * z * w / (4.0 * math.pi)
    return T


def dT_helmholtz(points, w, z, r=None):
    """d/dz of ``T_helmholtz``: w i exp(i z r)/(4 pi) off the diagonal, i w/(4 pi) on it."""
    if r is None:
        r = _distances(points)
    n = points.shape[0]
    z = complex(z)
    D = w * 1j * np.exp(1j * z * r) / (4.0 * math.pi)
    D[np.arange(n), np.arange(n)] = 1j * w / (4.0 * math.pi)
    return D


class Problem:
    """A NEP seen through T(z) (and T'(z)) only, for either family."""

    def __init__(self, nep):
        self.nep = nep
        if hasattr(nep, "A"):
            self.kind = "separable"
            self.n = nep.A[0].shape[0]
            self._A = nep.A
        elif hasattr(nep, "csr"):
            # the sparse form is the separable one with its matrices stored by rows
            self.kind = "separable"
            self.n = nep.n
            self._A = [csr_dense(ip, ix, d, nep.n) for ip, ix, d in nep.csr]
        else:
            self.kind = "helmholtz"
            self.n = nep.points.shape[0]
            self._r = _distances(nep.points)

    def T(self, z):
        if self.kind == "separable":
            return T_separable(self._A, self.nep.terms, z)
        return T_helmholtz(self.nep.points, self.nep.w, z, self._r)

    def dT(self, z):
        if self.kind == "separable":
            return dT_separable(self._A, self.nep.terms, z)
        return dT_helmholtz(self.nep.points, self.nep.w, z, self._r)


# ---------------------------------------------------------------------------
# Step 2: resolvent sampling (eq. hatS)
# ---------------------------------------------------------------------------

def solve_point(T, U):
    """X = T^-1 U by LU with partial pivoting (zgetrf + zgetrs)."""
    lu, piv = sla.lu_factor(T, check_finite=True)
    return sla.lu_solve((lu, piv), U)


def sample(prob, z, U):
    """S = [T(z_0)^-1 U, ..., T(z_{N-1})^-1 U]  (n x N*L), block k = point k."""
    blocks = [solve_point(prob.T(zk), U) for zk in z]
    return np.concatenate(blocks, axis=1)


# ---------------------------------------------------------------------------
# Step 3: normalisation and the truncated SVD
# ---------------------------------------------------------------------------

def normalize(S):
    """Scale every column of S to unit 2-norm (Sec. 4.2); zero columns stay zero."""
    nrm = np.linalg.norm(S, axis=0)
    nrm[nrm == 0] = 1.0
    return S / nrm[None, :]


def basis(S, delta=1e-14):
    """Truncated SVD S ~ Q Sigma V^H keeping sigma_i > delta*sigma_1 (RSRR Step 3).

    Returns (Q, sigma, k) with Q the first k left singular vectors.
    """
    W, sig, _ = np.linalg.svd(S, full_matrices=False)
    if sig.size == 0 or sig[0] == 0.0:
        return W[:, :0], sig, 0
    k = int(np.sum(sig > delta * sig[0]))
    return W[:, :k], sig, k


# ---------------------------------------------------------------------------
# Step 4: projection and SS-FULL on the projected NEP
# ---------------------------------------------------------------------------

def project(prob, Q):
    """T_Q as a callable z -> Q^H T(z) Q (eq. Ts-NEP).

    For a separable T the projected coefficients Q^H A_j Q are formed once; for
    the Helmholtz family T(z) is evaluated at each requested z and projected.
    """
    QH = Q.conj().T
    if prob.kind == "separable":
        AQ = [QH @ Aj @ Q for Aj in prob._A]
        terms = prob.nep.terms

        def TQ(z):
            return T_separable(AQ, terms, z)
        TQ.AQ = AQ
        return TQ

    def TQh(z):
        return QH @ prob.T(z) @ Q
    return TQh


def ss_full(TQ, k, gamma, a, b, NQ=500, KQ=2, tol_gap=1e3):
    """SS-FULL (Sec. 3.3): SS-RI with F(z) = T_Q(z)^-1, nodes on the ellipse.

    Returns a dict with the eigenvalues ``lam``, the reduced eigenvectors
    ``G`` (k x m, one column per eigenvalue, unit norm), the singular values of
    H, the count n_C, g_max and the gap warning flag.
    """
    gamma = complex(gamma)
    rho = max(a, b)
    z, w = ellipse(gamma, a, b, NQ)
    zeta = (z - gamma) / rho
    # Step 3: moments A_alpha = sum_i w_i zeta_i^alpha F(z_i), alpha < 2K
    Amom = [np.zeros((k, k), dtype=np.complex128) for _ in range(2 * KQ)]
    I = np.eye(k, dtype=np.complex128)
    for zi, wi, zti in zip(z, w, zeta):
        F = solve_point(TQ(zi), I)
        p = wi
        for al in range(2 * KQ):
            Amom[al] += p * F
            p *= zti
    # Step 4: block Hankel matrices (eq. HH) and M = [M_0 ... M_{K-1}], M_a = A_a
    H = np.block([[Amom[i + j] for j in range(KQ)] for i in range(KQ)])
    Hs = np.block([[Amom[i + j + 1] for j in range(KQ)] for i in range(KQ)])
    M = np.concatenate([Amom[al] for al in range(KQ)], axis=1)
    # Step 5: SVD of H and the gap rule (eq. gap)
    V, sig, WH = np.linalg.svd(H)
    m = sig.size
    with np.errstate(divide="ignore", invalid="ignore"):
        ratios = np.where(sig[1:] == 0.0, np.inf, sig[:-1] / np.where(sig[1:] == 0.0, 1.0, sig[1:]))
    if m < 2 or sig[0] == 0.0:
        return {"lam": np.zeros(0, complex), "G": np.zeros((k, 0), complex), "sigma_H": sig,
                "nbar": 0, "gmax": 0.0, "warn_gap": True}
    jmax = int(np.argmax(ratios))
    gmax = float(ratios[jmax])
    nbar = jmax + 1
    warn = gmax < tol_gap
    V0 = V[:, :nbar]
    W0 = WH.conj().T[:, :nbar]
    S0inv = 1.0 / sig[:nbar]
    # Step 6: A = V0^H H^< W0 Sigma0^-1 and its eigenpairs (eq. A, eq. eigens)
    Ared = (V0.conj().T @ Hs @ W0) * S0inv[None, :]
    mu, B = sla.eig(Ared)
    lam = gamma + rho * mu
    G = M @ (W0 * S0inv[None, :]) @ B
    nrm = np.linalg.norm(G, axis=0)
    nrm[nrm == 0] = 1.0
    G = G / nrm[None, :]
    return {"lam": lam, "G": G, "sigma_H": sig, "nbar": nbar, "gmax": gmax, "warn_gap": bool(warn)}


# ---------------------------------------------------------------------------
# Residuals and the whole method
# ---------------------------------------------------------------------------

def residual(prob, lam, v):
    """||T(lambda) v||_2 / (||T(lambda)||_1 ||v||_2)."""
    T = prob.T(lam)
    return float(np.linalg.norm(T @ v) / (np.linalg.norm(T, 1) * np.linalg.norm(v)))


def rsrr(prob, contour, U, delta=1e-14, NQ=500, KQ=2, tol_gap=1e3, S=None):
    """RSRR (Sec. 4.3): sample, normalise, truncate, project, SS-FULL, lift.

    ``contour`` has fields gamma, a, b, N.  Returns a dict with the eigenvalues,
    eigenvectors (n x m, unit columns), their levels and residuals, k, the
    singular values of S and the SS-FULL diagnostics.
    """
    z, _ = ellipse(contour.gamma, contour.a, contour.b, contour.N)
    if S is None:
        S = sample(prob, z, U)
    Sn = normalize(S)
    Q, sigS, k = basis(Sn, delta)
    TQ = project(prob, Q)
    ss = ss_full(TQ, k, contour.gamma, contour.a, contour.b, NQ=NQ, KQ=KQ, tol_gap=tol_gap)
    V = Q @ ss["G"]
    res = np.array([residual(prob, l, V[:, i]) for i, l in enumerate(ss["lam"])])
    return {"lam": ss["lam"], "V": V, "level": level(ss["lam"], contour.gamma, contour.a, contour.b),
            "res": res, "k": k, "sigma_S": sigS, "ss": ss, "z": z, "S": S, "Q": Q}


def distinct_inside(lam, gamma, a, b, rel=1e-6):
    """Eigenvalue estimates inside the ellipse (level < 1), in the given order, without
    those closer than rel*max(1, |lambda|) to one already taken (reading: the paper
    keeps the mutually different estimates)."""
    out = []
    for l in lam[level(lam, gamma, a, b) < 1]:
        if all(abs(l - m) > rel * max(1.0, abs(l)) for m in out):
            out.append(l)
    return np.array(out, dtype=np.complex128)


def two_stage(prob, contour, U, delta=1e-14, NQ=500, KQ=2, tol_gap=1e3):
    """Two-stage RSRR (Sec. 5.4, Example 2; Sec. 6, Example 3): stage 1 on contour.N points,
    stage 2 with the stage-1 estimates inside the contour appended as sampling points
    (their T(z)^-1 U appended to the stage-1 S, which is reused)."""
    r1 = rsrr(prob, contour, U, delta=delta, NQ=NQ, KQ=KQ, tol_gap=tol_gap)
    znew = distinct_inside(r1["lam"], contour.gamma, contour.a, contour.b)
    S2 = np.hstack([r1["S"], sample(prob, znew, U)]) if znew.size else r1["S"]
    r2 = rsrr(prob, contour, U, delta=delta, NQ=NQ, KQ=KQ, tol_gap=tol_gap, S=S2)
    r2["z"] = np.concatenate([r1["z"], znew])
    return r1, r2, znew


# ---------------------------------------------------------------------------
# Interpolation weights and the moment scheme
# ---------------------------------------------------------------------------

def barycentric_weights(z, capacity=1.0):
    """omega_i = 1 / prod_{j != i} ((z_i - z_j) / C) (eq. bary-wt with every factor scaled by
    1/C), the product taken as a sum of logarithms."""
    z = np.asarray(z, dtype=np.complex128)
    w = np.empty(z.size, dtype=np.complex128)
    for i in range(z.size):
        d = np.delete(z[i] - z, i) / capacity
        w[i] = np.exp(-np.sum(np.log(d)))
    return w


def chebyshev_points(N):
    """Chebyshev points of the first kind on [-1, 1] (eq. Chebyshev-pts)."""
    i = np.arange(N)
    return np.cos((2 * i + 1) * np.pi / (2 * N))


def chebyshev_weights(N):
    """Their simplified barycentric weights (eq. Chebyshev-wts)."""
    i = np.arange(N)
    return (-1.0) ** i * np.sin((2 * i + 1) * np.pi / (2 * N))


def moments(S, z, L, K, gamma, rho, capacity):
    """M = [M_0 ... M_{K-1}], M_alpha = sum_i omega_i zeta_i^alpha X_i with X_i the i-th block
    of S, zeta = (z - gamma)/rho and omega the barycentric weights of the zeta_i
    (eq. Malpha, eq. M-pr; reading: the shifted and scaled variable as for SS-FULL)."""
    zeta = (np.asarray(z) - gamma) / rho
    w = barycentric_weights(zeta, capacity)
    n = S.shape[0]
    M = np.zeros((n, K * L), dtype=np.complex128)
    for a in range(K):
        for i, zi in enumerate(zeta):
            M[:, a * L:(a + 1) * L] += w[i] * zi ** a * S[:, i * L:(i + 1) * L]
    return M


def rsrr_moment(prob, contour, U, K, delta=1e-14, NQ=500, KQ=2, tol_gap=1e3):
    """SS-RR with the moment matrix M in place of S (Steps 3-5 on M)."""
    z, _ = ellipse(contour.gamma, contour.a, contour.b, contour.N)
    S = sample(prob, z, U)
    rho = max(contour.a, contour.b)
    M = moments(S, z, U.shape[1], K, contour.gamma, rho, (contour.a + contour.b) / (2 * rho))
    r = rsrr(prob, contour, U, delta=delta, NQ=NQ, KQ=KQ, tol_gap=tol_gap, S=M)
    r["M"] = M
    r["S_sampled"] = S
    return r

