"""Independent checks that pin the oracle to mathematics other than itself.

TEST INFRASTRUCTURE ONLY (imported by the tests).  Nothing here reuses the
RSRR steps of ``rsrr_oracle``: these are closed forms, textbook reductions and
brute-force root finding that the oracle's answers must agree with.

* ``qep_roots``            roots of z^2 + c_i z + k_i (rotated diagonal QEP).
* ``delay_eigs``           delay NEP -z + mu + a1 e^{-z} = 0 per Laplacian mode,
                           all Lambert-W branches, by Newton in log space.
* ``companion_eigs``       quadratic NEP A0 + z A1 + z^2 A2 through its first
                           companion linearisation and LAPACK's QZ.
* ``argument_count``       (1/2 pi i) \\oint tr(T^-1 T') dz, the number of
                           eigenvalues inside a contour (argument principle).
* ``det_newton_roots``     Newton on det T(z) with d/dz log det T = tr(T^-1 T')
                           from a grid of seeds, for tiny n.
"""
from __future__ import annotations

import cmath
import math

import numpy as np
import scipy.linalg as sla


def qep_roots(c, k):
    """All 2n roots (-c_i +- sqrt(c_i^2 - 4 k_i)) / 2."""
    c = np.asarray(c, dtype=np.complex128)
    k = np.asarray(k, dtype=np.complex128)
    d = np.sqrt(c * c - 4.0 * k)
    return np.concatenate([(-c + d) / 2.0, (-c - d) / 2.0])


def _delay_branch(mu, a1, branch):
    """Solve lambda = mu + w, w e^w = a1 e^{-mu}, on Lambert-W branch ``branch``.

    With log: w + log w = log(a1) - mu + 2 pi i branch; Newton on
    g(w) = w + log w - rhs from w0 = rhs - log(rhs) (asymptotic start), then a
    polish of -lambda + mu + a1 e^{-lambda} = 0 when the exponential is finite.
    """
    rhs = complex(math.log(a1) - mu, 2.0 * math.pi * branch)
    w = rhs - cmath.log(rhs) if abs(rhs) > 1.0 else complex(0.5, 0.5 * branch)
    for _ in range(100):
        g = w + cmath.log(w) - rhs
        dw = g / (1.0 + 1.0 / w)
        w -= dw
        if abs(dw) <= 1e-16 * max(1.0, abs(w)):
            break
    lam = mu + w
    for _ in range(5):
        try:
            e = a1 * cmath.exp(-lam)
        except OverflowError:
            break
        f = -lam + mu + e
        df = -1.0 - e
        step = f / df
        lam -= step
        if abs(step) <= 1e-16 * max(1.0, abs(lam)):
            break
    return lam


def delay_eigs(modes, a1=0.5, branches=range(-3, 4)):
    """Eigenvalues of -z I + A0 + a1 e^{-z} I for the given A0 eigenvalues (all listed branches).

    Branch 0 with a1 e^{-mu} > 0 is real; duplicates from the same branch are
    not removed (each mode contributes one eigenvalue per branch).
    """
    out = []
    for mu in np.asarray(modes, dtype=np.float64):
        for br in branches:
            out.append(_delay_branch(float(mu), a1, br))
    return np.array(out, dtype=np.complex128)


def companion_eigs(A0, A1, A2):
    """Eigenvalues of A0 + z A1 + z^2 A2 via [[0, I], [-A0, -A1]] v = z [[I, 0], [0, A2]] v."""
    n = A0.shape[0]
    Z = np.zeros((n, n), dtype=np.complex128)
    I = np.eye(n, dtype=np.complex128)
    AA = np.block([[Z, I], [-A0, -A1]])
    BB = np.block([[I, Z], [Z, A2]])
    ev = sla.eig(AA, BB, right=False)
    return ev[np.isfinite(ev)]


def argument_count(Tfun, dTfun, gamma, a, b, M=1024):
    """(1/2 pi i) \\oint tr(T(z)^-1 T'(z)) dz on the ellipse, M-point trapezoid rule."""
    t = 2.0 * math.pi * (np.arange(M) + 0.5) / M
    z = gamma + a * np.cos(t) + 1j * b * np.sin(t)
    dz = (-a * np.sin(t) + 1j * b * np.cos(t)) * (2.0 * math.pi / M)
    acc = 0j
    for zi, dzi in zip(z, dz):
        X = np.linalg.solve(Tfun(zi), dTfun(zi))
        acc += np.trace(X) * dzi
    return acc / (2j * math.pi)


def det_newton_roots(Tfun, dTfun, seeds, tol=1e-13, maxit=60):
    """Newton on det T: z <- z - 1 / tr(T^-1 T'); converged roots, deduplicated."""
    roots = []
    for z in seeds:
        z = complex(z)
        ok = False
        for _ in range(maxit):
            try:
                tr = np.trace(np.linalg.solve(Tfun(z), dTfun(z)))
            except np.linalg.LinAlgError:
                ok = True
                break
            if tr == 0:
                break
            step = 1.0 / tr
            z -= step
            if abs(step) <= tol * max(1.0, abs(z)):
                ok = True
                break
        if ok and np.isfinite(z):
            if all(abs(z - r) > 1e-8 * max(1.0, abs(r)) for r in roots):
                roots.append(z)
    return np.array(roots, dtype=np.complex128)
