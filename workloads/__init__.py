"""Seeded synthetic NEP instances shared by the tests, the benchmark and the oracle.

This module only *builds inputs*: coefficient matrices, collocation points,
probe matrices and contour parameters.  It holds none of the RSRR arithmetic
(no assembly of T(z), no solves, no SVD, no projection), so both the HIP path
and the CPU oracle can take their inputs from it without sharing any step of
the method.

Every NEP here is in the separable form T(z) = sum_j f_j(z) A_j of the paper's
problem statement (Sec. 2.1, eq. gnep and the examples eq. QEP, eq.
REP-string), except the Helmholtz single-layer problem, whose entries are a
kernel of the distance (Sec. 2.1, eq. nyes) and which is described by its
points and quadrature weight only.

A scalar coefficient f_j is given as a *term*: the dict
``{"c": c, "p": p, "z0": z0, "tau": tau, "s": s, "q": q}`` meaning

    f(z) = c * (z - z0)**p * exp(-tau * z) / (z - s)**q .

Every example of Sec. 2.1 that the build covers fits this form (polynomial,
rational and delay terms).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def term(c=1.0, p=0, z0=0.0, tau=0.0, s=0.0, q=0):
    return {"c": complex(c), "p": int(p), "z0": complex(z0), "tau": float(tau),
            "s": complex(s), "q": int(q)}


@dataclass
class Contour:
    """Ellipse gamma + a cos(t) + i b sin(t) sampled at N trapezoid nodes (Sec. 5.1, eq. ellip-contour)."""
    gamma: complex
    a: float
    b: float
    N: int


@dataclass
class SeparableNEP:
    name: str
    A: list            # list of J dense (n, n) complex128 arrays
    terms: list        # list of J term dicts
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.A[0].shape[0]

    @property
    def J(self):
        return len(self.A)


@dataclass
class HelmholtzNEP:
    name: str
    points: np.ndarray  # (n, 3) float64, unit sphere
    w: float            # area weight per point (4 pi / n)

    @property
    def n(self):
        return self.points.shape[0]


@dataclass
class SparseNEP:
    """T(z) = sum_j f_j(z) A_j with every A_j in compressed sparse row form.

    ``csr[j] = (indptr, indices, data)``: int32 row pointers (n+1), int32
    column indices and complex128 values (nnz each); row i holds the entries
    indptr[i] .. indptr[i+1]-1.
    """
    name: str
    n: int
    csr: list
    terms: list
    extra: dict = field(default_factory=dict)

    @property
    def J(self):
        return len(self.csr)


def complex_gaussian(rng, shape):
    """(N(0,1) + i N(0,1)) / sqrt(2) entries."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)


def haar_unitary(rng, n):
    """Haar-distributed unitary: QR of a complex Gaussian with the phases of diag(R) folded in."""
    G = complex_gaussian(rng, (n, n))
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


def rotated_diagonal_qep(n, seed, c_range=(0.1, 0.5), k_range=(1.0, 100.0)):
    """T(z) = Q^H (z^2 I + z C + K) Q with C, K diagonal and Q a seeded Haar unitary.

    Quadratic eigenvalue problem of Sec. 2.1 (eq. QEP, M = I).  Draw order from
    ``default_rng(seed)``: c, then k, then the Gaussian for Q.  The closed-form
    eigenvalues are the roots of z^2 + c_i z + k_i, eigenvectors Q^H e_i.
    """
    rng = np.random.default_rng(seed)
    c = rng.uniform(c_range[0], c_range[1], n)
    k = rng.uniform(k_range[0], k_range[1], n)
    Q = haar_unitary(rng, n)
    QH = Q.conj().T
    A0 = (QH * k[None, :]) @ Q          # Q^H K Q
    A1 = (QH * c[None, :]) @ Q          # Q^H C Q
    A2 = np.eye(n, dtype=np.complex128)
    nep = SeparableNEP(
        name=f"qep_rotdiag_n{n}_s{seed}",
        A=[np.ascontiguousarray(A0), np.ascontiguousarray(A1), A2],
        terms=[term(1.0, 0), term(1.0, 1), term(1.0, 2)],
        extra={"c": c, "k": k, "Q": Q, "rng": rng},
    )
    return nep


def dirichlet_laplacian_2d(nx, ny):
    """5-point Dirichlet Laplacian on an nx-by-ny interior grid of the unit square, scaled by 1/h^2.

    Lexicographic ordering (x fastest), h_x = 1/(nx+1), h_y = 1/(ny+1); the matrix
    is negative definite.  Returns a dense float64 array.
    """
    hx = 1.0 / (nx + 1)
    hy = 1.0 / (ny + 1)
    Tx = (np.diag(-2.0 * np.ones(nx)) + np.diag(np.ones(nx - 1), 1) + np.diag(np.ones(nx - 1), -1)) / hx**2
    Ty = (np.diag(-2.0 * np.ones(ny)) + np.diag(np.ones(ny - 1), 1) + np.diag(np.ones(ny - 1), -1)) / hy**2
    return np.kron(np.eye(ny), Tx) + np.kron(Ty, np.eye(nx))


def delay_laplacian(nx, ny=None, a1=0.5):
    """Delay NEP T(z) = -z I + A0 + a1 e^{-z} I, A0 the scaled 2D Dirichlet Laplacian.

    Terms: A0 with f=1, I with f=-z, a1*I with f=e^{-z}.  Eigenvalues per
    Laplacian mode mu are mu + W_k(a1 e^{-mu}) (Lambert W, all branches).
    """
    ny = nx if ny is None else ny
    n = nx * ny
    A0 = dirichlet_laplacian_2d(nx, ny).astype(np.complex128)
    I = np.eye(n, dtype=np.complex128)
    nep = SeparableNEP(
        name=f"delay_lap_{nx}x{ny}",
        A=[A0, I, a1 * I],
        terms=[term(1.0, 0), term(-1.0, 1), term(1.0, 0, tau=1.0)],
        extra={"nx": nx, "ny": ny, "a1": a1},
    )
    return nep


def laplacian_modes(nx, ny):
    """Eigenvalues of the scaled Dirichlet Laplacian (closed form), with their (p, q) labels."""
    hx = 1.0 / (nx + 1)
    hy = 1.0 / (ny + 1)
    p = np.arange(1, nx + 1)
    q = np.arange(1, ny + 1)
    mx = -(4.0 / hx**2) * np.sin(p * math.pi * hx / 2) ** 2
    my = -(4.0 / hy**2) * np.sin(q * math.pi * hy / 2) ** 2
    return (my[:, None] + mx[None, :]).ravel()


def laplacian_csr(dims):
    """Dirichlet Laplacian on the interior grid of the unit square (2 dims, 5 points)
    or cube (3 dims, 7 points), 1/h^2 scaled, in CSR.

    Lexicographic order with the first dimension fastest (the order of
    ``dirichlet_laplacian_2d``); each row lists its entries in increasing column
    order.  Returns (indptr, indices, data) with complex128 data.
    """
    dims = tuple(int(d) for d in dims)
    h2 = [1.0 / (d + 1) ** 2 for d in dims]
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    n = int(np.prod(dims))
    indptr = np.zeros(n + 1, dtype=np.int32)
    indices, data = [], []
    diag = -2.0 * sum(1.0 / h for h in h2)
    for i in range(n):
        rem, coord = i, []
        for d in dims:
            coord.append(rem % d)
            rem //= d
        row = [(i, diag)]
        for a, d in enumerate(dims):
            if coord[a] > 0:
                row.append((i - strides[a], 1.0 / h2[a]))
            if coord[a] < d - 1:
                row.append((i + strides[a], 1.0 / h2[a]))
        row.sort()
        indices.extend(c for c, _ in row)
        data.extend(v for _, v in row)
        indptr[i + 1] = len(indices)
    return indptr, np.asarray(indices, dtype=np.int32), np.asarray(data, dtype=np.complex128)


def identity_csr(n, scale=1.0):
    return (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
            np.full(n, scale, dtype=np.complex128))


def delay_laplacian_sparse(dims, a1=0.5):
    """The delay NEP of ``delay_laplacian`` (-z I + A0 + a1 e^{-z} I) on a 2D or 3D
    grid, its three matrices in CSR (the storage of a finite-element model)."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    return SparseNEP(
        name="delay_lap_sparse_" + "x".join(str(d) for d in dims),
        n=n,
        csr=[laplacian_csr(dims), identity_csr(n), identity_csr(n, a1)],
        terms=[term(1.0, 0), term(-1.0, 1), term(1.0, 0, tau=1.0)],
        extra={"dims": dims, "a1": a1},
    )


def laplacian_modes_nd(dims):
    """Eigenvalues of the scaled Dirichlet Laplacian on a grid of any dimension (closed form)."""
    vals = np.zeros(1)
    for d in dims:
        h = 1.0 / (d + 1)
        m = -(4.0 / h**2) * np.sin(np.arange(1, d + 1) * math.pi * h / 2) ** 2
        vals = (vals[:, None] + m[None, :]).ravel()
    return vals


def fibonacci_sphere(n):
    """Fibonacci lattice on the unit sphere: z_i = 1-(2i+1)/n, phi_i = i*pi*(3-sqrt5)."""
    i = np.arange(n, dtype=np.float64)
    zc = 1.0 - (2.0 * i + 1.0) / n
    phi = i * math.pi * (3.0 - math.sqrt(5.0))
    rxy = np.sqrt(np.maximum(0.0, 1.0 - zc * zc))
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), zc], axis=1)


def helmholtz_sphere(n):
    """Single-layer Helmholtz Nystrom NEP on the unit sphere (kernel of Sec. 2.1, eq. nyes).

    Off-diagonal T_ij(z) = w exp(i z r_ij) / (4 pi r_ij); diagonal (flat disk
    self-patch of radius sqrt(w/pi)) sqrt(w/pi)/2 + i z w/(4 pi); w = 4 pi / n.
    """
    return HelmholtzNEP(name=f"helmholtz_sphere_n{n}", points=fibonacci_sphere(n), w=4.0 * math.pi / n)


def loaded_string(n):
    """Loaded string of Example 1 (Sec. 5.1): T(z) = K_s + z/(z-1) e_n e_n^T - z M (real symmetric).

    Reading: the last diagonal entry of K_s is n (a free end, matching the
    halved last diagonal entry of M).  The printed matrix shows 2n there, but
    with 2n the interval [3, 10000] holds 31 eigenvalues, not the 32 that the
    example states; with n it holds 32.
    """
    Ks = n * (2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1))
    Ks[n - 1, n - 1] = float(n)
    M = (4.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)) / (6.0 * n)
    M[n - 1, n - 1] = 2.0 / (6.0 * n)
    E = np.zeros((n, n))
    E[n - 1, n - 1] = 1.0
    return SeparableNEP(
        name=f"loaded_string_n{n}",
        A=[Ks.astype(np.complex128), E.astype(np.complex128), M.astype(np.complex128)],
        terms=[term(1.0, 0), term(1.0, 1, s=1.0, q=1), term(-1.0, 1)],
        extra={},
    )


def probes(n, L, seed):
    """Random probe matrix U (n x L) of the paper's Step 1, complex Gaussian / sqrt 2."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(complex_gaussian(rng, (n, L)))


def real_probes(n, L, seed):
    """Real probe matrix (standard normal) for real sampling of a real NEP, stored complex."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, L)).astype(np.complex128))


def interval_points(lo, hi, N):
    """Chebyshev points of the first kind mapped to the real interval [lo, hi] (complex dtype)."""
    i = np.arange(N)
    x = np.cos((2 * i + 1) * np.pi / (2 * N))
    return ((lo + hi) / 2 + (hi - lo) / 2 * x).astype(np.complex128)


# ---------------------------------------------------------------------------
# The benchmark configurations, with the readings of the paper-silent details.
# ---------------------------------------------------------------------------

def cfg_qep(n=200, N=32, L=16, seed=0, literal=False):
    """Rotated diagonal QEP, ellipse of semi-axes (4, 1); literal centre 5 (empty) or 5i (34 roots inside)."""
    nep = rotated_diagonal_qep(n, seed)
    U = np.asfortranarray(complex_gaussian(nep.extra["rng"], (n, L)))
    if literal:
        C = Contour(5.0 + 0j, 4.0, 1.0, N)
    else:
        C = Contour(0.0 + 5.0j, 4.0, 1.0, N)
    return nep, C, U


def cfg_delay(nx=32, ny=None, N=48, L=32, seed=1000, parity=True):
    """Delay Laplacian NEP; parity circle (-4, 0.75) or the throughput circle (-20, 15)."""
    nep = delay_laplacian(nx, ny)
    U = probes(nep.n, L, seed)
    C = Contour(-4.0 + 0j, 0.75, 0.75, N) if parity else Contour(-20.0 + 0j, 15.0, 15.0, N)
    return nep, C, U


def cfg_sparse(dims=(20, 20, 20), N=32, L=8, seed=5000):
    """Sparse delay NEP on a 3D grid (n = 8000 at 20^3), circle (-4, 0.75): the
    eigenvalues mu + W(a1 e^-mu) of the four lowest modes lie inside (one simple,
    one triple)."""
    nep = delay_laplacian_sparse(dims)
    U = probes(nep.n, L, seed)
    return nep, Contour(-4.0 + 0j, 0.75, 0.75, N), U


def cfg_helmholtz(n=4096, N=64, L=64, seed=2000):
    """Helmholtz sphere NEP, ellipse centre 3.8, semi-axes (1.4, 0.3)."""
    nep = helmholtz_sphere(n)
    U = probes(n, L, seed)
    return nep, Contour(3.8 + 0j, 1.4, 0.3, N), U


def cfg_batched_sizes(count=256, lo=64, hi=1024, seed=3000):
    """Per-instance sizes of the ragged batch: n ~ U{lo..hi} inclusive."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)


DELAY_GRIDS = {512: (16, 32), 1024: (32, 32), 2048: (32, 64)}


def cfg_serving_stream(count=2000, rate=20.0, seed=4000):
    """Seeded request stream of the serving workload.

    Poisson arrivals (rate per second), half delay NEPs (n in {512, 1024,
    2048}, grids 16x32, 32x32, 32x64; N=48, L=32) and half Helmholtz sphere
    NEPs (n in {2048, 4096, 8192}; N=64, L=64).  Contours are jittered by up to
    +-10% around the delay parity circle (-4, 0.75) and the Helmholtz ellipse
    (3.8; 1.4, 0.3).  Each entry: t (arrival, s), kind, n, grid, gamma, a, b,
    N, L, seed (of its probes).  Draw order per request: kind, size, three
    jitters; arrivals are drawn first for the whole stream.
    """
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        delay = rng.random() < 0.5
        if delay:
            n = int(rng.choice([512, 1024, 2048]))
            j = rng.uniform(-0.1, 0.1, 3)
            out.append({"t": float(t[i]), "kind": "delay", "n": n, "grid": DELAY_GRIDS[n],
                        "gamma": -4.0 * (1 + j[0]) + 0j, "a": 0.75 * (1 + j[1]), "b": 0.75 * (1 + j[1]),
                        "N": 48, "L": 32, "seed": seed + 1 + i})
        else:
            n = int(rng.choice([2048, 4096, 8192]))
            j = rng.uniform(-0.1, 0.1, 3)
            out.append({"t": float(t[i]), "kind": "helmholtz", "n": n, "grid": None,
                        "gamma": 3.8 * (1 + j[0]) + 0j, "a": 1.4 * (1 + j[1]), "b": 0.3 * (1 + j[2]),
                        "N": 64, "L": 64, "seed": seed + 1 + i})
    return out


def serving_nep(req):
    """The NEP of one serving-stream entry."""
    if req["kind"] == "delay":
        return delay_laplacian(*req["grid"])
    return helmholtz_sphere(req["n"])
