"""Thin Python binding of the C ABI in include/rsrr.h (argument marshalling only).

Every computation runs in the HIP library ``librsrr.so``; this module only
converts NumPy/PyTorch arguments to pointers and sizes, and raises when the
library is missing or a call fails.  Device memory is held in PyTorch CUDA
(HIP) tensors; matrices are column-major, which a row-major PyTorch tensor
of shape (cols, rows) provides (``colmajor``/``from_colmajor``).

Names follow the C ABI: ``rsrr_create``, ``rsrr_sample``, ``rsrr_basis``,
``rsrr_project``, ``rsrr_solve``, ``rsrr_contour``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsrr.so")

RSRR_OK = 0
RSRR_ESINGULAR = 1
RSRR_WARN_FALLBACK = 2
RSRR_WARN_GAP = 3
RSRR_ENOMEM = 4
RSRR_EDEVICE = 5
RSRR_ENOTCONV = 6
RSRR_ENAN = 7
RSRR_ETIMEOUT = 8
RSRR_ELIMIT = 9
RSRR_WARN_MORE = 10
RSRR_T_SEPARABLE = 0
RSRR_T_HELMHOLTZ = 1
RSRR_T_SPARSE = 2
RSRR_PREC_C128 = 0
RSRR_PREC_C64_IR = 1
RSRR_PREC_R32_IR = 2

STATUS_NAMES = {0: "OK", 1: "ESINGULAR", 2: "WARN_FALLBACK", 3: "WARN_GAP", 4: "ENOMEM", 5: "EDEVICE",
                6: "ENOTCONV", 7: "ENAN", 8: "ETIMEOUT", 9: "ELIMIT", 10: "WARN_MORE"}

EXPORTS = ["rsrr_create", "rsrr_destroy", "rsrr_contour", "rsrr_sample", "rsrr_sample_batched", "rsrr_basis",
           "rsrr_project", "rsrr_solve", "rsrr_last_timings", "rsrr_update_stats", "rsrr_version",
           "rsrr_two_stage", "rsrr_moments", "rsrr_server_create", "rsrr_server_submit", "rsrr_server_wait", "rsrr_server_stats",
           "rsrr_server_destroy", "rsrr_sample_gmres", "rsrr_options_init", "rsrr_set_options", "rsrr_get_options",
           "rsrr_moments_noalloc", "rsrr_server_footprint"]
RSRR_BATCH_GRAPH = 1
RSRR_BATCH_AUTOTUNE = 2
RSRR_SERVE_NO_BATCH = 1
RSRR_SERVE_SERIAL = 2


class RsrrTerm(C.Structure):
    _fields_ = [("c_re", C.c_double), ("c_im", C.c_double), ("p", C.c_int), ("z0_re", C.c_double),
                ("z0_im", C.c_double), ("tau", C.c_double), ("s_re", C.c_double), ("s_im", C.c_double),
                ("q", C.c_int)]


class RsrrCsr(C.Structure):
    _fields_ = [("nnz", C.c_int), ("pad", C.c_int), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


class RsrrNep(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_int), ("J", C.c_int), ("A", C.c_void_p), ("lda", C.c_int),
                ("terms", C.POINTER(RsrrTerm)), ("points", C.c_void_p), ("w", C.c_double),
                ("csr", C.POINTER(RsrrCsr))]


class RsrrGmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int), ("ref", C.c_int),
                ("resid", C.c_double), ("matrix_free", C.c_int), ("pad", C.c_int)]


class RsrrInstance(C.Structure):
    _fields_ = [("nep", RsrrNep), ("N", C.c_int), ("z", C.POINTER(C.c_double)), ("U", C.c_void_p), ("L", C.c_int),
                ("ldu", C.c_int), ("S", C.c_void_p), ("lds", C.c_int)]


class RsrrPointInfo(C.Structure):
    _fields_ = [("info", C.c_int), ("ir_iters", C.c_int), ("fallback", C.c_int), ("pad", C.c_int),
                ("resid", C.c_double)]


class RsrrSolveInfo(C.Structure):
    _fields_ = [("nbar", C.c_int), ("warn_gap", C.c_int), ("gmax", C.c_double), ("n_sigma", C.c_int),
                ("truncated", C.c_int)]


class RsrrTwoStageInfo(C.Structure):
    _fields_ = [("k1", C.c_int), ("count1", C.c_int), ("nbar1", C.c_int), ("n_new", C.c_int), ("k2", C.c_int),
                ("nbar2", C.c_int), ("resid1_max", C.c_double)]


class RsrrOptions(C.Structure):
    _fields_ = [("size", C.c_ulonglong), ("version", C.c_int), ("ir_max_iters", C.c_int),
                ("ir_max_iters_batched", C.c_int), ("basis_sketch_max", C.c_int), ("ir_tol", C.c_double),
                ("fallback_resid", C.c_double), ("delta", C.c_double), ("tol_gap", C.c_double)]


OPTION_FIELDS = [f for f, _ in RsrrOptions._fields_ if f not in ("size", "version")]


class RsrrServerConfig(C.Structure):
    _fields_ = [("device", C.c_int), ("prec", C.c_int), ("max_slots", C.c_int), ("flags", C.c_int),
                ("solvers", C.c_int), ("pad", C.c_int), ("arena_bytes", C.c_ulonglong),
                ("batch_bytes", C.c_ulonglong), ("solve_bytes", C.c_ulonglong), ("options", C.POINTER(RsrrOptions))]


class RsrrRequest(C.Structure):
    _fields_ = [("nep", RsrrNep), ("gamma_re", C.c_double), ("gamma_im", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("N", C.c_int), ("L", C.c_int), ("U", C.c_void_p), ("ldu", C.c_int),
                ("NQ", C.c_int), ("KQ", C.c_int), ("delta", C.c_double), ("max_eigs", C.c_int),
                ("lambda_", C.POINTER(C.c_double)), ("resid", C.POINTER(C.c_double)),
                ("V", C.POINTER(C.c_double)), ("L_extra", C.c_int), ("pad", C.c_int)]


class RsrrResult(C.Structure):
    _fields_ = [("id", C.c_int), ("status", C.c_int), ("count", C.c_int), ("k", C.c_int), ("nbar", C.c_int),
                ("fallbacks", C.c_int), ("ir_iters_max", C.c_int), ("launches", C.c_int),
                ("sample_resid_max", C.c_double), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_sampled", C.c_double), ("t_done", C.c_double), ("reprobes", C.c_int), ("L_used", C.c_int),
                ("footprint", C.c_ulonglong)]


class RsrrError(RuntimeError):
    def __init__(self, fn, code):
        name = STATUS_NAMES.get(code, f"invalid argument {-code}" if code < 0 else str(code))
        super().__init__(f"{fn} failed: {name} ({code})")
        self.code = code


_lib = None


def lib():
    """Load librsrr.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
    L = C.CDLL(LIB_PATH)
    missing = [f for f in EXPORTS if not hasattr(L, f)]
    if missing:
        raise RuntimeError(f"{LIB_PATH} does not export {missing}")
    dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
    L.rsrr_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    L.rsrr_destroy.argtypes = [vp]
    L.rsrr_contour.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp, dp]
    L.rsrr_sample.argtypes = [vp, C.POINTER(RsrrNep), C.c_int, dp, vp, C.c_int, C.c_int, C.c_int, vp, C.c_int,
                              C.POINTER(RsrrPointInfo)]
    L.rsrr_sample_gmres.argtypes = [vp, C.POINTER(RsrrNep), C.c_int, dp, C.c_int, dp, ip, vp, C.c_int, C.c_int,
                                    C.c_double, C.c_int, C.c_int, C.c_int, vp, C.c_int, C.POINTER(RsrrGmresInfo)]
    L.rsrr_sample_batched.argtypes = [vp, C.c_int, C.POINTER(RsrrInstance), C.c_int, C.c_int,
                                      C.POINTER(RsrrPointInfo)]
    L.rsrr_basis.argtypes = [vp, C.c_int, C.c_int, vp, C.c_int, C.c_double, vp, C.c_int, C.c_int, ip, dp]
    L.rsrr_project.argtypes = [vp, C.POINTER(RsrrNep), vp, C.c_int, C.c_int, dp, C.c_double, vp, C.c_int, ip,
                               C.POINTER(RsrrTerm)]
    L.rsrr_solve.argtypes = [vp, C.POINTER(RsrrNep), C.c_int, vp, C.c_int, C.POINTER(RsrrTerm), vp, C.c_int, dp,
                             C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, C.c_int, dp, vp, C.c_int, dp,
                             ip, dp, C.POINTER(RsrrSolveInfo)]
    L.rsrr_last_timings.argtypes = [vp, dp]
    L.rsrr_update_stats.argtypes = [vp, C.c_int, C.c_int, dp]
    L.rsrr_two_stage.argtypes = [vp, C.POINTER(RsrrNep), dp, C.c_double, C.c_double, C.c_int, vp, C.c_int, C.c_int,
                                 C.c_int, vp, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_double, C.c_int,
                                 dp, vp, C.c_int, dp, ip, dp, C.POINTER(RsrrTwoStageInfo)]
    L.rsrr_moments.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, C.c_int, dp, dp, C.c_double, C.c_double, C.c_int,
                               vp, C.c_int]
    L.rsrr_moments_noalloc.argtypes = L.rsrr_moments.argtypes
    L.rsrr_server_create.argtypes = [C.POINTER(vp), C.POINTER(RsrrServerConfig)]
    L.rsrr_server_submit.argtypes = [vp, C.POINTER(RsrrRequest), ip]
    L.rsrr_server_footprint.argtypes = [C.POINTER(RsrrServerConfig), C.POINTER(RsrrRequest),
                                        C.POINTER(C.c_ulonglong)]
    L.rsrr_server_wait.argtypes = [vp, C.c_int, C.c_double, C.POINTER(RsrrResult)]
    L.rsrr_server_stats.argtypes = [vp, dp]
    L.rsrr_server_destroy.argtypes = [vp]
    L.rsrr_options_init.argtypes = [C.POINTER(RsrrOptions)]
    L.rsrr_set_options.argtypes = [vp, C.POINTER(RsrrOptions)]
    L.rsrr_get_options.argtypes = [vp, C.POINTER(RsrrOptions)]
    L.rsrr_version.restype = C.c_char_p
    for f in EXPORTS:
        if f != "rsrr_version":
            getattr(L, f).restype = C.c_int
    _lib = L
    return L


def _check(fn, code, ok=(RSRR_OK,)):
    if code not in ok:
        raise RsrrError(fn, code)
    return code


def _torch():
    import torch
    return torch


# ----------------------------------------------------------------------------- layout helpers

def colmajor(M, device="cuda"):
    """Host (rows, cols) complex array -> device tensor holding it column-major; returns (tensor, ld)."""
    torch = _torch()
    M = np.asarray(M, dtype=np.complex128)
    if M.ndim == 1:
        M = M[:, None]
    t = torch.from_numpy(np.ascontiguousarray(M.T)).to(device)
    return t, M.shape[0]


def from_colmajor(t, rows=None):
    """Device tensor of shape (cols, ld) -> host (rows, cols) complex array."""
    a = t.detach().cpu().numpy()
    if rows is None:
        rows = a.shape[1]
    return np.ascontiguousarray(a[:, :rows].T)


def term_struct(t):
    return RsrrTerm(t["c"].real, t["c"].imag, int(t["p"]), t["z0"].real, t["z0"].imag, float(t["tau"]),
                    t["s"].real, t["s"].imag, int(t["q"]))


def terms_array(terms):
    arr = (RsrrTerm * len(terms))()
    for i, t in enumerate(terms):
        arr[i] = term_struct(t)
    return arr


def term_from_struct(s):
    return {"c": complex(s.c_re, s.c_im), "p": s.p, "z0": complex(s.z0_re, s.z0_im), "tau": s.tau,
            "s": complex(s.s_re, s.s_im), "q": s.q}


class DeviceNEP:
    """A NEP whose data lives on the GPU, with the rsrr_nep descriptor pointing at it."""

    def __init__(self, nep, device="cuda"):
        torch = _torch()
        self.host = nep
        if hasattr(nep, "A"):
            self.kind = RSRR_T_SEPARABLE
            self.n = nep.A[0].shape[0]
            stack = np.stack([np.ascontiguousarray(np.asarray(A, dtype=np.complex128).T) for A in nep.A])
            self.A = torch.from_numpy(stack).to(device)
            self.terms = list(nep.terms)
            self._terms = terms_array(self.terms)
            self.desc = RsrrNep(RSRR_T_SEPARABLE, self.n, len(nep.A), self.A.data_ptr(), self.n,
                                C.cast(self._terms, C.POINTER(RsrrTerm)), None, 0.0)
        elif hasattr(nep, "csr"):
            self.kind = RSRR_T_SPARSE
            self.n = int(nep.n)
            self.mats = []
            for ip, ix, d in nep.csr:
                self.mats.append((torch.from_numpy(np.ascontiguousarray(ip, dtype=np.int32)).to(device),
                                  torch.from_numpy(np.ascontiguousarray(ix, dtype=np.int32)).to(device),
                                  torch.from_numpy(np.ascontiguousarray(d, dtype=np.complex128)).to(device)))
            self._csr = (RsrrCsr * len(self.mats))()
            for j, (ip, ix, d) in enumerate(self.mats):
                self._csr[j] = RsrrCsr(int(ix.numel()), 0, ip.data_ptr(), ix.data_ptr(), d.data_ptr())
            self.terms = list(nep.terms)
            self._terms = terms_array(self.terms)
            self.desc = RsrrNep(RSRR_T_SPARSE, self.n, len(self.mats), None, self.n,
                                C.cast(self._terms, C.POINTER(RsrrTerm)), None, 0.0,
                                C.cast(self._csr, C.POINTER(RsrrCsr)))
        else:
            self.kind = RSRR_T_HELMHOLTZ
            self.n = nep.points.shape[0]
            self.points = torch.from_numpy(np.ascontiguousarray(nep.points, dtype=np.float64)).to(device)
            self.w = float(nep.w)
            self._terms = None
            self.desc = RsrrNep(RSRR_T_HELMHOLTZ, self.n, 0, None, self.n, None, self.points.data_ptr(), self.w)


class Context:
    """An rsrr_ctx bound to a device and a HIP stream (default: torch's current stream)."""

    def __init__(self, device=0, stream=None):
        torch = _torch()
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        self.stream = stream
        self.device = device
        self.h = C.c_void_p()
        _check("rsrr_create", L.rsrr_create(C.byref(self.h), device, C.c_void_p(stream)))

    def close(self):
        if self.h:
            lib().rsrr_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def timings(self):
        t = (C.c_double * 5)()
        _check("rsrr_last_timings", lib().rsrr_last_timings(self.h, t))
        return {"assemble_ms": t[0], "lu_ms": t[1], "solve_ms": t[2], "residual_ms": t[3], "total_ms": t[4]}

    def raw_timings(self):
        """The five phase times (ms) of the last call, in the order its entry point documents."""
        t = (C.c_double * 5)()
        _check("rsrr_last_timings", lib().rsrr_last_timings(self.h, t))
        return list(t)


def rsrr_options(**kw):
    """An rsrr_options struct: the library's defaults with the given fields changed."""
    o = RsrrOptions()
    _check("rsrr_options_init", lib().rsrr_options_init(C.byref(o)))
    for f, v in kw.items():
        if f not in OPTION_FIELDS:
            raise KeyError(f)
        setattr(o, f, v)
    return o


def rsrr_set_options(ctx, **kw):
    """Change a context's options (rsrr_set_options); returns the options now in force."""
    o = rsrr_get_options(ctx)
    for f, v in kw.items():
        if f not in OPTION_FIELDS:
            raise KeyError(f)
        setattr(o, f, v)
    _check("rsrr_set_options", lib().rsrr_set_options(ctx.h, C.byref(o)))
    return rsrr_get_options(ctx)


def rsrr_get_options(ctx):
    o = RsrrOptions()
    o.size = C.sizeof(RsrrOptions)
    _check("rsrr_get_options", lib().rsrr_get_options(ctx.h, C.byref(o)))
    return o


def rsrr_update_stats(ctx, enable=True, reset=False):
    """Trailing-update kernel statistics: dict(launches, ms, flops, untimed)."""
    out = (C.c_double * 8)()
    _check("rsrr_update_stats", lib().rsrr_update_stats(ctx.h, int(enable), int(reset), out))
    return {"launches": int(out[0]), "ms": out[1], "flops": out[2], "untimed": int(out[3]), "bytes": out[4],
            "masked_ms": out[5], "masked_flops": out[6], "masked_cu_share": out[7]}


def rsrr_create(device=0, stream=None):
    return Context(device, stream)


def rsrr_contour(gamma, a, b, N):
    """Ellipse nodes and trapezoid weights (host, computed by the library)."""
    z = (C.c_double * (2 * N))()
    w = (C.c_double * (2 * N))()
    g = complex(gamma)
    _check("rsrr_contour", lib().rsrr_contour(g.real, g.imag, float(a), float(b), int(N), z, w))
    za = np.frombuffer(z, dtype=np.float64).view(np.complex128).copy()
    wa = np.frombuffer(w, dtype=np.float64).view(np.complex128).copy()
    return za, wa


def _zbuf(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return z, z.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))


def rsrr_sample(ctx, dnep, z, U, prec=RSRR_PREC_C64_IR, S=None, ok=(RSRR_OK, RSRR_WARN_FALLBACK)):
    """S = [T(z_k)^-1 U]_k on the GPU.  U: device tensor (L, n) (column-major n x L) or host array.

    Returns (S tensor of shape (N*L, n) = column-major n x N*L, info list, status).
    """
    torch = _torch()
    n = dnep.n
    if not torch.is_tensor(U):
        U, _ = colmajor(U)
    L = U.shape[0]
    ldu = U.shape[1]
    zc, zp = _zbuf(z)
    N = zc.size
    if S is None:
        S = torch.empty((N * L, n), dtype=torch.complex128, device=U.device)
    lds = S.shape[1]
    info = (RsrrPointInfo * N)()
    code = lib().rsrr_sample(ctx.h, C.byref(dnep.desc), N, zp, U.data_ptr(), L, ldu, int(prec), S.data_ptr(), lds,
                             info)
    _check("rsrr_sample", code, ok)
    infos = [{"info": i.info, "ir_iters": i.ir_iters, "fallback": i.fallback, "resid": i.resid} for i in info]
    return S, infos, code


RSRR_GMRES_MATRIX_FREE = 1


def rsrr_sample_gmres(ctx, dnep, z, U, zref, ref=None, tol=1e-10, restart=32, max_iters=300, flags=0, S=None,
                      ok=(RSRR_OK,)):
    """S = [T(z_k)^-1 U]_k by flexible GMRES preconditioned with complex FP32 LU factors of T at the
    reference points zref (point k uses ref[k], or the nearest reference when ref is None).

    Returns (S tensor of shape (N*L, n) = column-major n x N*L, info list, status).
    """
    torch = _torch()
    n = dnep.n
    if not torch.is_tensor(U):
        U, _ = colmajor(U)
    L = U.shape[0]
    ldu = U.shape[1]
    zc, zp = _zbuf(z)
    rc, rp = _zbuf(np.atleast_1d(zref))
    N = zc.size
    rarr = None
    if ref is not None:
        rarr = (C.c_int * N)(*[int(r) for r in ref])
    if S is None:
        S = torch.empty((N * L, n), dtype=torch.complex128, device=U.device)
    lds = S.shape[1]
    info = (RsrrGmresInfo * N)()
    code = lib().rsrr_sample_gmres(ctx.h, C.byref(dnep.desc), N, zp, rc.size, rp, rarr, U.data_ptr(), L, ldu,
                                   float(tol), int(restart), int(max_iters), int(flags), S.data_ptr(), lds, info)
    _check("rsrr_sample_gmres", code, ok)
    infos = [{"iters": i.iters, "restarts": i.restarts, "converged": i.converged, "ref": i.ref, "resid": i.resid,
              "matrix_free": i.matrix_free} for i in info]
    return S, infos, code


class BatchItem:
    """One instance of a ragged batch: a DeviceNEP, its points (host), probes and output (device)."""

    def __init__(self, dnep, z, U, S=None):
        torch = _torch()
        self.dnep = dnep
        self.z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
        if not torch.is_tensor(U):
            U, _ = colmajor(U)
        self.U = U
        L = U.shape[0]
        if S is None:
            S = torch.empty((self.z.size * L, dnep.n), dtype=torch.complex128, device=U.device)
        self.S = S


def rsrr_sample_batched(ctx, items, prec=RSRR_PREC_C64_IR, flags=0, ok=(RSRR_OK, RSRR_WARN_FALLBACK)):
    """Ragged batch of sampling problems.  Returns (per-item info lists, status)."""
    arr = (RsrrInstance * len(items))()
    keep = []
    for i, it in enumerate(items):
        zp = it.z.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))
        keep.append(it.z)
        arr[i] = RsrrInstance(it.dnep.desc, it.z.size, zp, it.U.data_ptr(), it.U.shape[0], it.U.shape[1],
                              it.S.data_ptr(), it.S.shape[1])
    total = sum(it.z.size for it in items)
    info = (RsrrPointInfo * total)()
    code = lib().rsrr_sample_batched(ctx.h, len(items), arr, int(prec), int(flags), info)
    _check("rsrr_sample_batched", code, ok)
    out, p = [], 0
    for it in items:
        out.append([{"info": info[p + k].info, "ir_iters": info[p + k].ir_iters, "fallback": info[p + k].fallback,
                     "resid": info[p + k].resid} for k in range(it.z.size)])
        p += it.z.size
    return out, code


def rsrr_basis(ctx, S, n, delta=1e-14, kmax=None):
    """Normalise S in place, truncated SVD basis.  Returns (Q tensor (kmax, n), k, sigma)."""
    torch = _torch()
    NL = S.shape[0]
    lds = S.shape[1]
    m = min(n, NL)
    kmax = m if kmax is None else kmax
    Q = torch.zeros((kmax, n), dtype=torch.complex128, device=S.device)
    k = C.c_int(0)
    sig = (C.c_double * m)()
    _check("rsrr_basis", lib().rsrr_basis(ctx.h, n, NL, S.data_ptr(), lds, float(delta), Q.data_ptr(), n, kmax,
                                          C.byref(k), sig))
    return Q, k.value, np.frombuffer(sig, dtype=np.float64).copy()


def rsrr_project(ctx, dnep, Q, k, gamma, radius, max_terms=64):
    """Projected coefficients Q^H A_j Q (device tensor (J_eff, k, k) column-major) and their terms."""
    torch = _torch()
    n = dnep.n
    ldq = Q.shape[1]
    AQ = torch.zeros((max_terms, k, k), dtype=torch.complex128, device=Q.device)
    J = C.c_int(0)
    tout = (RsrrTerm * max_terms)()
    g = (C.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    _check("rsrr_project", lib().rsrr_project(ctx.h, C.byref(dnep.desc), Q.data_ptr(), ldq, k, g, float(radius),
                                              AQ.data_ptr(), max_terms, C.byref(J), tout))
    terms = [term_from_struct(tout[i]) for i in range(J.value)]
    return AQ[:J.value], terms


def rsrr_solve(ctx, dnep, Q, k, AQ, terms, gamma, a, b, NQ=500, KQ=2, tol_gap=1e3, max_eigs=None,
               ok=(RSRR_OK, RSRR_WARN_GAP, RSRR_WARN_MORE)):
    """SS-FULL on the projected NEP and lift.  Returns dict with lam, V (host), resid, info, status."""
    torch = _torch()
    n = dnep.n
    ldq = Q.shape[1]
    max_eigs = max_eigs or min(k * KQ, 1024)
    lam = (C.c_double * (2 * max_eigs))()
    V = torch.zeros((max_eigs, n), dtype=torch.complex128, device=Q.device)
    res = (C.c_double * max_eigs)()
    cnt = C.c_int(0)
    sigH = (C.c_double * (KQ * k))()
    sinfo = RsrrSolveInfo()
    tarr = terms_array(terms)
    g = (C.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    code = lib().rsrr_solve(ctx.h, C.byref(dnep.desc), k, AQ.data_ptr(), len(terms),
                            C.cast(tarr, C.POINTER(RsrrTerm)), Q.data_ptr(), ldq, g, float(a), float(b), int(NQ),
                            int(KQ), float(tol_gap), max_eigs, lam, V.data_ptr(), n, res, C.byref(cnt), sigH,
                            C.byref(sinfo))
    _check("rsrr_solve", code, ok)
    m = cnt.value
    lam_np = np.frombuffer(lam, dtype=np.float64).view(np.complex128)[:m].copy()
    return {"lam": lam_np, "V": from_colmajor(V[:m], n), "resid": np.frombuffer(res, dtype=np.float64)[:m].copy(),
            "nbar": sinfo.nbar, "warn_gap": bool(sinfo.warn_gap), "gmax": sinfo.gmax,
            "truncated": bool(sinfo.truncated),
            "sigma_H": np.frombuffer(sigH, dtype=np.float64)[:sinfo.n_sigma].copy(), "status": code}


def rsrr_two_stage(ctx, dnep, gamma, a, b, N1, U, prec=RSRR_PREC_C64_IR, max_new=64, delta=1e-14, NQ=500, KQ=2,
                   tol_gap=1e3, max_eigs=256, ok=(RSRR_OK, RSRR_WARN_FALLBACK, RSRR_WARN_GAP)):
    """Two-stage sampling.  Returns dict with the stage-2 lam, V (host), resid, the added points z_new,
    the stage figures (k1, count1, nbar1, n_new, k2, nbar2, resid1_max) and the status."""
    torch = _torch()
    n = dnep.n
    if not torch.is_tensor(U):
        U, _ = colmajor(U)
    L = U.shape[0]
    S = torch.empty(((N1 + max_new) * L, n), dtype=torch.complex128, device=U.device)
    V = torch.zeros((max_eigs, n), dtype=torch.complex128, device=U.device)
    lam = (C.c_double * (2 * max_eigs))()
    res = (C.c_double * max_eigs)()
    zn = (C.c_double * (2 * max(1, max_new)))()
    cnt = C.c_int(0)
    ti = RsrrTwoStageInfo()
    g = (C.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    code = lib().rsrr_two_stage(ctx.h, C.byref(dnep.desc), g, float(a), float(b), int(N1), U.data_ptr(), L, U.shape[1],
                                int(prec), S.data_ptr(), n, int(max_new), float(delta), int(NQ), int(KQ),
                                float(tol_gap), int(max_eigs), lam, V.data_ptr(), n, res, C.byref(cnt), zn,
                                C.byref(ti))
    _check("rsrr_two_stage", code, ok)
    m = cnt.value
    out = {f: getattr(ti, f) for f, _ in RsrrTwoStageInfo._fields_}
    out.update({"lam": np.frombuffer(lam, dtype=np.float64).view(np.complex128)[:m].copy(),
                "V": from_colmajor(V[:m], n), "resid": np.frombuffer(res, dtype=np.float64)[:m].copy(),
                "z_new": np.frombuffer(zn, dtype=np.float64).view(np.complex128)[:ti.n_new].copy(),
                "status": code})
    return out


def rsrr_moments(ctx, S, n, z, L, K, gamma, rho, capacity):
    """M = S Z of the moment scheme.  S: device tensor (N*L, n); z: the N points of its blocks.
    Returns the device tensor (K*L, n) holding M column-major."""
    torch = _torch()
    zc, zp = _zbuf(z)
    N = zc.size
    M = torch.empty((K * L, n), dtype=torch.complex128, device=S.device)
    g = (C.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    _check("rsrr_moments", lib().rsrr_moments(ctx.h, n, N, L, S.data_ptr(), S.shape[1], zp, g, float(rho),
                                              float(capacity), int(K), M.data_ptr(), n))
    return M


def rsrr_moments_noalloc(ctx, S, n, z, L, K, gamma, rho, capacity, M):
    """rsrr_moments into a caller-provided device tensor M ((K*L, n), column-major n x K*L),
    with no device allocation by the library."""
    zc, zp = _zbuf(z)
    g = (C.c_double * 2)(complex(gamma).real, complex(gamma).imag)
    _check("rsrr_moments_noalloc", lib().rsrr_moments_noalloc(ctx.h, n, zc.size, L, S.data_ptr(), S.shape[1], zp, g,
                                                              float(rho), float(capacity), int(K), M.data_ptr(),
                                                              M.shape[1]))
    return M


def rsrr_version():
    return lib().rsrr_version().decode()


# ----------------------------------------------------------------------------- serving


class Server:
    """rsrr_server_*: a request loop running the whole method for many NEPs with
    continuous batching of their sampling points.  The binding keeps every
    buffer of a request alive until wait() has returned it."""

    def __init__(self, device=0, prec=RSRR_PREC_C64_IR, max_slots=8, arena_bytes=16 << 30,
                 batch_bytes=24 << 30, flags=0, solvers=0, options=None, solve_bytes=0):
        L = lib()
        self._opt = options
        self.cfg = RsrrServerConfig(device, int(prec), int(max_slots), int(flags), int(solvers), 0,
                                    int(arena_bytes), int(batch_bytes), int(solve_bytes),
                                    C.pointer(options) if options is not None else None)
        self.h = C.c_void_p()
        _check("rsrr_server_create", L.rsrr_server_create(C.byref(self.h), C.byref(self.cfg)))
        self._live = {}

    def _request(self, dnep, U, gamma, a, b, N, max_eigs, NQ, KQ, delta, L, L_extra, want_V):
        n = dnep.n
        lam = (C.c_double * (2 * max_eigs))()
        res = (C.c_double * max_eigs)()
        V = np.zeros((max_eigs, n), dtype=np.complex128) if want_V else None
        vptr = V.ctypes.data_as(C.POINTER(C.c_double)) if want_V else None
        g = complex(gamma)
        req = RsrrRequest(dnep.desc, g.real, g.imag, float(a), float(b), int(N), int(L), U.data_ptr(),
                          U.shape[1], int(NQ), int(KQ), float(delta), int(max_eigs),
                          C.cast(lam, C.POINTER(C.c_double)), C.cast(res, C.POINTER(C.c_double)), vptr,
                          int(L_extra), 0)
        return req, lam, res, V

    def submit(self, dnep, U, gamma, a, b, N, max_eigs=64, NQ=0, KQ=0, delta=0.0, want_V=False, L_extra=0):
        """U: device tensor (L + L_extra, n) holding the n x (L + L_extra) probes column-major; the
        last L_extra columns are solved only on a re-probe.  Returns the request id."""
        L = U.shape[0] - int(L_extra)
        req, lam, res, V = self._request(dnep, U, gamma, a, b, N, max_eigs, NQ, KQ, delta, L, L_extra, want_V)
        rid = C.c_int(0)
        _check("rsrr_server_submit", lib().rsrr_server_submit(self.h, C.byref(req), C.byref(rid)))
        self._live[rid.value] = (dnep, U, lam, res, V, req)
        return rid.value

    def footprint(self, dnep, U, gamma, a, b, N, max_eigs=64, L_extra=0):
        """Bytes of the arena block that admission charges for this request."""
        L = U.shape[0] - int(L_extra)
        req, _, _, _ = self._request(dnep, U, gamma, a, b, N, max_eigs, 0, 0, 0.0, L, L_extra, False)
        out = C.c_ulonglong(0)
        _check("rsrr_server_footprint", lib().rsrr_server_footprint(C.byref(self.cfg), C.byref(req), C.byref(out)))
        return out.value

    def wait(self, rid, timeout=-1.0):
        """Block until request rid has finished; returns its eigenpairs and timings."""
        out = RsrrResult()
        _check("rsrr_server_wait", lib().rsrr_server_wait(self.h, int(rid), float(timeout), C.byref(out)))
        dnep, U, lam, res, V, req = self._live.pop(rid)
        m = out.count
        r = {f: getattr(out, f) for f, _ in RsrrResult._fields_}
        r["lam"] = np.frombuffer(lam, dtype=np.float64).view(np.complex128)[:m].copy()
        r["resid"] = np.frombuffer(res, dtype=np.float64)[:m].copy()
        r["V"] = np.ascontiguousarray(V[:m].T) if V is not None else None
        return r

    def stats(self):
        out = (C.c_double * 12)()
        _check("rsrr_server_stats", lib().rsrr_server_stats(self.h, out))
        keys = ["finished", "points", "launches", "arena_peak_bytes", "max_launch_points", "sampler_busy_s",
                "solver_busy_s", "device_mem_peak_bytes", "now_s", "queued", "reprobe_points", "reprobes"]
        return dict(zip(keys, list(out)))

    def close(self):
        if self.h:
            lib().rsrr_server_destroy(self.h)
            self.h = C.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

