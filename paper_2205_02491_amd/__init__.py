"""Python binding of the MI355X ChASE library (libchase.so, C ABI in
include/chase.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Torch tensors provide device memory and streams.

Layout: torch tensors are row-major, the library is column-major.  The
column-major reading of a row-major Hermitian H is conj(H), which has the
same eigenvalues and conjugated eigenvectors, so vectors are passed and
returned conjugate-transposed (``X.mH``) and H is passed as is, without a
copy.  Gradients w.r.t. H come back directly in torch's convention.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchase.so")

C128, F64 = 0, 1
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_BF16X2 = 0, 1, 2, 3
EIG_AUTO, EIG_LIBRARY, EIG_JACOBI = 0, 1, 2
OK, ERR_ARG, ERR_NOMEM, ERR_HIP, ERR_NOCONV, ERR_NUMERIC = range(6)
_STATUS = {1: "CHASE_ERR_ARG", 2: "CHASE_ERR_NOMEM", 3: "CHASE_ERR_HIP",
           4: "CHASE_ERR_NOCONV", 5: "CHASE_ERR_NUMERIC"}

EXPORTED = ["chase_default_opts", "chase_workspace_bytes", "chase_create", "chase_destroy",
            "chase_solve", "chase_lanczos", "chase_lanczos_noalloc", "chase_filter",
            "chase_filter_ritz", "chase_qr",
            "chase_rayleigh_ritz", "chase_heev", "chase_cholesky", "chase_eigval_adjoint",
            "chase_eigvec_adjoint",
            "chase_filter_adjoint", "chase_filter_coefficients", "chase_spectral_bounds",
            "chase_degrees", "chase_last_error"]


class ChaseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("max_deg", ctypes.c_int), ("deg_extra", ctypes.c_int),
                ("optimize_degree", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("lanczos_vecs", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("filter_prec", ctypes.c_int), ("switch_tol", ctypes.c_double),
                ("verbose", ctypes.c_int), ("initial_rr", ctypes.c_int),
                ("fp64_tail", ctypes.c_int), ("seed", ctypes.c_int),
                ("debug", ctypes.c_int), ("adjoint_reserve", ctypes.c_int),
                ("eig_solver", ctypes.c_int), ("fp64_emulation", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("locked", ctypes.c_int),
                ("matvecs_fp64", ctypes.c_int64), ("matvecs_low", ctypes.c_int64),
                ("t_all", ctypes.c_double), ("t_lanczos", ctypes.c_double),
                ("t_filter", ctypes.c_double), ("t_qr", ctypes.c_double),
                ("t_rr", ctypes.c_double), ("t_resid", ctypes.c_double),
                ("t_filter_kernels", ctypes.c_double), ("filter_launches", ctypes.c_int64),
                ("filter_flops", ctypes.c_double), ("b_sup", ctypes.c_double),
                ("mu_1", ctypes.c_double), ("mu_ne", ctypes.c_double),
                ("qr_shifted", ctypes.c_int), ("qr_householder", ctypes.c_int),
                ("t_lanczos_gemv", ctypes.c_double), ("lanczos_gemv_launches", ctypes.c_int64),
                ("lanczos_gemv_bytes", ctypes.c_double),
                ("t_filter_kernels_low", ctypes.c_double),
                ("filter_launches_low", ctypes.c_int64), ("fp64_tail", ctypes.c_int),
                ("debug_herm_defect", ctypes.c_double),
                ("debug_orth_defect", ctypes.c_double), ("t_rr_eig", ctypes.c_double),
                ("eig_jacobi_calls", ctypes.c_int), ("eig_jacobi_sweeps", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libchase.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2205_02491_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, ci, cd = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    pd, pi, pi64 = ctypes.POINTER(cd), ctypes.POINTER(ci), ctypes.POINTER(i64)
    L.chase_default_opts.argtypes = [ctypes.POINTER(Opts)]
    L.chase_default_opts.restype = None
    L.chase_workspace_bytes.argtypes = [ci, i64, ci, ci, ctypes.POINTER(Opts)]
    L.chase_workspace_bytes.restype = ctypes.c_size_t
    L.chase_create.argtypes = [ctypes.POINTER(vp), ci, i64, ci, ci, ctypes.POINTER(Opts)]
    L.chase_create.restype = ci
    L.chase_destroy.argtypes = [vp]
    L.chase_destroy.restype = None
    L.chase_solve.argtypes = [vp, vp, i64, cd, ci, vp, vp, pd, vp, i64, pd,
                              ctypes.POINTER(Stats), vp]
    L.chase_solve.restype = ci
    L.chase_lanczos.argtypes = [vp, vp, i64, vp, ci, ci, pd, pd, pd, pd, pd, pi, vp]
    L.chase_lanczos.restype = ci
    L.chase_lanczos_noalloc.argtypes = [ci, vp, i64, i64, ci, vp, ci, ci, pd, pd, pd, pd, pd, pi,
                                        vp]
    L.chase_lanczos_noalloc.restype = ci
    L.chase_filter.argtypes = [vp, vp, i64, vp, i64, ci, pi, cd, cd, cd, ci, ci, pi64, vp]
    L.chase_filter.restype = ci
    L.chase_filter_ritz.argtypes = [vp, vp, i64, vp, i64, vp, i64, pd, ci, pi, cd, cd, cd, ci,
                                    pi64, vp]
    L.chase_filter_ritz.restype = ci
    L.chase_qr.argtypes = [vp, vp, i64, ci, ci, pi, pi, vp]
    L.chase_qr.restype = ci
    L.chase_rayleigh_ritz.argtypes = [vp, vp, i64, vp, i64, ci, cd, pd, pd, vp]
    L.chase_rayleigh_ritz.restype = ci
    L.chase_heev.argtypes = [vp, vp, i64, ci, ci, pd, pi, vp]
    L.chase_heev.restype = ci
    L.chase_cholesky.argtypes = [vp, vp, i64, ci, pi, vp]
    L.chase_cholesky.restype = ci
    L.chase_eigval_adjoint.argtypes = [vp, vp, i64, ci, pd, vp, i64, vp]
    L.chase_eigval_adjoint.restype = ci
    L.chase_filter_adjoint.argtypes = [vp, vp, i64, vp, i64, vp, i64, vp, vp]
    L.chase_filter_adjoint.restype = ci
    L.chase_eigvec_adjoint.argtypes = [vp, vp, i64, vp, i64, ci, pd, vp, i64, vp, i64, cd, ci,
                                       ctypes.POINTER(ctypes.c_int), vp]
    L.chase_eigvec_adjoint.restype = ci
    L.chase_filter_coefficients.argtypes = [ci, cd, cd, cd, pd]
    L.chase_filter_coefficients.restype = ci
    L.chase_spectral_bounds.argtypes = [pd, pd, ci, ci, i64, ci, pd, pd, pd, pi]
    L.chase_spectral_bounds.restype = ci
    L.chase_degrees.argtypes = [pd, pd, ci, cd, cd, cd, ci, ctypes.POINTER(Opts), pi]
    L.chase_degrees.restype = ci
    L.chase_last_error.argtypes = []
    L.chase_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status, allow_noconv=False):
    if status == OK or (allow_noconv and status == ERR_NOCONV):
        return status
    raise ChaseError(status, lib().chase_last_error().decode())


def default_opts(**kw) -> Opts:
    o = Opts()
    lib().chase_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def chase_workspace_bytes(n, nev, nex, cplx=True, opts: Opts | None = None) -> int:
    return int(lib().chase_workspace_bytes(C128 if cplx else F64, n, nev, nex,
                                           ctypes.byref(opts) if opts else None))


def _dtype_code(t):
    import torch
    if t.dtype == torch.complex128:
        return C128
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"unsupported dtype {t.dtype}: complex128 or float64")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t):
    if t.is_conj() or t.is_neg():
        # a lazy conjugate/negative view: its memory holds the other values
        raise ValueError("tensor is a lazy conjugate or negative view; call "
                         "resolve_conj() / resolve_neg() first")
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def _colmajor(x):
    """Column-major buffer (as a row-major (k, n) tensor) of the vectors of x
    (n, k) in the conj(H) frame: x.mH materialised in new memory.  (For a
    single vector x.mH is already contiguous, and .contiguous() would return
    the lazy conjugate view of x's own memory.)"""
    import torch
    return x.mH.resolve_conj().clone(memory_format=torch.contiguous_format)


def _check_square(H):
    """H: a square, contiguous complex128 or float64 tensor (the library
    reads n x n entries with leading dimension n)."""
    if H.dim() != 2 or H.shape[0] != H.shape[1]:
        raise ValueError(f"H must be a square matrix, got shape {tuple(H.shape)}")
    if not H.is_contiguous():
        raise ValueError("H must be contiguous")
    _dtype_code(H)


def _check_handle(handle, n, dtype, nev=None, nex=None, k=None):
    """The handle's sizes and element type must match the arguments: the
    library sizes every read and write by the handle."""
    import torch
    if handle.n != n:
        raise ValueError(f"handle was created for n={handle.n}, the arguments have n={n}")
    if handle.cplx != (dtype == torch.complex128):
        raise ValueError(f"handle was created for {'complex128' if handle.cplx else 'float64'}, "
                         f"the arguments are {dtype}")
    if nev is not None and (handle.nev, handle.nex) != (nev, nex):
        raise ValueError(f"handle was created for nev={handle.nev}, nex={handle.nex}; "
                         f"the call asks for nev={nev}, nex={nex}")
    if k is not None and not 1 <= k <= handle.nev + handle.nex:
        raise ValueError(f"{k} columns do not fit the handle (1 <= k <= nev+nex = "
                         f"{handle.nev + handle.nex})")


def _check_block(X, n, k=None, name="X"):
    if X.dim() != 2 or X.shape[0] != n or (k is not None and X.shape[1] != k):
        want = f"({n}, {k})" if k is not None else f"({n}, k)"
        raise ValueError(f"{name} must have shape {want}, got {tuple(X.shape)}")


def _host_vec(a, length, dtype, name):
    out = np.ascontiguousarray(np.asarray(a, dtype=dtype)).ravel()
    if out.shape[0] != length:
        raise ValueError(f"{name} must have {length} entries, got {out.shape[0]}")
    return out


class Handle:
    """Owns the library handle and its device workspace (allocated once)."""

    def __init__(self, n, nev, nex, dtype=None, opts: Opts | None = None, **kw):
        import torch
        dtype = dtype or torch.complex128
        self.cplx = dtype == torch.complex128
        self.n, self.nev, self.nex = int(n), int(nev), int(nex)
        self.opts = opts or default_opts(**kw)
        self.dtype = dtype
        self.tape_k = None
        h = ctypes.c_void_p()
        _check(lib().chase_create(ctypes.byref(h), C128 if self.cplx else F64, self.n,
                                  self.nev, self.nex, ctypes.byref(self.opts)))
        self._h = h

    @property
    def ptr(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            lib().chase_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _ensure_handle(handle, H, nev, nex, opts):
    if handle is not None:
        return handle, False
    return Handle(H.shape[0], nev, nex, H.dtype, opts), True


def chase_solve(H, nev, nex, tol=1e-10, degree=20, V0=None, S=None, opts=None, handle=None):
    """Lowest nev eigenpairs of the Hermitian H (n x n torch tensor on the GPU,
    complex128 or float64).  V0 (n x (nev+nex)) and S (n x lanczos_vecs) are
    the start block and the Lanczos start vectors; when omitted the library
    draws them (seeded by opts.seed).  Returns (evals numpy[nev], evecs tensor
    (n, nev), resid numpy[nev], stats dict).  NOCONV returns the best pairs
    with stats['converged'] = False."""
    import torch
    _check_square(H)
    n = H.shape[0]
    if handle is not None:
        _check_handle(handle, n, H.dtype, nev, nex)
    h, own = _ensure_handle(handle, H, nev, nex, opts)
    try:
        ne = nev + nex
        nl = h.opts.lanczos_vecs
        if V0 is not None:
            _check_block(V0, n, ne, "V0")
        if S is not None:
            _check_block(S, n, nl, "S")
        v0c = None if V0 is None else _colmajor(V0.to(H.dtype))
        sc = None if S is None else _colmajor(S.to(H.dtype))
        evecs_buf = torch.empty((nev, n), dtype=H.dtype, device=H.device)
        ev = np.zeros(nev)
        rs = np.zeros(nev)
        st = Stats()
        status = lib().chase_solve(h.ptr, _dev(H), n, float(tol), int(degree),
                                   None if v0c is None else _dev(v0c),
                                   None if sc is None else _dev(sc),
                                   ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   _dev(evecs_buf), n,
                                   rs.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(st), _stream())
        _check(status, allow_noconv=True)
        d = st.as_dict()
        d["converged"] = status == OK
        return ev, evecs_buf.mH, rs, d
    finally:
        if own:
            h.close()


def chase_lanczos(H, S, steps=None, handle=None, n_e=None, opts=None):
    """Lanczos bounds from the start vectors S (n x nvec).  Returns
    (b_sup, mu_1, mu_ne, alpha[nvec, steps], beta[nvec, steps], lengths)."""
    _check_square(H)
    n = H.shape[0]
    _check_block(S, n, None, "S")
    nvec = S.shape[1]
    if handle is None:
        if n_e is None:
            raise ValueError("n_e (= nev + nex) is needed when no handle is given")
        nev = max(1, n_e // 2)
        handle = Handle(n, nev, n_e - nev, H.dtype, opts)
    _check_handle(handle, n, H.dtype)
    steps = steps or handle.opts.lanczos_steps
    sc = _colmajor(S.to(H.dtype))
    a = np.zeros((nvec, steps))
    b = np.zeros((nvec, steps))
    lens = np.zeros(nvec, dtype=np.int32)
    out = [ctypes.c_double() for _ in range(3)]
    pd = ctypes.POINTER(ctypes.c_double)
    _check(lib().chase_lanczos(handle.ptr, _dev(H), n, _dev(sc), nvec, steps,
                               ctypes.byref(out[0]), ctypes.byref(out[1]), ctypes.byref(out[2]),
                               a.ctypes.data_as(pd), b.ctypes.data_as(pd),
                               lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _stream()))
    return out[0].value, out[1].value, out[2].value, a, b, lens


def chase_lanczos_noalloc(H, S, n_e, steps=25):
    """chase_lanczos without a handle and without device allocations: the
    library's fixed scratch holds the work buffers.  No copy is made of S, so
    it must already be in the form the library reads: column-major (S.mT
    contiguous, e.g. a view of an (nvec, n) tensor) and, for complex H, in
    the library's frame (the column-major buffer of conj(H) is torch's H, so
    start vectors s of H are passed as s.conj(); chase_lanczos does that
    conjugating copy itself).  Returns (b_sup, mu_1, mu_ne, alpha[nvec, steps],
    beta[nvec, steps], lengths), the same as chase_lanczos."""
    _check_square(H)
    n = H.shape[0]
    _check_block(S, n, None, "S")
    if S.dtype != H.dtype:
        raise ValueError("S must have H's dtype")
    if not S.mT.is_contiguous():
        raise ValueError("S must be column-major (S.mT contiguous): no copy is made here")
    nvec = S.shape[1]
    a = np.zeros((nvec, steps))
    b = np.zeros((nvec, steps))
    lens = np.zeros(nvec, dtype=np.int32)
    out = [ctypes.c_double() for _ in range(3)]
    pd = ctypes.POINTER(ctypes.c_double)
    _check(lib().chase_lanczos_noalloc(_dtype_code(H), _dev(H), n, n, int(n_e), _dev(S),
                                       nvec, int(steps), ctypes.byref(out[0]),
                                       ctypes.byref(out[1]), ctypes.byref(out[2]),
                                       a.ctypes.data_as(pd), b.ctypes.data_as(pd),
                                       lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                       _stream()))
    return out[0].value, out[1].value, out[2].value, a, b, lens


def chase_filter(H, X, degrees, b_sup, mu_1, mu_ne, prec=PREC_FP64, record_tape=False,
                 handle=None):
    """Chebyshev filter of the columns of X (n x k) with per-column even,
    non-decreasing degrees.  Returns (Y, matvecs); X is not modified."""
    _check_square(H)
    n = H.shape[0]
    _check_block(X, n, None, "X")
    k = X.shape[1]
    if handle is None:
        handle = Handle(n, max(1, k - 1) if k > 1 else 1, 1 if k > 1 else 1, H.dtype,
                        filter_prec=int(prec))
    _check_handle(handle, n, H.dtype, k=k)
    buf = _colmajor(X.to(H.dtype))
    deg = _host_vec(degrees, k, np.int32, "degrees")
    mv = ctypes.c_int64()
    _check(lib().chase_filter(handle.ptr, _dev(H), n, _dev(buf), n, k,
                              deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), float(b_sup),
                              float(mu_1), float(mu_ne), int(prec), int(bool(record_tape)),
                              ctypes.byref(mv), _stream()))
    # the recorded tape (the adjoint reads k columns of its gradient)
    handle.tape_k = k if record_tape else None
    return buf.mH, mv.value


def chase_filter_ritz(H, V, R, theta, degrees, b_sup, mu_1, mu_ne, prec=PREC_FP64,
                      handle=None):
    """p(H) V in the defect-correction form for vectors V (n x k) with shifts
    theta (k) and residuals R = H V - V diag(theta).  Returns (Y, matvecs)."""
    _check_square(H)
    n = H.shape[0]
    _check_block(V, n, None, "V")
    k = V.shape[1]
    _check_block(R, n, k, "R")
    if handle is None:
        handle = Handle(n, max(1, k - 1) if k > 1 else 1, 1, H.dtype, filter_prec=int(prec))
    _check_handle(handle, n, H.dtype, k=k)
    vbuf = _colmajor(V.to(H.dtype))
    rbuf = _colmajor(R.to(H.dtype))
    th = _host_vec(theta, k, np.float64, "theta")
    deg = _host_vec(degrees, k, np.int32, "degrees")
    mv = ctypes.c_int64()
    _check(lib().chase_filter_ritz(handle.ptr, _dev(H), n, _dev(vbuf), n, _dev(rbuf), n,
                                   th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), k,
                                   deg.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   float(b_sup), float(mu_1), float(mu_ne), int(prec),
                                   ctypes.byref(mv), _stream()))
    return vbuf.mH, mv.value


def chase_qr(X, locked=0, handle=None, return_stats=False):
    """Orthonormalise X (n x k) keeping its first `locked` columns.  With
    return_stats, also returns {'shifted_passes', 'householder'}."""
    if X.dim() != 2:
        raise ValueError(f"X must be a matrix, got shape {tuple(X.shape)}")
    n, k = X.shape
    if handle is None:
        handle = Handle(n, max(1, k - 1), 1, X.dtype)
    _check_handle(handle, n, X.dtype, k=k)
    buf = _colmajor(X)
    sp, hh = ctypes.c_int(), ctypes.c_int()
    _check(lib().chase_qr(handle.ptr, _dev(buf), n, k, int(locked), ctypes.byref(sp),
                          ctypes.byref(hh), _stream()))
    if return_stats:
        return buf.mH, {"shifted_passes": sp.value, "householder": hh.value}
    return buf.mH


def chase_rayleigh_ritz(H, Q, norm_scale=1.0, handle=None):
    """Rayleigh-Ritz + residuals on the orthonormal Q (n x k): returns
    (ritz numpy[k], V tensor (n, k), resid numpy[k])."""
    _check_square(H)
    n = H.shape[0]
    _check_block(Q, n, None, "Q")
    k = Q.shape[1]
    if handle is None:
        handle = Handle(n, max(1, k - 1), 1, H.dtype)
    _check_handle(handle, n, H.dtype, k=k)
    buf = _colmajor(Q.to(H.dtype))
    ritz = np.zeros(k)
    res = np.zeros(k)
    pd = ctypes.POINTER(ctypes.c_double)
    _check(lib().chase_rayleigh_ritz(handle.ptr, _dev(H), n, _dev(buf), n, k, float(norm_scale),
                                     ritz.ctypes.data_as(pd), res.ctypes.data_as(pd), _stream()))
    return ritz, buf.mH, res


def chase_heev(G, method=EIG_AUTO, handle=None):
    """Dense Hermitian eigensolve of G (k x k) with the eigensolver of the
    library's Rayleigh-Ritz step (method: EIG_AUTO, EIG_LIBRARY or
    EIG_JACOBI).  Returns (eigenvalues numpy[k] ascending, W tensor (k, k)
    with the eigenvectors as columns, Jacobi sweeps (0 when the library's
    divide and conquer ran)).  G is not modified."""
    import torch
    _check_square(G)
    k = G.shape[0]
    if handle is None:
        handle = Handle(max(k, 2), max(1, k - 1), 1, G.dtype)
    if handle.cplx != (G.dtype == torch.complex128):
        raise ValueError("handle and G differ in element type")
    if not 1 <= k <= handle.nev + handle.nex:
        raise ValueError(f"k={k} exceeds the handle's nev+nex={handle.nev + handle.nex}")
    # the row-major buffer of G is the column-major buffer of conj(G): same
    # eigenvalues, conjugated eigenvectors
    buf = G.resolve_conj().clone(memory_format=torch.contiguous_format)
    ev = np.zeros(k)
    sw = ctypes.c_int()
    _check(lib().chase_heev(handle.ptr, _dev(buf), k, k, int(method),
                            ev.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            ctypes.byref(sw), _stream()))
    return ev, buf.mH, sw.value


def chase_cholesky(A, handle=None):
    """Cholesky factor A = R^H R of the Hermitian positive definite A (k x k)
    with the factorisation of the library's Cholesky QR passes.  Returns
    (R tensor (k, k) upper triangular, info): info is 0, or the 1-based
    order of the first leading minor that is not positive definite (then R
    is partial).  A is not modified."""
    import torch
    _check_square(A)
    k = A.shape[0]
    if handle is None:
        handle = Handle(2, 1, 1, A.dtype)
    if handle.cplx != (A.dtype == torch.complex128):
        raise ValueError("handle and A differ in element type")
    # a row-major copy of A^T is A in column-major order (the library reads
    # the upper triangle of A itself)
    buf = A.transpose(0, 1).resolve_conj().clone(memory_format=torch.contiguous_format)
    info = ctypes.c_int()
    _check(lib().chase_cholesky(handle.ptr, _dev(buf), max(1, k), k, ctypes.byref(info),
                                _stream()))
    # buf^T is the column-major result: R over A's upper triangle
    return torch.triu(buf.transpose(0, 1)), info.value


def chase_eigval_adjoint(V, g, dH, handle=None):
    """dH += V diag(g) V^H (in place on the torch tensor dH, n x n)."""
    if V.dim() != 2:
        raise ValueError(f"V must be a matrix, got shape {tuple(V.shape)}")
    n, m = V.shape
    _check_square(dH)
    if dH.shape[0] != n or dH.dtype != V.dtype:
        raise ValueError(f"dH must be a contiguous ({n}, {n}) {V.dtype} matrix")
    if handle is None:
        handle = Handle(n, max(1, m - 1) if m > 1 else 1, 1, V.dtype)
    _check_handle(handle, n, V.dtype, k=m)
    buf = _colmajor(V)
    gg = _host_vec(g, m, np.float64, "g")
    _check(lib().chase_eigval_adjoint(handle.ptr, _dev(buf), n, m,
                                      gg.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _dev(dH), n, _stream()))
    return dH


def chase_eigvec_adjoint(H, V, lam, G, dH, handle=None, tol=1e-10, max_iter=5000):
    """dH += dL/dH for a phase-invariant loss of the lowest eigenvectors V
    (n x m torch tensor, eigenvalues lam ascending) with G = dL/dV (torch's
    convention), in place on the torch tensor dH (n x n).  Returns the number
    of conjugate-gradient iterations of the complement solves."""
    _check_square(H)
    n = H.shape[0]
    _check_block(V, n, None, "V")
    m = V.shape[1]
    _check_block(G, n, m, "G")
    _check_square(dH)
    if dH.shape[0] != n or dH.dtype != H.dtype:
        raise ValueError(f"dH must be a contiguous ({n}, {n}) {H.dtype} matrix")
    if handle is None:
        handle = Handle(n, m, 1 if m < n - 1 else max(1, n - m), H.dtype)
    _check_handle(handle, n, H.dtype, k=m)
    vbuf = _colmajor(V.to(H.dtype))
    gbuf = _colmajor(G.to(H.dtype))
    lm = _host_vec(lam, m, np.float64, "lam")
    its = ctypes.c_int()
    _check(lib().chase_eigvec_adjoint(handle.ptr, _dev(H), n, _dev(vbuf), n, m,
                                      lm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _dev(gbuf), n, _dev(dH), n, float(tol), int(max_iter),
                                      ctypes.byref(its), _stream()))
    return its.value


def chase_filter_adjoint(H, gY, dH, handle, want_gX=False):
    """Adjoint of the last recorded chase_filter on `handle`: dH += dL/dH;
    returns dL/dX0 (n x k) if want_gX."""
    import torch
    _check_square(H)
    n = H.shape[0]
    _check_handle(handle, n, H.dtype)
    if getattr(handle, "tape_k", None) is None:
        raise ValueError("no recorded filter tape on this handle (call chase_filter with "
                         "record_tape=True)")
    _check_block(gY, n, handle.tape_k, "gY")
    _check_square(dH)
    if dH.shape[0] != n or dH.dtype != H.dtype:
        raise ValueError(f"dH must be a contiguous ({n}, {n}) {H.dtype} matrix")
    k = gY.shape[1]
    gbuf = _colmajor(gY.to(H.dtype))
    gx = torch.empty_like(gbuf) if want_gX else None
    _check(lib().chase_filter_adjoint(handle.ptr, _dev(H), n, _dev(gbuf), n, _dev(dH), n,
                                      _dev(gx) if gx is not None else None, _stream()))
    return gx.mH if gx is not None else None


def _pd(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def chase_filter_coefficients(m, b_sup, mu_1, mu_ne):
    """Scaled Chebyshev coefficients of Eq. (3) used by chase_filter: an
    (m, 3) float64 array of (alpha, gamma, beta) per step."""
    out = np.zeros((m, 3))
    _check(lib().chase_filter_coefficients(int(m), float(b_sup), float(mu_1), float(mu_ne),
                                           _pd(out)))
    return out


def chase_spectral_bounds(alpha, beta, n, n_e):
    """b_sup, mu_1, mu_ne and per-run lengths from Lanczos tridiagonals
    (alpha, beta: nvec x steps, one run per row, as chase_lanczos returns)."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    if a.ndim != 2 or a.shape != b.shape:
        raise ValueError("alpha and beta must be 2-D arrays of one shape (nvec, steps)")
    nvec, steps = a.shape
    bs, m1, mne = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lens = (ctypes.c_int * nvec)()
    _check(lib().chase_spectral_bounds(_pd(a), _pd(b), nvec, steps, int(n), int(n_e),
                                       ctypes.byref(bs), ctypes.byref(m1), ctypes.byref(mne),
                                       lens))
    return bs.value, m1.value, mne.value, list(lens)


def chase_degrees(resid, ritz, b_sup, mu_ne, tol, degree=20, opts: Opts | None = None):
    """Per-vector filter degrees of Algorithm 1's degree step."""
    r = np.ascontiguousarray(resid, dtype=np.float64).ravel()
    t = np.ascontiguousarray(ritz, dtype=np.float64).ravel()
    if r.shape != t.shape:
        raise ValueError("resid and ritz must have the same length")
    out = (ctypes.c_int * max(len(r), 1))()
    _check(lib().chase_degrees(_pd(r), _pd(t), len(r), float(b_sup), float(mu_ne), float(tol),
                               int(degree), ctypes.byref(opts) if opts is not None else None,
                               out))
    return np.array(out[: len(r)], dtype=np.int64)


from .autograd import ChaseEigh, chase_eigh, filtered_block  # noqa: E402

__all__ = ["Handle", "Opts", "Stats", "ChaseError", "default_opts", "chase_workspace_bytes",
           "chase_solve", "chase_lanczos", "chase_lanczos_noalloc", "chase_filter",
           "chase_filter_ritz", "chase_qr",
           "chase_rayleigh_ritz", "chase_heev", "chase_cholesky",
           "chase_eigval_adjoint", "chase_eigvec_adjoint", "chase_filter_adjoint",
           "chase_filter_coefficients", "chase_spectral_bounds", "chase_degrees", "ChaseEigh",
           "chase_eigh",
           "filtered_block", "lib", "EXPORTED"]
