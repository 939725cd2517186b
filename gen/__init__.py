"""Seeded synthetic inputs shaped like the paper's test problems.

This module only draws random numbers and assembles test matrices with a
prescribed spectrum (the construction of the paper's test-matrix suite,
Section "Test matrix suite", Table 1: a diagonal of prescribed eigenvalues
conjugated by the Q factor of a Gaussian matrix). It contains none of the
eigensolver's arithmetic and is shared by the oracle-side and the GPU-side
tests, the benchmark and the smoke run.

Every draw comes from numpy's PCG64 seeded with ``BASE_SEED + 10*cfg + slot``
(slots below), so that both sides of a parity test see the same bytes. The
large workloads can also be drawn on the device with torch (``make_torch``);
those inputs are documented as a different (but equally seeded) stream.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 220502491

# seed slots inside one configuration
SLOT_Q, SLOT_LAMBDA, SLOT_V0, SLOT_S, SLOT_W, SLOT_B = range(6)

# configuration indices used to derive seeds
CFG_SMALL, CFG_GEO20K, CFG_MIXED30K, CFG_HUGE100K, CFG_DIFF8K, CFG_TABLE2 = range(6)


def rng(cfg: int, slot: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(BASE_SEED + 10 * cfg + slot))


def gaussian(g: np.random.Generator, shape, cplx: bool) -> np.ndarray:
    """i.i.d. standard normal entries; complex ones have Re, Im ~ N(0, 1/2)."""
    if cplx:
        re = g.standard_normal(shape)
        im = g.standard_normal(shape)
        return (re + 1j * im) * math.sqrt(0.5)
    return g.standard_normal(shape)


def haar(n: int, g: np.random.Generator, cplx: bool) -> np.ndarray:
    """Haar-distributed unitary (orthogonal) matrix: QR of a Gaussian matrix
    with the phases of R's diagonal moved into Q (Mezzadri 2007)."""
    z = gaussian(g, (n, n), cplx)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r)
    ph = d / np.abs(d)
    return q * ph[None, :]


def planted(lam: np.ndarray, q: np.ndarray) -> np.ndarray:
    """H = Q diag(lam) Q^H, symmetrised so both triangles agree bitwise."""
    h = (q * lam[None, :]) @ q.conj().T
    return (h + h.conj().T) / 2


# ---------------------------------------------------------------- spectra
def spectrum_uniform_iid(n: int, g: np.random.Generator, lo=-1.0, hi=1.0) -> np.ndarray:
    return np.sort(g.uniform(lo, hi, size=n))


def spectrum_geometric_low(n: int, g: np.random.Generator, n_geo: int) -> np.ndarray:
    """Lowest n_geo values -1 + 10^(-4(1 - i/n_geo)), i = 1..n_geo (from -0.9999
    up to 0), the rest i.i.d. uniform in [0, 1]."""
    i = np.arange(1, n_geo + 1, dtype=np.float64)
    low = -1.0 + 10.0 ** (-4.0 * (1.0 - i / n_geo))
    high = np.sort(g.uniform(0.0, 1.0, size=n - n_geo))
    return np.concatenate([low, high])


def spectrum_121_cluster(n: int, g: np.random.Generator, n_low: int, top=10.0) -> np.ndarray:
    """Lowest n_low eigenvalues of the (1-2-1) matrix of size n
    (2 - 2 cos(pi k/(n+1)), Table 1), the rest i.i.d. uniform in
    [lambda_{n_low}, top]."""
    k = np.arange(1, n_low + 1, dtype=np.float64)
    low = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    high = np.sort(g.uniform(low[-1], top, size=n - n_low))
    return np.concatenate([low, high])


def table1_uniform(n: int, dmax=1.0, eps=1e-4) -> np.ndarray:
    k = np.arange(1, n + 1, dtype=np.float64)
    return dmax * (eps + (k - 1) * (1 - eps) / (n - 1))


def table1_geometric(n: int, dmax=1.0, eps=1e-4) -> np.ndarray:
    k = np.arange(1, n + 1, dtype=np.float64)
    return dmax * eps ** ((n - k) / (n - 1))


def tridiag_121(n: int):
    """(1-2-1) matrix as (diagonal, off-diagonal)."""
    return np.full(n, 2.0), np.full(n - 1, 1.0)


def tridiag_wilkinson(n: int):
    """Wilkinson matrix: off-diagonal ones, diagonal |i - (n-1)/2|, i = 0..n-1
    (the paper's printed diagonal has the wrong length; this reading gives a
    symmetric V-shaped diagonal of length n)."""
    i = np.arange(n, dtype=np.float64)
    return np.abs(i - (n - 1) / 2.0), np.full(n - 1, 1.0)


def dense_from_tridiag(d: np.ndarray, e: np.ndarray) -> np.ndarray:
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def spectrum_table1(kind: str, n: int) -> np.ndarray:
    """Ascending eigenvalues of the paper's matrix types (Table 1): Uniform
    and Geometric (d_max = 1, eps = 1e-4), and the spectra of the (1-2-1)
    and Wilkinson tridiagonal matrices of order n (the (1-2-1) one in closed
    form, the Wilkinson one from LAPACK's tridiagonal eigensolver)."""
    if kind == "uniform":
        return table1_uniform(n)
    if kind == "geometric":
        return table1_geometric(n)
    if kind == "121":
        k = np.arange(1, n + 1, dtype=np.float64)
        return 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
    if kind == "wilkinson":
        import scipy.linalg
        d, e = tridiag_wilkinson(n)
        return scipy.linalg.eigvalsh_tridiagonal(d, e)
    raise ValueError(kind)


# ---------------------------------------------------------------- problems
@dataclasses.dataclass
class Problem:
    name: str
    H: np.ndarray          # n x n, C order (row-major) numpy array
    lam: np.ndarray        # planted spectrum, ascending
    Q: np.ndarray | None   # planted eigenvectors (columns), or None
    V0: np.ndarray         # n x (nev+nex) start block
    S: np.ndarray          # n x n_lanczos Lanczos start vectors
    nev: int
    nex: int
    deg: int
    tol: float

    @property
    def n(self):
        return self.H.shape[0]

    @property
    def cplx(self):
        return np.iscomplexobj(self.H)


def start_blocks(cfg: int, n: int, n_e: int, n_lanczos: int, cplx: bool):
    v0 = gaussian(rng(cfg, SLOT_V0), (n, n_e), cplx)
    s = gaussian(rng(cfg, SLOT_S), (n, n_lanczos), cplx)
    return v0, s


def make_uniform(n=1000, nev=100, nex=40, deg=20, tol=1e-10, cplx=True,
                 cfg=CFG_SMALL, n_lanczos=4, name=None) -> Problem:
    """Haar Q, lambda i.i.d. U[-1, 1] sorted (the small plain-FP64 workload
    at n=1000, nev=100, nex=40; the differentiation workload at n=8000)."""
    lam = spectrum_uniform_iid(n, rng(cfg, SLOT_LAMBDA))
    q = haar(n, rng(cfg, SLOT_Q), cplx)
    v0, s = start_blocks(cfg, n, nev + nex, n_lanczos, cplx)
    return Problem(name or f"uniform{n}", planted(lam, q), lam, q, v0, s, nev, nex, deg, tol)


def make_geometric(n=20000, nev=1000, nex=300, n_geo=None, deg=20, tol=1e-10,
                   cplx=True, cfg=CFG_GEO20K, n_lanczos=4) -> Problem:
    """Geometric cluster of the lowest 6% (1200 at n=20000) plus uniform [0,1]."""
    if n_geo is None:
        n_geo = (nev + nex) * 12 // 13 if n != 20000 else 1200
    lam = spectrum_geometric_low(n, rng(cfg, SLOT_LAMBDA), n_geo)
    q = haar(n, rng(cfg, SLOT_Q), cplx)
    v0, s = start_blocks(cfg, n, nev + nex, n_lanczos, cplx)
    return Problem(f"geometric{n}", planted(lam, q), lam, q, v0, s, nev, nex, deg, tol)


def make_cluster121(n=30000, nev=1500, nex=500, n_low=None, deg=20, tol=1e-10,
                    cplx=True, cfg=CFG_MIXED30K, n_lanczos=4) -> Problem:
    if n_low is None:
        n_low = nev + nex
    lam = spectrum_121_cluster(n, rng(cfg, SLOT_LAMBDA), n_low)
    q = haar(n, rng(cfg, SLOT_Q), cplx)
    v0, s = start_blocks(cfg, n, nev + nex, n_lanczos, cplx)
    return Problem(f"cluster121_{n}", planted(lam, q), lam, q, v0, s, nev, nex, deg, tol)


def make_tridiag(kind: str, n: int, nev: int, nex: int, deg=20, tol=1e-10,
                 cfg=CFG_SMALL, n_lanczos=4) -> Problem:
    d, e = tridiag_121(n) if kind == "121" else tridiag_wilkinson(n)
    h = dense_from_tridiag(d, e)
    if kind == "121":
        k = np.arange(1, n + 1)
        lam = 2.0 - 2.0 * np.cos(np.pi * k / (n + 1))
        # off-diagonal +1: the eigenvector of 2 - 2cos(pi k/(n+1)) is
        # sin(j (n+1-k) pi/(n+1)), j = 1..n
        j = np.arange(1, n + 1)[:, None]
        q = np.sin(j * (n + 1 - k[None, :]) * np.pi / (n + 1)) * math.sqrt(2.0 / (n + 1))
    else:
        lam, q = None, None
    v0, s = start_blocks(cfg, n, nev + nex, n_lanczos, False)
    return Problem(f"{kind}{n}", h, lam, q, v0, s, nev, nex, deg, tol)


def loss_weights(cfg: int, nev: int, ncols_b: int, n: int, cplx: bool):
    """w (nev) and B (n x ncols_b) for the loss sum w_i lambda_i + ||V^H B||_F^2."""
    w = rng(cfg, SLOT_W).standard_normal(nev)
    b = gaussian(rng(cfg, SLOT_B), (n, ncols_b), cplx)
    return w, b


# ------------------------------------------------------- device-side draws
def make_torch(kind: str, n: int, nev: int, nex: int, device="cuda", cplx=True,
               cfg=None, n_lanczos=4, deg=20, tol=1e-10, lam=None):
    """Large workloads drawn on the device with torch (seeded torch.Generator),
    the same recipe as the numpy builders: Haar Q from the QR of a Gaussian
    with phases fixed, H = Q diag(lam) Q^H symmetrised. Returns a dict of
    torch tensors in row-major layout plus the planted spectrum (numpy).
    ``lam`` (ascending) overrides the kind's spectrum."""
    import torch

    if cfg is None:
        cfg = {"geometric": CFG_GEO20K, "cluster121": CFG_MIXED30K, "uniform": CFG_DIFF8K}[kind]
    if lam is not None:
        lam = np.asarray(lam, dtype=np.float64)
    elif kind == "geometric":
        lam = spectrum_geometric_low(n, rng(cfg, SLOT_LAMBDA), 1200 if n == 20000 else (nev + nex) * 12 // 13)
    elif kind == "cluster121":
        lam = spectrum_121_cluster(n, rng(cfg, SLOT_LAMBDA), nev + nex)
    else:
        lam = spectrum_uniform_iid(n, rng(cfg, SLOT_LAMBDA))
    dt = torch.complex128 if cplx else torch.float64
    gq = torch.Generator(device=device)
    gq.manual_seed(BASE_SEED + 10 * cfg + SLOT_Q)
    z = torch.randn((n, n), generator=gq, dtype=dt, device=device)
    q, r = torch.linalg.qr(z)
    del z
    d = torch.diagonal(r)
    q *= (d / d.abs())[None, :]
    del r
    lam_t = torch.tensor(lam, dtype=torch.float64, device=device)
    h = torch.matmul(q * lam_t[None, :].to(dt), q.conj().T.contiguous())
    del q
    h = (h + h.conj().T) / 2
    gv = torch.Generator(device=device)
    gv.manual_seed(BASE_SEED + 10 * cfg + SLOT_V0)
    v0 = torch.randn((n, nev + nex), generator=gv, dtype=dt, device=device)
    gs = torch.Generator(device=device)
    gs.manual_seed(BASE_SEED + 10 * cfg + SLOT_S)
    s = torch.randn((n, n_lanczos), generator=gs, dtype=dt, device=device)
    return dict(H=h, lam=lam, V0=v0, S=s, nev=nev, nex=nex, deg=deg, tol=tol)


def make_torch_reflectors(n=100000, nev=2000, nex=600, nrefl=8, width=256, device="cuda",
                          block=4096, n_lanczos=4, cfg=CFG_HUGE100K, deg=20, tol=1e-10,
                          lam=None):
    """H = Q diag(lam) Q^H with Q = R_1 R_2 ... R_nrefl, R_j = I - 2 U_j U_j^H a
    block reflector (U_j: n x width, orthonormal columns from the QR of a
    seeded Gaussian), lam i.i.d. U[-1, 1].  H (complex128, n x n, row-major
    torch tensor) is assembled on the device one block of columns at a
    time and symmetrised block-pairwise, so no second n x n buffer is needed.
    Returns dict(H, lam, U (list), V0, S, ...).  ``apply_q(X, U, adjoint)``
    applies Q or Q^H to a block using the factored form."""
    import torch

    if lam is None:
        lam = spectrum_uniform_iid(n, rng(cfg, SLOT_LAMBDA))
    g = torch.Generator(device=device)
    g.manual_seed(BASE_SEED + 10 * cfg + SLOT_Q)
    us = []
    for _ in range(nrefl):
        z = torch.randn((n, width), generator=g, dtype=torch.complex128, device=device)
        if width == 1:  # elementary reflector: no factorization needed
            us.append((z / torch.linalg.vector_norm(z)).contiguous())
        else:
            u, _r = torch.linalg.qr(z)
            us.append(u.contiguous())
            del _r
        del z
    lam_t = torch.tensor(lam, dtype=torch.float64, device=device)
    H = torch.empty((n, n), dtype=torch.complex128, device=device)
    for j0 in range(0, n, block):
        j1 = min(n, j0 + block)
        x = torch.zeros((n, j1 - j0), dtype=torch.complex128, device=device)
        x[j0:j1, :] = torch.eye(j1 - j0, dtype=torch.complex128, device=device)
        x = apply_q(x, us, adjoint=True)
        x *= lam_t[:, None]
        x = apply_q(x, us, adjoint=False)
        H[:, j0:j1] = x
        del x
    # symmetrise: H <- (H + H^H)/2, block pair by block pair
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        for j0 in range(i0, n, block):
            j1 = min(n, j0 + block)
            t = (H[i0:i1, j0:j1] + H[j0:j1, i0:i1].mH) / 2
            H[i0:i1, j0:j1] = t
            H[j0:j1, i0:i1] = t.mH
            del t
    gv = torch.Generator(device=device)
    gv.manual_seed(BASE_SEED + 10 * cfg + SLOT_V0)
    v0 = torch.randn((n, nev + nex), generator=gv, dtype=torch.complex128, device=device)
    gs = torch.Generator(device=device)
    gs.manual_seed(BASE_SEED + 10 * cfg + SLOT_S)
    s = torch.randn((n, n_lanczos), generator=gs, dtype=torch.complex128, device=device)
    return dict(H=H, lam=lam, U=us, V0=v0, S=s, nev=nev, nex=nex, deg=deg, tol=tol)


def apply_q(x, us, adjoint):
    """Q x (adjoint=False) or Q^H x for Q = R_1 ... R_m, R_j = I - 2 U_j U_j^H."""
    order = us if adjoint else us[::-1]
    for u in order:
        x = x - 2.0 * (u @ (u.mH @ x))
    return x
