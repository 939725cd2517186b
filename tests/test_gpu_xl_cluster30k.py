"""Full-size checks on the mixed-precision workload: n=30000 complex128, the
lowest 2000 eigenvalues those of the (1-2-1) matrix of order 30000 (Table 1's
(1-2-1) type: a cluster with gaps down to 1e-8), the rest uniform up to 10;
nev=1500, nex=500, degree 20, tol 1e-10.

This is the workload on which the low-precision policy does its work: the
solve takes more than ten iterations, so Ritz vectors are filtered in the
defect-correction form, pairs lock over many iterations, degrees are
re-optimised and the block is re-sorted into precision groups.  No oracle
finishes at this size; the checks are properties that hold at any size:
- eigenvalues against the planted spectrum, and mixed against FP64;
- every residual recomputed without the library (torch's GEMM on the stored
  H) and bounded by tol * ||H||_2;
- orthonormality of the returned vectors;
- the mixed solve's eigenspace against the FP64 one, within the sum of the
  two Davis-Kahan bounds ||R||_F / gap.
"""
import numpy as np
import pytest

import gen
from gpu_util import announce

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(400)]

N, NEV, NEX, TOL, DEG = 30000, 1500, 500, 1e-10, 20
_RESULTS = {}


@pytest.fixture(scope="module")
def problem():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    announce(f"generating cluster121 n={N} on the GPU")
    prob = gen.make_torch("cluster121", N, NEV, NEX, device="cuda")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    yield pk, prob
    _RESULTS.clear()
    del prob
    torch.cuda.empty_cache()


def _dk_bound(R_norms, ev, lam):
    """Davis-Kahan sin(theta) bound of the nev-subspace: ||R||_F over the gap
    between the largest returned eigenvalue and the rest of the spectrum."""
    gap = lam[NEV] - ev[NEV - 1]
    return float(np.sqrt(np.sum(R_norms ** 2)) / gap)


def _sin_angle(Va, Vb):
    """Sine of the largest principal angle between two orthonormal blocks,
    from the projection residual (accurate for tiny angles)."""
    import torch
    P = Vb - Va @ (Va.mH @ Vb)
    return float(torch.linalg.eigvalsh(P.mH @ P).max().clamp(min=0).sqrt())


@pytest.mark.parametrize("prec", ["fp64", "bf16x2", "fp32", "bf16x2i8", "fp64i8"])
def test_solve_cluster30k(problem, prec):
    """fp64i8 / bf16x2i8: the FP64 products (the filter's FP64 steps and
    Rayleigh-Ritz's H Q) on the INT8 matrix cores, 14 moduli."""
    import torch
    pk, prob = problem
    announce(f"full-size solve cluster121 n={N} prec={prec}")
    code = {"fp64": pk.PREC_FP64, "fp32": pk.PREC_FP32, "bf16x2": pk.PREC_BF16X2,
            "bf16x2i8": pk.PREC_BF16X2, "fp64i8": pk.PREC_FP64}[prec]
    H = prob["H"]
    ev, vec, res, st = pk.chase_solve(
        H, NEV, NEX, TOL, DEG, prob["V0"], prob["S"],
        opts=pk.default_opts(filter_prec=code, fp64_emulation=14 if prec.endswith("i8") else 0))
    announce(f"  {prec}: {st['t_all']:.1f} s, {st['iterations']} it, "
             f"matvecs fp64 {st['matvecs_fp64']} low {st['matvecs_low']}")
    assert st["converged"]
    # the multi-iteration path: locking over several iterations, degree
    # re-optimisation, and in the mixed modes the defect-form passes
    assert st["iterations"] >= 2
    if prec not in ("fp64", "fp64i8"):
        assert st["matvecs_low"] > 0
        assert st["matvecs_low"] > st["matvecs_fp64"]
    lam = prob["lam"]
    norm = max(abs(lam[0]), abs(lam[-1]))
    assert np.max(np.abs(ev - lam[:NEV])) <= 2e-10 * norm
    assert np.all(res <= TOL)
    # residuals recomputed without the library
    lam_t = torch.tensor(ev, dtype=torch.float64, device=vec.device)
    v = vec.contiguous()
    rn = torch.linalg.vector_norm(torch.matmul(H, v) - v * lam_t[None, :], dim=0).cpu().numpy()
    assert np.all(rn <= TOL * norm), (rn.max() / norm)
    g = v.mH @ v
    eye = torch.eye(NEV, dtype=g.dtype, device=g.device)
    assert float(torch.linalg.matrix_norm(g - eye)) < 1e-12
    _RESULTS[prec] = (ev, v, rn)
    if prec != "fp64" and "fp64" in _RESULTS:
        ev64, v64, rn64 = _RESULTS["fp64"]
        assert np.max(np.abs(ev - ev64)) <= 1e-10 * norm
        sin = _sin_angle(v64, v)
        bound = _dk_bound(rn64, ev64, lam) + _dk_bound(rn, ev, lam)
        announce(f"  {prec} vs fp64: max|dlambda|/||H|| "
                 f"{np.max(np.abs(ev - ev64)) / norm:.2e}, sin angle {sin:.2e} "
                 f"(Davis-Kahan {bound:.2e})")
        assert sin <= bound
