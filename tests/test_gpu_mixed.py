"""Mixed-precision filter (FP32 or split-BF16 products, FP64 elsewhere,
per-column switch back to FP64): the final eigenpairs must meet the FP64 bar
against the FP64 oracle."""
import numpy as np
import pytest

import gen
import oracle
from gpu_util import announce, subspace_sin, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
@pytest.mark.parametrize("cplx", [True, False])
def test_mixed_solve_meets_fp64_bar(pk, cplx, prec):
    announce(f"mixed solve n=1000 cplx={cplx} prec={prec}")
    p = gen.make_uniform(n=1000, nev=100, nex=40, cplx=cplx, cfg=21)
    ev_o, v_o, r_o, st_o = oracle.solve(p.H, p.nev, p.nex, p.tol, p.deg, p.V0, p.S)
    o = pk.default_opts(filter_prec=pk.PREC_FP32 if prec == "fp32" else pk.PREC_BF16X3)
    ev, vec, res, st = pk.chase_solve(to_gpu(p.H), p.nev, p.nex, p.tol, p.deg, to_gpu(p.V0),
                                      to_gpu(p.S), opts=o)
    assert st["converged"]
    assert st["matvecs_low"] > 0
    norm = max(abs(p.lam[0]), abs(p.lam[-1]))
    assert np.max(np.abs(ev - ev_o)) <= 1e-10 * norm
    assert np.all(res <= p.tol)
    v = to_np(vec)
    assert np.linalg.norm(v.conj().T @ v - np.eye(p.nev)) <= 1e-12
    r = p.H @ v - v * ev[None, :]
    gap = p.lam[p.nev] - p.lam[p.nev - 1]
    bound = (np.linalg.norm(r) + np.linalg.norm(p.H @ v_o - v_o * ev_o[None, :])) / gap
    assert subspace_sin(v, v_o) <= max(2 * bound, 1e-8)
