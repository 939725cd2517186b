"""chase_lanczos_noalloc (the entry point for callers that cannot allocate
device memory) against chase_lanczos, which runs the same kernels on a
handle's workspace: identical tridiagonals and bounds, on two calls in a
row, the second with a smaller problem (the fixed scratch keeps the first
call's contents, so whatever must start at zero has to be cleared by the
call itself)."""
import numpy as np
import pytest

import gen
from gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2205_02491_amd as pk
    pk.lib()
    return pk


def _case(pk, n, nvec, steps, n_e, cplx, seed):
    import torch
    g = np.random.Generator(np.random.PCG64(seed))
    lam = gen.spectrum_uniform_iid(n, g)
    H = torch.from_numpy(gen.planted(lam, gen.haar(n, g, cplx))).cuda()
    s = gen.gaussian(g, (n, nvec), cplx)
    # the no-allocation call takes S as the library reads it: the column-major
    # buffer of conj(S) (a view of an nvec x n tensor), which is what the
    # handle call's binding builds by copying
    S_cm = torch.from_numpy(np.ascontiguousarray(s.conj().T)).cuda().mT
    S_rm = torch.from_numpy(s).cuda()
    announce(f"lanczos no-alloc n={n} nvec={nvec} steps={steps} cplx={cplx}")
    ref = pk.chase_lanczos(H, S_rm, steps=steps, n_e=n_e,
                           opts=pk.default_opts(lanczos_vecs=nvec, lanczos_steps=steps))
    got = pk.chase_lanczos_noalloc(H, S_cm, n_e, steps=steps)
    assert got[0] == ref[0] and got[1] == ref[1] and got[2] == ref[2]
    np.testing.assert_array_equal(got[3], ref[3])
    np.testing.assert_array_equal(got[4], ref[4])
    np.testing.assert_array_equal(got[5], ref[5])


@pytest.mark.parametrize("cplx", [True, False])
def test_noalloc_lanczos_matches_handle_twice(pk, cplx):
    _case(pk, 1500, 4, 25, 120, cplx, 91 + cplx)
    _case(pk, 700, 2, 12, 40, cplx, 93 + cplx)

