"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, validates arguments before touching a GPU, and sizes its
workspace consistently with the paper's one-GPU memory estimate."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chase.h")


def _lib():
    import paper_2205_02491_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pk.build_lib = __import__("paper_2205_02491_amd.build", fromlist=["build"])
        pk.build_lib.build()
    return pk


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chase_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    pk = _lib()
    L = pk.lib()
    names = header_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert sorted(pk.EXPORTED) == names


def test_default_opts():
    pk = _lib()
    o = pk.default_opts()
    assert (o.max_deg, o.deg_extra, o.optimize_degree, o.lanczos_steps, o.lanczos_vecs,
            o.max_iter, o.filter_prec, o.initial_rr, o.fp64_tail) == (36, 2, 1, 25, 4, 50, 0, 0, -1)
    assert (o.seed, o.debug, o.adjoint_reserve, o.eig_solver, o.fp64_emulation) == (0, 0, 0, 0, 0)


@pytest.mark.parametrize("struct", ["chase_opts", "chase_stats"])
def test_binding_structs_match_the_header(tmp_path, struct):
    """Every field of the ctypes mirrors sits at the offset the C compiler
    gives it in include/chase.h, and the sizes agree (a field added to one
    side only would shift the library's reads and writes)."""
    import subprocess
    pk = _lib()
    cls = {"chase_opts": pk.Opts, "chase_stats": pk.Stats}[struct]
    lines = [f'printf("%zu\\n", offsetof({struct}, {f}));' for f, _ in cls._fields_]
    lines.append(f'printf("%zu\\n", sizeof({struct}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "chase.h"\n'
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert out[:-1] == [getattr(cls, f).offset for f, _ in cls._fields_]
    assert out[-1] == ctypes.sizeof(cls)


def test_workspace_bytes_matches_one_gpu_memory_estimate():
    """Eq. (7) with a single GPU and a single rank (p = q = n, r_g = c_g = 1)
    gives n^2 + 3 n n_e + (2n + n_e) n_e elements, n^2 of which is the
    caller's matrix.  The library keeps three n x n_e blocks and two
    n_e x n_e matrices plus small buffers: it must stay within the estimate's
    non-matrix part plus the split-K workspace and Lanczos buffers, and
    grow linearly in n at fixed n_e."""
    pk = _lib()
    for n, nev, nex in [(1000, 100, 40), (20000, 1000, 300), (30000, 1500, 500)]:
        ne = nev + nex
        b = pk.chase_workspace_bytes(n, nev, nex, cplx=True)
        eq7_rest = (3 * n * ne + (2 * n + ne) * ne) * 16
        assert 3 * n * ne * 16 <= b <= eq7_rest + 400 * 2**20, (n, b, eq7_rest)
        b_real = pk.chase_workspace_bytes(n, nev, nex, cplx=False)
        assert b_real < b
    o = pk.default_opts(filter_prec=1)
    assert pk.chase_workspace_bytes(20000, 1000, 300, opts=o) >= 20000 ** 2 * 8
    # split-BF16 mode adds the split of H (rows padded to 32, columns to 256,
    # 4 bf16 per complex entry), two splits of the block (columns padded to
    # 128: a step's operand and the next step's, written by its epilogue),
    # 256 FP32 partial tiles of 256 x 128 (re and im) for the GEMM's split-K
    # tail and the residual block
    for n, nev, nex, cplx in [(30000, 1500, 500, True), (1000, 100, 40, False)]:
        ne, esz = nev + nex, (16 if cplx else 8)
        rows = -(-n // 32) * 32
        per = 8 if cplx else 4
        extra = rows * per * (-(-n // 256) * 256) + 2 * rows * per * (-(-ne // 128) * 128) \
            + 256 * 256 * 128 * (2 if cplx else 1) * 4 + n * ne * esz
        o3 = pk.default_opts(filter_prec=pk.PREC_BF16X3)
        b3 = pk.chase_workspace_bytes(n, nev, nex, cplx=cplx, opts=o3)
        assert b3 - pk.chase_workspace_bytes(n, nev, nex, cplx=cplx) == extra
        # the two-term form keeps the same splits (it only skips MFMAs)
        o2 = pk.default_opts(filter_prec=pk.PREC_BF16X2)
        assert pk.chase_workspace_bytes(n, nev, nex, cplx=cplx, opts=o2) == b3
    # adjoint buffers reserved at creation: two n x ne blocks for the
    # eigenvector adjoint and a tape of (steps + 1) n x ne blocks
    for cplx in (True, False):
        n, ne, esz = 8000, 260, (16 if cplx else 8)
        base = pk.chase_workspace_bytes(n, 200, 60, cplx=cplx)
        res = pk.chase_workspace_bytes(n, 200, 60, cplx=cplx,
                                       opts=pk.default_opts(adjoint_reserve=20))
        assert res - base == (2 + 21) * n * ne * esz
    # FP64 products on INT8: residue planes of H (three per modulus for
    # complex: Re, Im, Re + Im; one real) and row exponents, per-step planes
    # of the block with their INT32 products and column exponents
    for cplx, planes in ((True, 3), (False, 1)):
        n, ne, nm = 20000, 1300, 14
        base = pk.chase_workspace_bytes(n, 1000, 300, cplx=cplx)
        emu = pk.chase_workspace_bytes(n, 1000, 300, cplx=cplx,
                                       opts=pk.default_opts(fp64_emulation=nm))
        a256 = lambda b: -(-b // 256) * 256
        assert emu - base == (a256(planes * nm * n * n) + 4 * n + a256(planes * nm * n * ne)
                              + a256(4 * planes * nm * n * ne) + 4 * ne + 256)
    assert pk.chase_workspace_bytes(10, 8, 4) == 0      # nev + nex > n
    assert pk.chase_workspace_bytes(10, 0, 4) == 0


def test_create_rejects_bad_sizes_without_gpu():
    pk = _lib()
    L = pk.lib()
    h = ctypes.c_void_p()
    st = L.chase_create(ctypes.byref(h), 0, 10, 8, 4, None)
    assert st == pk.ERR_ARG
    assert b"nev + nex" in L.chase_last_error()
    st = L.chase_create(ctypes.byref(h), 7, 10, 2, 2, None)
    assert st == pk.ERR_ARG
    o = pk.default_opts(lanczos_vecs=9)
    st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
    assert st == pk.ERR_ARG
    o = pk.default_opts(filter_prec=4)
    st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
    assert st == pk.ERR_ARG and b"filter_prec" in L.chase_last_error()
    o = pk.default_opts(initial_rr=2)
    st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
    assert st == pk.ERR_ARG and b"initial_rr" in L.chase_last_error()
    for bad in (-2, 1001):
        o = pk.default_opts(fp64_tail=bad)
        st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
        assert st == pk.ERR_ARG and b"fp64_tail" in L.chase_last_error()
    for bad in (-1, 4, 9, 18):
        o = pk.default_opts(fp64_emulation=bad)
        st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
        assert st == pk.ERR_ARG and b"fp64_emulation" in L.chase_last_error()
    o = pk.default_opts(eig_solver=3)
    st = L.chase_create(ctypes.byref(h), 0, 100, 2, 2, ctypes.byref(o))
    assert st == pk.ERR_ARG and b"eig_solver" in L.chase_last_error()
    assert L.chase_eigvec_adjoint(None, None, 0, None, 0, 1, None, None, 0, None, 0, 1e-10, 10,
                                  None, None) == pk.ERR_ARG
    assert b"handle" in L.chase_last_error()
    assert L.chase_solve(None, None, 0, 0.0, 0, None, None, None, None, 0, None, None,
                         None) == pk.ERR_ARG
    assert L.chase_filter_adjoint(None, None, 0, None, 0, None, 0, None, None) == pk.ERR_ARG


def test_binding_refuses_to_run_without_library(tmp_path, monkeypatch):
    import paper_2205_02491_amd as pk
    monkeypatch.setattr(pk, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(pk, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        pk.lib()


def test_colmajor_buffers_are_materialised_copies():
    """The binding hands the library x.mH in new memory.  For a single
    vector x.mH is already contiguous: without materialising, the library
    would read x's unconjugated memory through a lazy conjugate view and
    write into the caller's tensor."""
    import torch
    pk = _lib()
    for shape in [(5, 1), (5, 3), (1, 1)]:
        for dt in (torch.complex128, torch.float64):
            x = torch.randn(shape, dtype=dt)
            b = pk._colmajor(x)
            assert not b.is_conj() and b.is_contiguous()
            assert b.data_ptr() != x.data_ptr()
            assert torch.equal(b, x.conj().T.resolve_conj())
    with pytest.raises(ValueError, match="lazy conjugate"):
        pk._dev(torch.randn(3, dtype=torch.complex128).conj())


def test_host_step_exports_match_oracle():
    """The three host-side exports (no GPU involved) against the oracle on
    the same Lanczos tridiagonals, coefficients and degree inputs."""
    import numpy as np

    import gen
    import oracle
    pk = _lib()
    g = np.random.Generator(np.random.PCG64(11))
    n, steps, nv, ne = 300, 25, 4, 40
    h = gen.planted(gen.spectrum_uniform_iid(n, g), gen.haar(n, g, True))
    s = gen.gaussian(g, (n, nv), True)
    runs = oracle.lanczos_runs(h, s, steps)
    a = np.zeros((nv, steps))
    b = np.zeros((nv, steps))
    for r, (ar, br) in enumerate(runs):
        a[r, : len(ar)] = ar
        b[r, : len(br)] = br
    b_ref, m1_ref, mne_ref, _ = oracle.spectral_bounds(h, s, steps, ne)
    b_sup, mu_1, mu_ne, lens = pk.chase_spectral_bounds(a, b, n, ne)
    assert lens == [len(ar) for ar, _ in runs]
    np.testing.assert_allclose([b_sup, mu_1, mu_ne], [b_ref, m1_ref, mne_ref], rtol=0, atol=1e-13)

    cf = pk.chase_filter_coefficients(20, b_sup, mu_1, mu_ne)
    ref = np.array(oracle.filter_coefficients(20, b_sup, mu_1, mu_ne)).reshape(20, 3)
    np.testing.assert_allclose(cf, ref, rtol=1e-15, atol=0)

    c, e = 0.5 * (b_sup + mu_ne), 0.5 * (b_sup - mu_ne)
    res = 10 ** g.uniform(-11, 0, 200)
    ritz = g.uniform(mu_1, mu_ne, 200)
    opts = oracle.Options()
    got = pk.chase_degrees(res, ritz, b_sup, mu_ne, 1e-10, 20)
    want = np.array([int(d) for d in oracle.degrees(res, ritz, c, e, 1e-10, opts, 20)])
    np.testing.assert_array_equal(got, want)
    fixed = pk.chase_degrees(res, ritz, b_sup, mu_ne, 1e-10, 17,
                             opts=pk.default_opts(optimize_degree=0))
    assert (fixed == 18).all()
    assert len(pk.chase_degrees([], [], b_sup, mu_ne, 1e-10)) == 0


def test_host_step_exports_reject_bad_arguments():
    import numpy as np
    pk = _lib()
    bad_coef = [(0, 1.0, -1.0, 0.0), (1001, 1.0, -1.0, 0.0), (5, 1.0, 0.5, 0.2),
                (5, float("nan"), -1.0, 0.0)]
    for args in bad_coef:
        with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
            pk.chase_filter_coefficients(*args)
    a = np.ones((2, 5))
    with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
        pk.chase_spectral_bounds(a, -a, 100, 10)            # negative beta
    with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
        pk.chase_spectral_bounds(a, a, 100, 101)            # n_e > n
    with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
        pk.chase_degrees([0.0], [0.1], 1.0, 0.5, 1e-10)     # zero residual
    with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
        pk.chase_degrees([1e-3], [0.1], 0.5, 1.0, 1e-10)    # mu_ne > b_sup
    with pytest.raises(pk.ChaseError, match="CHASE_ERR_ARG"):
        pk.chase_degrees([1e-3], [0.1], 1.0, 0.5, 1e-10, opts=pk.default_opts(max_deg=0))


class _FakeHandle:
    """Stand-in for a Handle (which needs a GPU to create): the binding checks
    its sizes against the arguments before any library call."""

    def __init__(self, n, nev, nex, cplx=True, tape_k=None):
        import paper_2205_02491_amd as pk
        self.n, self.nev, self.nex, self.cplx = n, nev, nex, cplx
        self.opts = pk.default_opts()
        self.tape_k = tape_k
        self.ptr = None


def test_binding_rejects_mismatched_handles_and_shapes():
    """The library sizes every device read and host write by the handle, so
    the binding refuses arguments that do not match it (a short V0 or degree
    array would otherwise be read past its end)."""
    import numpy as np
    import torch
    pk = _lib()
    n, nev, nex = 50, 6, 4
    ne = nev + nex
    c = torch.complex128
    H = torch.zeros((n, n), dtype=c)
    h = _FakeHandle(n, nev, nex)
    V0 = torch.zeros((n, ne), dtype=c)
    S = torch.zeros((n, 4), dtype=c)
    cases = [
        (lambda: pk.chase_solve(H, nev, nex, V0=V0, S=S, handle=_FakeHandle(n + 1, nev, nex)),
         "n=51"),
        (lambda: pk.chase_solve(H, nev, nex, V0=V0, S=S, handle=_FakeHandle(n, nev + 1, nex)),
         "nev=7"),
        (lambda: pk.chase_solve(H, nev, nex, V0=V0, S=S, handle=_FakeHandle(n, nev, nex, False)),
         "float64"),
        (lambda: pk.chase_solve(H, nev, nex, V0=V0[:, :ne - 1], S=S, handle=h), "V0 must"),
        (lambda: pk.chase_solve(H, nev, nex, V0=V0, S=S[:, :3], handle=h), "S must"),
        (lambda: pk.chase_solve(H[:, :n - 1], nev, nex, V0=V0, S=S, handle=h), "square"),
        (lambda: pk.chase_solve(H.T, nev, nex, V0=V0, S=S, handle=h) if not H.T.is_contiguous()
         else (_ for _ in ()).throw(ValueError("contiguous")), "contiguous"),
        (lambda: pk.chase_filter(H, V0, np.full(ne - 1, 2), 1.0, -1.0, 0.0, handle=h),
         "degrees must"),
        (lambda: pk.chase_filter(H, torch.zeros((n, ne + 1), dtype=c), np.full(ne + 1, 2),
                                 1.0, -1.0, 0.0, handle=h), "do not fit"),
        (lambda: pk.chase_filter(H, torch.zeros((n - 1, 3), dtype=c), np.full(3, 2),
                                 1.0, -1.0, 0.0, handle=h), "X must"),
        (lambda: pk.chase_filter_ritz(H, V0, V0[:, :3], np.zeros(ne), np.full(ne, 2),
                                      1.0, -1.0, 0.0, handle=h), "R must"),
        (lambda: pk.chase_filter_ritz(H, V0, V0, np.zeros(3), np.full(ne, 2),
                                      1.0, -1.0, 0.0, handle=h), "theta must"),
        (lambda: pk.chase_qr(torch.zeros((n, ne + 2), dtype=c), handle=h), "do not fit"),
        (lambda: pk.chase_qr(torch.zeros((n + 2, 3), dtype=c), handle=h), "n=52"),
        (lambda: pk.chase_rayleigh_ritz(H, torch.zeros((n - 2, 3), dtype=c), handle=h), "Q must"),
        (lambda: pk.chase_eigval_adjoint(V0[:, :3], np.zeros(2), torch.zeros((n, n), dtype=c),
                                         handle=h), "g must"),
        (lambda: pk.chase_eigval_adjoint(V0[:, :3], np.zeros(3), torch.zeros((n, n - 1), dtype=c),
                                         handle=h), "square"),
        (lambda: pk.chase_eigvec_adjoint(H, V0[:, :3], np.zeros(3), V0[:, :2],
                                         torch.zeros((n, n), dtype=c), handle=h), "G must"),
        (lambda: pk.chase_eigvec_adjoint(H, V0[:, :3], np.zeros(4), V0[:, :3],
                                         torch.zeros((n, n), dtype=c), handle=h), "lam must"),
        (lambda: pk.chase_filter_adjoint(H, V0, torch.zeros((n, n), dtype=c), h), "no recorded"),
        (lambda: pk.chase_filter_adjoint(H, V0[:, :2], torch.zeros((n, n), dtype=c),
                                         _FakeHandle(n, nev, nex, tape_k=3)), "gY must"),
        (lambda: pk.chase_lanczos(H, torch.zeros((n, 2), dtype=c), handle=_FakeHandle(n + 1, 2, 2)),
         "n=51"),
    ]
    for fn, msg in cases:
        with pytest.raises(ValueError, match=msg):
            fn()


def test_noalloc_lanczos_refuses_oversized_problems_without_gpu():
    """The no-allocation Lanczos entry point checks its scratch budget on the
    host: 200000 complex rows x 8 vectors need more than the 64 MiB array,
    so the call is refused before any pointer is read or GPU is touched."""
    pk = _lib()
    L = pk.lib()
    out = [ctypes.c_double() for _ in range(3)]
    st = L.chase_lanczos_noalloc(0, ctypes.c_void_p(256), 200000, 200000, 100,
                                 ctypes.c_void_p(256), 8, 25, ctypes.byref(out[0]),
                                 ctypes.byref(out[1]), ctypes.byref(out[2]), None, None, None,
                                 None)
    assert st == pk.ERR_ARG and b"scratch" in L.chase_last_error()
    st = L.chase_lanczos_noalloc(0, ctypes.c_void_p(256), 1000, 1000, 100, None, 4, 25,
                                 None, None, None, None, None, None, None)
    assert st == pk.ERR_ARG and b"NULL" in L.chase_last_error()
