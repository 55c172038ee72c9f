"""The C-ABI library on the CPU: it loads, exports every declared symbol, and
its host-only logic (argument checks, spectral intervals, Chebyshev setup, the
dense H^{-1/2} e_1 routines) agrees with the oracle.  No GPU computation."""
import ctypes as C
import os
import re

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import krylov as kr, operators as ops, polynomials as pl
from paper_2401_06684_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fa.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fa_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert len(names) >= 16
    for name in names:
        assert hasattr(L, name), name
    assert sorted(_lib.EXPORTS) == names


def test_status_strings():
    L = _lib.lib()
    for code in range(-9, 2):
        assert L.fa_status_string(code).decode().startswith("FA_")


def _stencil(dims, coeffs, flags=0):
    L = _lib.lib()
    h = C.c_void_p()
    d4 = (C.c_int32 * 4)(*dims, 1)
    c7 = (C.c_double * 7)(*coeffs)
    st = L.fa_create_stencil(C.byref(h), _lib.FA_STENCIL7, d4, c7, 7, None, flags, None, 0,
                             None)
    return st, h


def test_create_stencil_validation():
    st, _ = _stencil((0, 4, 4), wl.laplace_stencil(3))
    assert st == _lib.FA_ERR_ARG
    st, _ = _stencil((4, 4, 4), [1.0, float("nan"), 0, 0, 0, 0, 0])
    assert st == _lib.FA_ERR_ARG
    # Hermitian flag needs a symmetric stencil
    st, _ = _stencil((4, 4, 4), wl.convdiff_stencil(4, 50.0), _lib.FA_HERMITIAN)
    assert st == _lib.FA_ERR_ARG
    st, h = _stencil((4, 4, 4), wl.laplace_stencil(3), _lib.FA_HERMITIAN)
    assert st == _lib.FA_OK
    assert _lib.lib().fa_destroy(h) == _lib.FA_OK


def test_create_wilson_validation_and_link_copy_without_gpu():
    """The Wilson op copies its links into caller operator memory at
    creation: argument and memory errors come first, then, without a GPU, the
    copy's failure is reported (nothing is created)."""
    L = _lib.lib()
    h = C.c_void_p()
    p = (C.c_double * 1)(0.05)
    d4 = (C.c_int32 * 4)(4, 4, 4, 4)
    mem = C.c_void_p(1 << 20)
    nb = L.fa_op_device_bytes(_lib.FA_WILSON4D, d4, 0, 0)
    # missing links, lattice extent below 2, Hermitian flag: argument errors
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 1, None, 0,
                               mem, nb, None) == _lib.FA_ERR_ARG
    d_bad = (C.c_int32 * 4)(4, 1, 4, 4)
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d_bad, p, 1, C.c_void_p(256), 0,
                               mem, nb, None) == _lib.FA_ERR_ARG
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 1, C.c_void_p(256),
                               _lib.FA_HERMITIAN, mem, nb, None) == _lib.FA_ERR_ARG
    # Q^2 (Gamma_5 D squared): only for the Wilson op; Hermitian only without a
    # chemical potential; at most 2 parameters, finite
    p2 = (C.c_double * 3)(-1.4, 0.3, 0.0)
    assert L.fa_create_stencil(C.byref(h), _lib.FA_STENCIL7, (C.c_int32 * 4)(4, 4, 4, 1),
                               (C.c_double * 7)(*([1.0] * 7)), 7, None, _lib.FA_Q2,
                               None, 0, None) == _lib.FA_ERR_ARG
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p2, 2, C.c_void_p(256),
                               _lib.FA_Q2 | _lib.FA_HERMITIAN, mem, nb, None) == _lib.FA_ERR_ARG
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p2, 3, C.c_void_p(256),
                               _lib.FA_Q2, mem, nb, None) == _lib.FA_ERR_ARG
    pinf = (C.c_double * 2)(-1.4, float("inf"))
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, pinf, 2, C.c_void_p(256),
                               _lib.FA_Q2, mem, nb, None) == _lib.FA_ERR_ARG
    # mu = 0: the Hermitian Q^2 passes the checks (then needs the GPU)
    p0 = (C.c_double * 2)(-1.4, 0.0)
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p0, 2, C.c_void_p(256),
                               _lib.FA_Q2 | _lib.FA_HERMITIAN, mem, nb, None) == _lib.FA_ERR_HIP
    # operator memory missing, too small for the two-row links, misaligned
    V = 4 ** 4
    for m, b in ((None, nb), (mem, 4 * 6 * 16 * V - 256), (C.c_void_p((1 << 20) + 8), nb)):
        assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 1, C.c_void_p(256), 0,
                                   m, b, None) == _lib.FA_ERR_WORKSPACE
    assert L.fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 1, C.c_void_p(256), 0,
                               mem, nb, None) == _lib.FA_ERR_HIP


def test_operator_memory_query():
    """fa_op_device_bytes: the caller-provided device memory of each operator
    kind (the library itself allocates none)."""
    L = _lib.lib()
    d4 = (C.c_int32 * 4)(16, 16, 16, 16)
    V = 16 ** 4
    # Wilson: whole links in the kernels' order, 4 directions x 9 complex per site
    assert L.fa_op_device_bytes(_lib.FA_WILSON4D, d4, 0, 0) == 4 * 9 * 16 * V
    d_odd = (C.c_int32 * 4)(3, 5, 7, 2)
    assert L.fa_op_device_bytes(_lib.FA_WILSON4D, d_odd, 0, 0) == \
        -(-4 * 9 * 16 * 210 // 256) * 256
    assert L.fa_op_device_bytes(_lib.FA_WILSON4D, (C.c_int32 * 4)(4, 1, 4, 4), 0, 0) == 0
    assert L.fa_op_device_bytes(_lib.FA_WILSON4D, None, 0, 0) == 0
    # CSR: the tables of row blocks (at most n, 4 int32 each), of chunks of
    # long rows (4 int32 each) and of long rows (3 int32 each), 256-byte rounded
    def up(b):
        return -(-b // 256) * 256

    for n, nnz in ((281903, 2594228), (1024, 4992), (5, 40000)):
        nl = nnz // 4097 + 1
        nc = 2 * nl + nnz // 4096
        assert L.fa_op_device_bytes(_lib.FA_CSR, None, n, nnz) == \
            up(16 * n) + up(16 * nc) + up(12 * nl)
    assert L.fa_op_device_bytes(_lib.FA_CSR, None, 0, 0) == 0
    assert L.fa_op_device_bytes(_lib.FA_STENCIL7, (C.c_int32 * 4)(8, 8, 8, 1), 0, 0) == 0
    assert L.fa_op_device_bytes(7, d4, 0, 0) == 0


@pytest.mark.parametrize("coeffs,dims", [
    (wl.laplace_stencil(2), (32, 32, 1)),
    (wl.laplace_stencil(3), (100, 100, 100)),
    (wl.convdiff_stencil(128, 50.0), (128, 128, 128)),
    (wl.convdiff_stencil(96, 50.0), (96, 96, 96)),
])
def test_stencil_interval_matches_oracle(coeffs, dims):
    st, h = _stencil(dims, coeffs)
    assert st == 0
    lo, hi = C.c_double(), C.c_double()
    assert _lib.lib().fa_get_spectral_interval(h, C.byref(lo), C.byref(hi)) == 0
    rlo, rhi = ops.stencil_interval(coeffs, dims)
    assert lo.value == pytest.approx(rlo, rel=1e-13)
    assert hi.value == pytest.approx(rhi, rel=1e-13)
    _lib.lib().fa_destroy(h)


@pytest.mark.parametrize("degree", [1, 2, 4, 8, 16, 32, 64])
def test_chebyshev_setup_matches_oracle(degree):
    dims = (128, 128, 128)
    coeffs = wl.convdiff_stencil(128, 50.0)
    st, h = _stencil(dims, coeffs)
    L = _lib.lib()
    assert L.fa_poly_setup(h, degree, _lib.FA_POLY_CHEB, None, None, 0, None) == 0
    deg, meth = C.c_int(), C.c_int()
    c = (C.c_double * (degree + 1))()
    iv = (C.c_double * 2)()
    assert L.fa_poly_get(h, C.byref(deg), C.byref(meth), c, None, None, None, iv, None) == 0
    assert deg.value == degree and meth.value == _lib.FA_POLY_CHEB
    a, b = ops.stencil_interval(coeffs, dims)
    ref = pl.chebyshev(a, b, degree).c
    assert np.allclose(np.array(c), ref, rtol=1e-13, atol=1e-15)
    L.fa_destroy(h)


def test_setup_and_apply_argument_errors_without_gpu():
    L = _lib.lib()
    st, h = _stencil((8, 8, 8), wl.laplace_stencil(3))
    # fa_apply before fa_poly_setup
    dummy = C.c_void_p(256)
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, None, 0, 0, None, None) == \
        _lib.FA_ERR_NO_POLY
    assert L.fa_poly_setup(h, 4, _lib.FA_POLY_CHEB, None, None, 0, None) == 0
    # workspace missing / too small / misaligned
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, None, 0, 0, None, None) == \
        _lib.FA_ERR_WORKSPACE
    need = L.fa_workspace_bytes(h, 10, 0)
    assert need > 11 * 512 * 8
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, C.c_void_p(4096), need - 8,
                      0, None, None) == _lib.FA_ERR_WORKSPACE
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, C.c_void_p(4100), need,
                      0, None, None) == _lib.FA_ERR_WORKSPACE
    # bad kind, aliasing, m_max
    assert L.fa_apply(h, 7, dummy, C.c_void_p(512), 10, 1e-8, 0, None, 0, 0, None, None) == \
        _lib.FA_ERR_ARG
    assert L.fa_apply(h, 0, dummy, dummy, 10, 1e-8, 0, None, 0, 0, None, None) == _lib.FA_ERR_ARG
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 0, 1e-8, 0, None, 0, 0, None, None) == \
        _lib.FA_ERR_ARG
    # a CSR op reads its row pointers to the host at creation: without a
    # GPU that copy fails and creation reports it
    h2 = C.c_void_p()
    assert L.fa_create_csr(C.byref(h2), 4, 4, C.c_void_p(256), C.c_void_p(512),
                           C.c_void_p(768), 0, 0, None, 0, None) == _lib.FA_ERR_HIP
    # Chebyshev without an interval: a stencil whose x pair has a negative
    # product (complex spectrum) gets none until it is set
    st, h2 = _stencil((4, 4, 4), [6.0, -1.0, 1.0, -1.0, -1.0, -1.0, -1.0])
    assert st == 0
    assert L.fa_poly_setup(h2, 3, _lib.FA_POLY_CHEB, None, None, 0, None) == _lib.FA_ERR_NO_INTERVAL
    assert L.fa_set_spectral_interval(h2, 2.0, 1.0) == _lib.FA_ERR_ARG
    assert L.fa_set_spectral_interval(h2, 0.5, 4.0) == 0
    assert L.fa_poly_setup(h2, 3, _lib.FA_POLY_CHEB, None, None, 0, None) == 0
    # Ritz needs a start vector
    assert L.fa_poly_setup(h2, 3, _lib.FA_POLY_RITZ, None, None, 0, None) == _lib.FA_ERR_ARG
    L.fa_destroy(h)
    L.fa_destroy(h2)


def test_chebyshev_branch_error_on_cut_interval():
    # a user interval that misses the top of the spectrum still passes the
    # positivity check on that interval (q > 0 there), like the oracle; the
    # error fires for an interval whose polynomial changes sign on it
    L = _lib.lib()
    st, h = _stencil((8, 8, 8), wl.laplace_stencil(3))
    assert L.fa_set_spectral_interval(h, 1e-9, 12.0) == 0
    ok = [L.fa_poly_setup(h, d, _lib.FA_POLY_CHEB, None, None, 0, None) for d in (1, 5, 31)]
    ref = []
    for d in (1, 5, 31):
        try:
            pl.chebyshev(1e-9, 12.0, d)
            ref.append(0)
        except pl.BranchError:
            ref.append(_lib.FA_ERR_BRANCH)
    assert ok == ref
    L.fa_destroy(h)


# ---- host dense routines against the oracle / scipy ----------------------
def _call_dense(H, beta):
    import paper_2401_06684_amd as fa
    return fa.dense_invsqrt_e1(H, beta)


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("m", [1, 2, 3, 17, 64, 150])
def test_dense_invsqrt_e1_matches_oracle(complex_, m):
    rng = np.random.default_rng(m)
    H = np.triu(rng.standard_normal((m, m)), -1) * 0.3 + 2.0 * np.eye(m)
    if complex_:
        H = H + 1j * np.triu(rng.standard_normal((m, m)), -1) * 0.3
    ref = kr.hessenberg_invsqrt_e1(H, 1.3)
    z = _call_dense(H, 1.3)
    assert np.allclose(z, ref, rtol=1e-11, atol=1e-13 * np.linalg.norm(ref))


def test_dense_invsqrt_e1_non_normal_arnoldi_hessenberg():
    # a Hessenberg from the oracle's Arnoldi on the non-normal conv-diff operator
    N = 10
    coeffs = wl.convdiff_stencil(N, 50.0)
    dims = (N, N, N)
    res = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), wl.rhs(N ** 3, seed=3), None,
                 "invsqrt", m_max=120, tol=0.0, keep_basis=True)
    H = res.H[:120, :120]
    ref = kr.hessenberg_invsqrt_e1(H, 2.0)
    assert np.allclose(_call_dense(H, 2.0), ref, rtol=1e-9, atol=1e-11 * np.linalg.norm(ref))


def test_dense_invsqrt_e1_branch_error():
    H = np.diag([2.0, -1.0, 3.0]) + np.diag([0.5, 0.5], -1)
    import paper_2401_06684_amd as fa
    with pytest.raises(fa.FAError) as e:
        fa.dense_invsqrt_e1(H, 1.0)
    assert e.value.status == _lib.FA_ERR_HESSENBERG


def test_dense_tridiag_matches_oracle():
    import paper_2401_06684_amd as fa
    rng = np.random.default_rng(5)
    for m in (1, 2, 40, 200):
        a = 2.0 + rng.random(m)
        b = 0.7 * rng.random(m - 1)
        ref = kr.tridiagonal_invsqrt_e1(a, b, 1.5)
        assert np.allclose(fa.dense_tridiag_invsqrt_e1(a, b, 1.5), ref, rtol=1e-11)
    # Toeplitz (equal diagonals: the shift meets ties), glued blocks with
    # negligible couplings (the deflation path), graded entries
    m = 300
    cases = [(np.full(m, 2.05), -np.ones(m - 1))]
    b = 0.5 * rng.random(m - 1)
    b[[40, 41, 150, 151, 152]] = [1e-18, 0.0, 1e-17, 3e-19, 0.0]
    cases.append((1.0 + rng.random(m), b))
    g = np.logspace(0, -6, 80)
    cases.append((g + 1e-3, 0.3 * np.sqrt(g[:-1] * g[1:])))
    for a, b in cases:
        ref = kr.tridiagonal_invsqrt_e1(a, b, 1.5)
        z = fa.dense_tridiag_invsqrt_e1(a, b, 1.5)
        assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    with pytest.raises(fa.FAError):
        fa.dense_tridiag_invsqrt_e1(np.array([1.0, -2.0]), np.array([0.1]), 1.0)


def test_fusion_flags():
    """The Python fuse argument maps onto the apply flags (True or 4: the
    default of four terms per launch; 3, 2; False or 1: one term per launch),
    and the library accepts each of those flags while rejecting an unknown
    bit (argument checks that run before any GPU work)."""
    import paper_2401_06684_amd as fa
    assert fa._fuse_flags(True) == 0 and fa._fuse_flags(4) == 0
    assert fa._fuse_flags(3) == _lib.FA_FUSE3
    assert fa._fuse_flags(2) == _lib.FA_FUSE2
    assert fa._fuse_flags(False) == _lib.FA_NO_FUSION and fa._fuse_flags(1) == _lib.FA_NO_FUSION
    with pytest.raises(ValueError):
        fa._fuse_flags(5)
    L = _lib.lib()
    st, h = _stencil((8, 8, 8), wl.laplace_stencil(3))
    assert st == 0
    assert L.fa_poly_setup(h, 4, _lib.FA_POLY_CHEB, None, None, 0, None) == 0
    dummy = C.c_void_p(256)
    for flags in (0, _lib.FA_FUSE3, _lib.FA_FUSE2, _lib.FA_NO_FUSION):
        # past the flag check: the missing workspace is what is reported
        assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, None, 0, flags, None,
                          None) == _lib.FA_ERR_WORKSPACE
    assert L.fa_apply(h, 0, dummy, C.c_void_p(512), 10, 1e-8, 0, None, 0, 1 << 20, None,
                      None) == _lib.FA_ERR_ARG
    L.fa_destroy(h)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; asked for more (flag or a multi-rank launch)
    it exits with status 2 and says why, before touching a GPU."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    bench = os.path.join(root, "bench.py")
    for extra, env in ((["--gpus", "2"], {}), ([], {"WORLD_SIZE": "2"})):
        r = subprocess.run([sys.executable, bench, *extra], capture_output=True, text=True,
                           env={**os.environ, **env}, timeout=120)
        assert r.returncode == 2
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_bench_oracle_leg_on_a_small_grid():
    """bench.py's oracle leg (the only bench code that calls the oracle): the
    references, the timed median of 3 whole solves with setup and host f(H)
    apart, and the 2D Poisson leg, on a 10^3 grid (CPU only)."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    N = 10
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 10.0)
    out = bench.cpu_baseline(coeffs, dims, 4, 1e-8)
    from oracle import exact
    b = wl.rhs(N ** 3, seed=0)
    xs = exact.stencil_fAb_dst(coeffs, dims, b, "invsqrt")
    assert np.linalg.norm(out["x_ref_invsqrt"] - xs) <= 1e-10 * np.linalg.norm(xs)
    xq = exact.stencil_fAb_dst(coeffs, dims, b, "sqrt")
    assert np.linalg.norm(out["x_ref_sqrt"] - xq) <= 1e-9 * np.linalg.norm(xq)
    assert out["kind"] == "oracle" and out["unit"] == "solves/s" and out["cores"] >= 1
    assert len(out["runs_s"]) == 3 and out["value"] == 1.0 / out["s_per_solve_median"]
    assert 0.0 <= out["s_setup"] < out["s_per_solve_median"]
    assert 0.0 < out["s_host_fH"] < out["s_per_solve_median"]
    assert out["rel_err_vs_ref"] < 1e-7
    for deg in (0, 8):
        assert out["poisson2d_32"][f"degree_{deg}"]["s_per_solve"] > 0
        r = out["poisson2d_32_ref"][deg]
        x2 = exact.stencil_fAb_dst(wl.laplace_stencil(2), (32, 32, 1), wl.rhs(1024, seed=0))
        assert np.linalg.norm(r - x2) <= 1e-10 * np.linalg.norm(x2)
