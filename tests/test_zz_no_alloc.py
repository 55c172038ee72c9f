"""fa_apply_noalloc (through the C ABI) against fa_apply: the same solve in
the library's static device array instead of a caller workspace."""
import ctypes as C

import numpy as np
import pytest

import workloads as wl
from oracle import krylov as kr, operators as ops, polynomials as pl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_2401_06684_amd import _lib as L
    return L


def _noalloc(op, b, x, m_max, tol, flags=0, kind=0):
    L = _lib()
    st = L.fa_stats()
    torch.cuda.synchronize()
    r = L.lib().fa_apply_noalloc(op._h, kind, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                 int(m_max), float(tol), 0, int(flags),
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream),
                                 C.byref(st))
    return r, st.as_dict()


def test_noalloc_matches_fa_apply_twice_then_smaller():
    """Two calls in a row on one device, the second with a smaller operator
    (so the array holds the first call's larger basis): each equals fa_apply
    on the same input bit for bit (same kernels, deterministic reductions),
    and the first agrees with the oracle to 1e-10."""
    import paper_2401_06684_amd as fa
    L = _lib()
    cases = [((26, 24, 22), 8, 1), ((12, 10, 9), 4, 2)]
    for dims, degree, seed in cases:
        coeffs = wl.convdiff_stencil(max(dims), 50.0)
        op = fa.Stencil7(dims, coeffs)
        op.poly_setup(degree, "cheb")
        assert op.workspace_bytes(120) <= (64 << 20)
        bh = wl.rhs(op.n, seed=seed)
        b = torch.from_numpy(bh).to(DEV)
        x_ref, s_ref = op.apply(b, m_max=120, tol=1e-11)
        x = torch.full_like(b, float("nan"))
        r, s = _noalloc(op, b, x, 120, 1e-11)
        torch.cuda.synchronize()
        assert r == L.FA_OK
        assert s["iters"] == s_ref["iters"] and s["mvms"] == s_ref["mvms"]
        assert s["converged"] == 1
        assert torch.equal(x, x_ref)
        if seed == 1:
            a, bb = ops.stencil_interval(coeffs, dims)
            orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), bh,
                         pl.chebyshev(a, bb, degree), "invsqrt", m_max=120, tol=1e-11)
            xh = x.cpu().numpy()
            assert np.linalg.norm(xh - orc.x) <= 1e-10 * np.linalg.norm(orc.x)


def test_noalloc_sqrt_and_lanczos_match_fa_apply():
    """The square root on a Hermitian operator (Lanczos) and a fixed-m
    Arnoldi run with both Gram-Schmidt passes in every step: same bits as
    fa_apply."""
    import paper_2401_06684_amd as fa
    L = _lib()
    op = fa.Stencil7((20, 20, 20), wl.laplace_stencil(3), hermitian=True)
    op.poly_setup(4, "cheb")
    b = torch.from_numpy(wl.rhs(op.n, seed=3)).to(DEV)
    x_ref, s_ref = op.apply(b, kind="sqrt", m_max=150, tol=1e-10)
    x = torch.empty_like(b)
    r, s = _noalloc(op, b, x, 150, 1e-10, kind=L.FA_SQRT)
    assert r == L.FA_OK and s["iters"] == s_ref["iters"]
    assert torch.equal(x, x_ref)
    op2 = fa.Stencil7((17, 13, 11), wl.convdiff_stencil(17, 50.0))
    op2.poly_setup(3, "cheb")
    b2 = torch.from_numpy(wl.rhs(op2.n, seed=4)).to(DEV)
    x_ref, s_ref = op2.apply(b2, m_max=9, tol=0.0, orth="cgs2")
    x2 = torch.empty_like(b2)
    r, s = _noalloc(op2, b2, x2, 9, 0.0, flags=L.FA_CGS2)
    assert r >= 0 and s["iters"] == 9
    assert torch.equal(x2, x_ref)


def test_noalloc_refuses_what_does_not_fit():
    """A workspace beyond the array, and profiling (which creates events),
    are refused before any device work."""
    import paper_2401_06684_amd as fa
    L = _lib()
    op = fa.Stencil7((64, 64, 64), wl.convdiff_stencil(64, 50.0))
    op.poly_setup(4, "cheb")
    b = torch.from_numpy(wl.rhs(op.n, seed=0)).to(DEV)
    x = torch.zeros_like(b)
    assert op.workspace_bytes(200) > (64 << 20)
    r, _ = _noalloc(op, b, x, 200, 1e-8)
    assert r == L.FA_ERR_WORKSPACE
    r, _ = _noalloc(op, b, x, 10, 1e-8, flags=L.FA_PROFILE)
    assert r == L.FA_ERR_ARG
    assert torch.count_nonzero(x).item() == 0
