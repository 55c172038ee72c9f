"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (FP64 mode): one operator application or chain step 1e-13
relative; q(A) x 1e-12; whole solves 1e-10 (the bar for all-FP64 results),
both at a fixed Krylov dimension and at convergence.  Comparisons are element
by element (max-norm relative to the reference's max-norm) and in 2-norm.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import exact, krylov as kr, operators as ops, polynomials as pl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2401_06684_amd as fa
    fa.lib()  # the HIP library must load: no fallback


def fa():
    import paper_2401_06684_amd as m
    return m


def exported_newton_poly(op, real_operator):
    """The oracle's Newton-form polynomial on the nodes, coefficients and
    scaling the GPU exported (fa_poly_get), so that an oracle evaluation with
    it isolates the chain and the solve from the setup's rounding."""
    p = op.poly()
    return pl.Poly(kind="newton", degree=p["degree"], theta=np.array(p["theta"]),
                   eta=np.array(p["eta"]), rho=p["rho"], real_operator=real_operator)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_close(x, ref, tol):
    x = np.asarray(x)
    ref = np.asarray(ref)
    r2 = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    rinf = np.max(np.abs(x - ref)) / np.max(np.abs(ref))
    assert r2 <= tol and rinf <= 10 * tol, (r2, rinf)
    return r2


# --------------------------------------------------------------------------
# operators: one application y = A x
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [(70, 9, 11), (64, 4, 1), (37, 41, 23), (5, 3, 130), (1, 1, 7)])
def test_stencil_apply(dims):
    coeffs = wl.convdiff_stencil(max(dims), 50.0)
    op = fa().Stencil7(dims, coeffs)
    x = wl.rhs(int(np.prod(dims)), seed=1)
    y = host(op.op_apply(dev(x)))
    assert_close(y, ops.stencil_apply(coeffs, dims, x), 1e-14)


@pytest.mark.parametrize("which", ["poisson32", "digraph", "complex"])
def test_csr_apply(which):
    if which == "poisson32":
        rp, ci, va = wl.stencil_csr((32, 32, 1), wl.laplace_stencil(2))
    elif which == "digraph":
        rp, ci, va = wl.powerlaw_digraph_laplacian_csr(5000, 45000, seed=2)
    else:
        rp, ci, va = wl.stencil_csr((13, 11, 7), wl.convdiff_stencil(13, 50.0))
        va = va * (1.0 + 0.3j)
    n = len(rp) - 1
    x = wl.rhs(n, seed=3, complex_=np.iscomplexobj(va))
    op = fa().CSR(rp, ci, va)
    y = host(op.op_apply(dev(x)))
    assert_close(y, ops.csr_apply(rp, ci, va, x), 1e-14)


@pytest.mark.parametrize("links", ["su3", "scaled", "phase"])
@pytest.mark.parametrize("shape", [(4, 4, 4, 4), (6, 2, 4, 5), (4, 8, 4, 32), (4, 2, 6, 16),
                                   (8, 4, 4, 16), (16, 3, 8, 8)])
def test_wilson_apply(shape, links):
    """(Lt, Lz, Ly, Lx); the third and fourth shapes have whole 16-site rows.
    Special unitary links are kept as two rows (the third rebuilt in the
    kernel); links scaled by 1.01 or multiplied by a phase (unitary, det != 1)
    are not special unitary and are kept whole.  The last two shapes (whole
    64-site (x, y) planes, Lt a multiple of 8) take the t-walk workgroup
    order, with z-blocks of two planes and of one (odd Lz)."""
    Lt, Lz, Ly, Lx = shape
    rng_links = wl.random_su3(4 * Lt * Lz * Ly * Lx, 0.8, np.random.default_rng(5))
    if links == "scaled":
        rng_links = 1.01 * rng_links
    elif links == "phase":
        rng_links = np.exp(0.3j) * rng_links
    U = rng_links.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    m0 = 0.05
    op = fa().Wilson(U, m0)
    x = wl.rhs(op.n, seed=4, complex_=True)
    y = host(op.op_apply(dev(x)))
    assert_close(y, ops.wilson_apply(U, m0, x), 1e-14)


def test_wilson_links_copied_at_creation():
    """The op keeps its own (reordered) copy of the links: the caller's
    device array can be overwritten and freed after creation."""
    import ctypes as C
    from paper_2401_06684_amd import _lib
    Lt = Lz = Ly = Lx = 4
    U = wl.random_su3(4 * Lt * Lz * Ly * Lx, 0.8, np.random.default_rng(7))
    U = U.reshape(4, Lt, Lz, Ly, Lx, 3, 3)
    dU = torch.from_numpy(np.ascontiguousarray(U)).to(DEV)
    h = C.c_void_p()
    d4 = (C.c_int32 * 4)(Lx, Ly, Lz, Lt)
    p = (C.c_double * 1)(0.05)
    nb = _lib.lib().fa_op_device_bytes(_lib.FA_WILSON4D, d4, 0, 0)
    mem = torch.empty(nb, dtype=torch.uint8, device=DEV)  # torch-owned operator memory
    assert mem.data_ptr() % 256 == 0
    st = _lib.lib().fa_create_stencil(C.byref(h), _lib.FA_WILSON4D, d4, p, 1,
                                      C.c_void_p(dU.data_ptr()), 0,
                                      C.c_void_p(mem.data_ptr()), nb, None)
    assert st == 0
    dU.fill_(float("nan"))  # the caller's array changes ...
    torch.cuda.synchronize()
    del dU                  # ... and goes away
    torch.cuda.empty_cache()
    x = wl.rhs(12 * Lt * Lz * Ly * Lx, seed=4, complex_=True)
    dx, dy = dev(x), torch.empty(x.shape, dtype=torch.complex128, device=DEV)
    torch.cuda.synchronize()
    assert _lib.lib().fa_op_apply(h, C.c_void_p(dx.data_ptr()), C.c_void_p(dy.data_ptr()),
                                  None, 0, None) == 0
    assert_close(host(dy), ops.wilson_apply(U, 0.05, x), 1e-14)
    assert _lib.lib().fa_destroy(h) == 0


# --------------------------------------------------------------------------
# polynomial chain q(A) x
# --------------------------------------------------------------------------
@pytest.mark.parametrize("degree", [1, 2, 3, 4, 16, 32])
def test_chebyshev_chain(degree):
    dims = (70, 9, 11)
    coeffs = wl.convdiff_stencil(70, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    a, b = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, b, degree)
    x = wl.rhs(op.n, seed=2)
    y = host(op.poly_apply(dev(x)))
    ref, _ = q.apply(lambda v: ops.stencil_apply(coeffs, dims, v), x)
    assert_close(y, ref, 1e-12)


def test_ritz_setup_and_chain_wilson():
    L = 4
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    op = fa().Wilson(U, m0)
    start = wl.rhs(op.n, seed=11, complex_=True)
    op.poly_setup(8, "ritz", start=dev(start))
    p = op.poly()
    apply_A = lambda v: ops.wilson_apply(U, m0, v)
    q = pl.ritz(apply_A, start, 8, real_operator=False)
    key = lambda z: (round(z.real, 6), round(z.imag, 6))
    gt = np.array(sorted(p["theta"], key=key))
    rt = np.array(sorted(q.theta, key=key))
    assert p["degree"] == q.degree == 8
    assert np.max(np.abs(gt - rt)) <= 1e-9 * np.max(np.abs(rt))
    x = wl.rhs(op.n, seed=12, complex_=True)
    y = host(op.poly_apply(dev(x)))
    # against the oracle's own setup: the nodes differ by setup rounding
    ref, _ = q.apply(apply_A, x)
    assert_close(y, ref, 1e-8)
    # against the oracle's Horner recurrence on the exported nodes
    ref, _ = exported_newton_poly(op, False).apply(apply_A, x)
    assert_close(y, ref, 1e-12)


# --------------------------------------------------------------------------
# whole solves
# --------------------------------------------------------------------------
@pytest.mark.parametrize("degree,m", [(0, 40), (4, 10), (16, 5)])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_convdiff_fixed_m(degree, m, kind):
    dims = (20, 18, 16)
    coeffs = wl.convdiff_stencil(20, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    b = wl.rhs(op.n, seed=0)
    x, st = op.apply(dev(b), kind=kind, m_max=m, tol=0.0)
    a, bb = ops.stencil_interval(coeffs, dims)
    ref = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, pl.chebyshev(a, bb, degree),
                 kind, m_max=m, tol=0.0)
    assert st["iters"] == ref.iters == m
    assert st["mvms"] == ref.mvms
    assert_close(host(x), ref.x, 1e-10)


@pytest.mark.parametrize("degree", [0, 4])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_cgs2_every_step_against_oracle(degree, kind):
    """orth="cgs2" (FA_CGS2): both classical Gram-Schmidt passes in every
    Arnoldi step, the oracle's own scheme, on the non-normal Pe = 50 stencil
    (ragged tiles): fixed m (same iterate, products with A and inner products)
    and at convergence with both sides at tol 1e-12; the delayed scheme (the
    default) gives the same result."""
    dims = (21, 18, 13)
    coeffs = wl.convdiff_stencil(21, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)  # noqa: E731
    b = wl.rhs(op.n, seed=0)
    m = 30 if degree == 0 else 12
    x, st = op.apply(dev(b), kind=kind, m_max=m, tol=0.0, orth="cgs2")
    ref = kr.fAb(A, b, q, kind, m_max=m, tol=0.0, orth="cgs2")
    assert st["iters"] == ref.iters == m
    assert st["mvms"] == ref.mvms and st["inner_products"] == ref.inner_products
    assert_close(host(x), ref.x, 1e-10)
    x, st = op.apply(dev(b), kind=kind, m_max=300, tol=1e-12, orth="cgs2")
    ref = kr.fAb(A, b, q, kind, m_max=300, tol=1e-12, orth="cgs2")
    assert st["converged"] == 1 and st["iters"] == ref.iters
    assert st["mvms"] == ref.mvms and st["inner_products"] == ref.inner_products
    assert_close(host(x), ref.x, 1e-10)
    xd, sd = op.apply(dev(b), kind=kind, m_max=300, tol=1e-12)
    assert sd["iters"] == st["iters"]
    assert_close(host(xd), host(x), 1e-10)


@pytest.mark.parametrize("degree", [0, 4, 16])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_convdiff_converged_against_closed_form(degree, kind):
    N = 24
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 10.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    b = wl.rhs(op.n, seed=0)
    x, st = op.apply(dev(b), kind=kind, m_max=400, tol=1e-12)
    assert st["converged"] == 1
    ref = exact.stencil_fAb_dst(coeffs, dims, b, kind)
    assert_close(host(x), ref, 1e-10)
    a, bb = ops.stencil_interval(coeffs, dims)
    orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, pl.chebyshev(a, bb, degree),
                 kind, m_max=400, tol=1e-12)
    assert st["iters"] == orc.iters
    assert_close(host(x), orc.x, 1e-10)


@pytest.mark.parametrize("hermitian", [False, True])
@pytest.mark.parametrize("check_every", [1, 3])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_check_overlap_leaves_no_trace(hermitian, check_every, kind):
    """At a check the first half of the next step is enqueued before the host
    waits for the check's copies; when the iteration stops at that check the
    half step must change nothing: iterations and products with A equal the
    oracle's (and Lanczos' inner products), x agrees with the oracle."""
    N = 20
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3) if hermitian else wl.convdiff_stencil(N, 10.0)
    op = fa().Stencil7(dims, coeffs, hermitian=hermitian)
    op.poly_setup(4, "cheb")
    b = wl.rhs(op.n, seed=3)
    x, st = op.apply(dev(b), kind=kind, m_max=300, tol=1e-11, check_every=check_every)
    assert st["converged"] == 1
    a, bb = ops.stencil_interval(coeffs, dims)
    orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, pl.chebyshev(a, bb, 4), kind,
                 m_max=300, tol=1e-11, check_every=check_every,
                 orth="lanczos" if hermitian else "cgs2")
    assert st["iters"] == orc.iters
    assert st["mvms"] == orc.mvms
    if hermitian:
        assert st["inner_products"] == orc.inner_products
    assert_close(host(x), orc.x, 1e-10)
    # the same solve again gives the same bits (the half steps are enqueued
    # at the same checks)
    x2, st2 = op.apply(dev(b), kind=kind, m_max=300, tol=1e-11, check_every=check_every)
    assert torch.equal(x, x2) and st2["mvms"] == st["mvms"]


@pytest.mark.parametrize("N,degree,tol", [(10, 48, 1e-6), (10, 32, 1e-6), (12, 16, 1e-6),
                                           (12, 48, 1e-8)])
def test_checks_every_step_count_no_work_enqueued_ahead(N, degree, tol):
    """Delayed CGS2 with a check after every step: a check the iteration is
    expected to pass enqueues the next step and the first half of the one
    after it; when the iteration stops at the following check (m = 2, 3, 4
    here) neither may show in the counts.  Iterations and products with A
    equal the oracle's, x agrees with it."""
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 10.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    b = wl.rhs(op.n, seed=3)
    x, st = op.apply(dev(b), m_max=50, tol=tol, check_every=1)
    a, bb = ops.stencil_interval(coeffs, dims)
    orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, pl.chebyshev(a, bb, degree),
                 "invsqrt", m_max=50, tol=tol, check_every=1, orth="cgs2")
    assert st["converged"] == 1
    assert st["iters"] == orc.iters
    assert st["mvms"] == orc.mvms
    assert_close(host(x), orc.x, 1e-10)


@pytest.mark.parametrize("degree", [0, 8])
def test_poisson2d_32_lanczos(degree):
    """2D Poisson 32x32, CSR, Hermitian: Lanczos, m_max 200.  Compared at
    convergence (plain Lanczos loses orthogonality, so fixed-m iterates are
    rounding-sensitive): both sides at tol 1e-12, agreement to 1e-10 with the
    oracle and with the DST closed form."""
    N = 32
    coeffs = wl.laplace_stencil(2)
    rp, ci, va = wl.stencil_csr((N, N, 1), coeffs)
    op = fa().CSR(rp, ci, va, hermitian=True)
    lo, hi = ops.stencil_interval(coeffs, (N, N, 1))
    op.set_spectral_interval(lo, hi)
    op.poly_setup(degree, "cheb")
    b = wl.rhs(N * N, seed=0)
    x, st = op.apply(dev(b), kind="invsqrt", m_max=200, tol=1e-12)
    assert st["inner_products"] == 2 * st["iters"]
    orc = kr.fAb(lambda v: ops.csr_apply(rp, ci, va, v), b, pl.chebyshev(lo, hi, degree),
                 "invsqrt", m_max=200, tol=1e-12, orth="lanczos")
    assert st["iters"] == orc.iters and st["converged"] == orc.converged
    assert_close(host(x), orc.x, 1e-10)
    assert_close(host(x), exact.stencil_fAb_dst(coeffs, (N, N, 1), b), 1e-10)
    # the configuration's own tolerance 1e-10: the error is below it
    x10, st10 = op.apply(dev(b), kind="invsqrt", m_max=200, tol=1e-10)
    assert st10["converged"] == 1
    assert_close(host(x10), exact.stencil_fAb_dst(coeffs, (N, N, 1), b), 1e-10)


@pytest.mark.parametrize("degree", [0, 8])
def test_wilson_solve(degree):
    L = 4
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    op = fa().Wilson(U, m0)
    start = wl.rhs(op.n, seed=11, complex_=True)
    op.poly_setup(degree, "ritz", start=dev(start))
    b = wl.rhs(op.n, seed=0, complex_=True)
    x, st = op.apply(dev(b), kind="invsqrt", m_max=400, tol=1e-12)
    assert st["converged"] == 1
    apply_A = lambda v: ops.wilson_apply(U, m0, v)
    q = pl.ritz(apply_A, start, degree, real_operator=False)
    orc = kr.fAb(apply_A, b, q, "invsqrt", m_max=400, tol=1e-12)
    assert_close(host(x), orc.x, 1e-10)


@pytest.mark.parametrize("L", [4, 8])
def test_wilson_free_field_closed_form(L):
    """(D = free Wilson operator) A^{-1/2} b against its momentum-space closed
    form; the 8^4 lattice takes the t-walk workgroup order."""
    Ls = (L, L, L, L)
    U = np.zeros((4, *Ls, 3, 3), dtype=complex)
    U[...] = np.eye(3)
    m0 = 0.1
    op = fa().Wilson(U, m0)
    op.poly_setup(6, "ritz", start=dev(wl.rhs(op.n, seed=1, complex_=True)))
    b = wl.rhs(op.n, seed=0, complex_=True)
    x, st = op.apply(dev(b), kind="invsqrt", m_max=400, tol=1e-12)
    assert_close(host(x), exact.wilson_free_fAb(Ls, m0, b), 1e-10)


# --------------------------------------------------------------------------
# degenerate cases and error paths
# --------------------------------------------------------------------------
def test_zero_rhs_returns_zero():
    op = fa().Stencil7((10, 10, 10), wl.convdiff_stencil(10, 50.0))
    op.poly_setup(4, "cheb")
    x, st = op.apply(torch.zeros(1000, dtype=torch.float64, device=DEV), m_max=20, tol=1e-10)
    assert st["converged"] == 1 and st["iters"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_nonfinite_rhs():
    op = fa().Stencil7((10, 10, 10), wl.convdiff_stencil(10, 50.0))
    op.poly_setup(4, "cheb")
    b = wl.rhs(1000, seed=0)
    b[17] = np.nan
    with pytest.raises(fa().FAError) as e:
        op.apply(dev(b), m_max=20, tol=1e-10)
    assert e.value.status == -7


def test_lucky_breakdown_diagonal():
    a = np.repeat([0.5, 1.5, 4.0, 9.0], 300)
    n = a.size
    rp = np.arange(n + 1, dtype=np.int32)
    op = fa().CSR(rp, np.arange(n, dtype=np.int32), a)
    op.poly_setup(0)
    b = wl.rhs(n, seed=3)
    for kind, f in (("invsqrt", a ** -0.5), ("sqrt", a ** 0.5)):
        x, st = op.apply(dev(b), kind=kind, m_max=50, tol=1e-12, check_every=5)
        assert st["breakdown"] == 1 and st["iters"] == 4
        assert_close(host(x), f * b, 1e-12)


def test_csr_creation_rejects_bad_indices():
    """fa_create_csr reads the index arrays to the host and refuses row
    pointers out of order and column indices outside [0, n) (the kernels
    index with them unchecked), before any kernel runs."""
    import ctypes as C
    from paper_2401_06684_amd import _lib
    rp, ci, va = wl.stencil_csr((8, 8, 1), wl.laplace_stencil(2))
    n, nnz = len(rp) - 1, len(ci)
    L = _lib.lib()
    mem = torch.empty(L.fa_op_device_bytes(_lib.FA_CSR, None, n, nnz), dtype=torch.uint8,
                      device=DEV)
    for bad in ("col_high", "col_neg", "rowptr"):
        r, c = rp.copy(), ci.copy()
        if bad == "col_high":
            c[nnz // 2] = n
        elif bad == "col_neg":
            c[3] = -1
        else:
            r[5], r[6] = r[6], r[5]
        dr = torch.from_numpy(r.astype(np.int32)).to(DEV)
        dc = torch.from_numpy(c.astype(np.int32)).to(DEV)
        dv = dev(va)
        h = C.c_void_p()
        st = L.fa_create_csr(C.byref(h), n, nnz, C.c_void_p(dr.data_ptr()),
                             C.c_void_p(dc.data_ptr()), C.c_void_p(dv.data_ptr()), 0, 0,
                             C.c_void_p(mem.data_ptr()), mem.numel(),
                             C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == _lib.FA_ERR_ARG, bad
    # the valid matrix is accepted
    with pytest.raises(fa().FAError):
        fa().CSR(rp, np.where(np.arange(nnz) == 7, n + 3, ci), va)
    op = fa().CSR(rp, ci, va)
    x = wl.rhs(n, seed=1)
    assert_close(host(op.op_apply(dev(x))), ops.csr_apply(rp, ci, va, x), 1e-14)


def test_branch_and_hessenberg_errors():
    a = np.concatenate([[-1.0], np.linspace(1, 3, 99)])
    n = a.size
    rp = np.arange(n + 1, dtype=np.int32)
    op = fa().CSR(rp, np.arange(n, dtype=np.int32), a)
    with pytest.raises(fa().FAError) as e:
        op.poly_setup(8, "ritz", start=dev(wl.rhs(n, seed=1)))
    assert e.value.status == -3
    op.poly_setup(0)
    with pytest.raises(fa().FAError) as e:
        op.apply(dev(wl.rhs(n, seed=2)), m_max=n, tol=1e-12, check_every=1)
    assert e.value.status == -4


def test_not_converged_warning():
    op = fa().Stencil7((16, 16, 16), wl.convdiff_stencil(16, 50.0))
    op.poly_setup(0)
    x, st = op.apply(dev(wl.rhs(op.n, seed=0)), m_max=10, tol=1e-12)
    assert st["status"] == 1 and st["converged"] == 0 and st["iters"] == 10


def test_bitwise_deterministic_and_profile():
    op = fa().Stencil7((40, 33, 29), wl.convdiff_stencil(40, 50.0))
    op.poly_setup(12, "cheb")
    b = dev(wl.rhs(op.n, seed=0))
    x1, s1 = op.apply(b, m_max=60, tol=1e-10)
    x2, s2 = op.apply(b, m_max=60, tol=1e-10, profile=True)
    assert torch.equal(x1, x2)
    # Clenshaw degree 12 = 12 terms = three launches of 4 terms per q(A), of
    # which the middle one reads x, v, b_{k+2} and writes its last two terms
    # (5 vectors); 2 q(A) per step plus c = q(A) b
    assert s2["n_chain"] == 2 * s2["iters"] + 1 and s2["ms_chain"] > 0
    assert s2["n_chain_terms"] == 4 * s2["n_chain"]
    assert s2["chain_bytes"] == 5 * 8 * op.n
    # at most three terms per launch: 4 triples, the 2nd and 3rd timed
    x5, s5 = op.apply(b, m_max=60, tol=1e-10, fuse=3, profile=True)
    assert s5["n_chain"] == 2 * (2 * s5["iters"] + 1)
    assert s5["n_chain_terms"] == 3 * s5["n_chain"]
    assert s5["chain_bytes"] == 5 * 8 * op.n
    # at most two terms per launch: 6 pairs, the 2nd to 5th timed
    x4, s4 = op.apply(b, m_max=60, tol=1e-10, fuse=2, profile=True)
    assert s4["n_chain"] == 4 * (2 * s4["iters"] + 1)
    assert s4["n_chain_terms"] == 2 * s4["n_chain"]
    assert s4["chain_bytes"] == 5 * 8 * op.n
    # the grouping only drops zero terms and keeps every rounding: same bits
    assert torch.equal(x5, x1)
    assert torch.equal(x4, x1)
    x3, s3 = op.apply(b, m_max=60, tol=1e-10, fuse=False, profile=True)
    # one term per launch: terms 2 .. 10 timed (the first two have no b_{k+2},
    # the last is not a middle term)
    assert s3["n_chain"] == 9 * (2 * s3["iters"] + 1)
    assert s3["chain_bytes"] == 4 * 8 * op.n
    assert_close(host(x3), host(x1), 1e-13)


@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5, 6, 7, 16, 17])
@pytest.mark.parametrize("dims", [(70, 9, 11), (128, 16, 24), (33, 65, 5), (20, 20, 1)])
def test_multi_term_launches_match_single_terms(degree, dims):
    """q(A) x and whole solves with four, three or two recurrence terms per
    launch equal the single-term path and the oracle (ragged tiles in x, y
    and z; degrees that leave a single term, a pair or a triple after the
    groups of four)."""
    coeffs = wl.convdiff_stencil(max(dims), 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    a, b = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, b, degree)
    x = wl.rhs(op.n, seed=2)
    ref, _ = q.apply(lambda v: ops.stencil_apply(coeffs, dims, v), x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-12)
    bd = dev(wl.rhs(op.n, seed=0))
    m = min(6, op.n)
    x1, _ = op.apply(bd, m_max=m, tol=0.0)
    x2, _ = op.apply(bd, m_max=m, tol=0.0, fuse=False)
    x3, _ = op.apply(bd, m_max=m, tol=0.0, fuse=2)
    x4, _ = op.apply(bd, m_max=m, tol=0.0, fuse=3)
    assert_close(host(x1), host(x2), 1e-12)
    # four- and three-term groups reproduce the pairs bit for bit (same roundings)
    assert torch.equal(x1, x3)
    assert torch.equal(x1, x4)



@pytest.mark.parametrize("degree", [4, 16, 17])
@pytest.mark.parametrize("dims", [(64, 256, 62), (64, 256, 63)])
def test_paired_slabs_uneven_last_pair(degree, dims):
    """Grids that take paired z-slabs (512 workgroups, 32 x-y tiles, slabs
    of 4 planes, the first of each pair 2 planes longer) where the last
    pair is cut by the grid: at nz = 62 its second slab is empty, at
    nz = 63 it has one plane.  q(A) x against the oracle; solves with four,
    three and two terms per launch the same bits."""
    coeffs = wl.convdiff_stencil(max(dims), 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    a, b = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, b, degree)
    x = wl.rhs(op.n, seed=4)
    ref, _ = q.apply(lambda v: ops.stencil_apply(coeffs, dims, v), x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-12)
    bd = dev(wl.rhs(op.n, seed=0))
    x1, _ = op.apply(bd, m_max=4, tol=0.0)
    x3, _ = op.apply(bd, m_max=4, tol=0.0, fuse=2)
    x4, _ = op.apply(bd, m_max=4, tol=0.0, fuse=3)
    assert torch.equal(x1, x3)
    assert torch.equal(x1, x4)



def test_convdiff_256_paired_slabs():
    """The 256^3 grid (one launch's five vectors 671 MB, beyond the
    Infinity Cache) in the launch the bench times there: 512 workgroups,
    paired slabs of 66 and 62 planes.  q(A) x (degree 4, one four-term
    launch) against the oracle, and a fixed-m degree-16 solve whose
    four-term launches equal the two-term path bit for bit."""
    N = 256
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(4, "cheb")
    a, b = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, b, 4)
    x = wl.rhs(op.n, seed=5)
    ref, _ = q.apply(lambda v: ops.stencil_apply(coeffs, dims, v), x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-12)
    del ref
    op.poly_setup(16, "cheb")
    bd = dev(wl.rhs(op.n, seed=0))
    x1, _ = op.apply(bd, m_max=2, tol=0.0)
    x2, _ = op.apply(bd, m_max=2, tol=0.0, fuse=2)
    assert torch.equal(x1, x2)


# --------------------------------------------------------------------------
# the 128^3 convection-diffusion workload at full size
# --------------------------------------------------------------------------
def test_convdiff_128_full_size():
    N = 128
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(16, "cheb")
    b = wl.rhs(op.n, seed=0)
    bd = dev(b)
    # fixed m = 3 against the oracle (the oracle needs ~10^2 products with A)
    x3, st = op.apply(bd, m_max=3, tol=0.0)
    a, bb = ops.stencil_interval(coeffs, dims)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    ref = kr.fAb(A, b, pl.chebyshev(a, bb, 16), "invsqrt", m_max=3, tol=0.0)
    assert_close(host(x3), ref.x, 1e-10)
    # converged solves: invsqrt and sqrt related by A, degree 16 vs 32
    xi, si = op.apply(bd, kind="invsqrt", m_max=200, tol=1e-10)
    xs, ss = op.apply(bd, kind="sqrt", m_max=200, tol=1e-10)
    assert si["converged"] and ss["converged"]
    assert_close(A(host(xi)), host(xs), 1e-8)
    op.poly_setup(32, "cheb")
    x32, s32 = op.apply(bd, kind="invsqrt", m_max=200, tol=1e-10)
    assert_close(host(x32), host(xi), 1e-8)


@pytest.fixture(scope="module")
def convdiff128():
    N = 128
    coeffs = wl.convdiff_stencil(N, 50.0)
    with open(os.path.join(GOLDEN, "convdiff128_reference.json")) as f:
        ref = json.load(f)
    assert ref["N"] == N and ref["Pe"] == 50.0 and ref["rhs_seed"] == 0
    op = fa().Stencil7((N, N, N), coeffs)
    return op, dev(wl.rhs(N ** 3, seed=0)), ref


def against_sampled_reference(x, ref, kind):
    """Relative errors of x against a sampled oracle reference: the largest
    sampled entry error over the largest sampled entry, the root-mean-square
    sampled error scaled to the 2-norm (an estimate of ||x - x*|| / ||x*||),
    and the difference of the 2-norms."""
    idx = torch.as_tensor(ref["indices"], device=x.device)
    xs = x[idx].cpu().numpy()
    ref = ref[kind]
    rv = np.array(ref["values"])
    d = xs - rv
    n = x.numel()
    e_inf = float(np.max(np.abs(d)) / np.max(np.abs(rv)))
    e_rms = float(math.sqrt(n / len(rv) * float(d @ d)) / ref["norm2"])
    e_norm = abs(float(torch.linalg.vector_norm(x).item()) - ref["norm2"]) / ref["norm2"]
    return e_inf, e_rms, e_norm


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
@pytest.mark.parametrize("degree", [0, 4, 16, 32])
def test_convdiff_128_every_degree_against_oracle_reference(convdiff128, degree, kind):
    """The 128^3 configuration at its own settings (Chebyshev degrees 0, 4,
    16, 32; A^{-1/2} b and A^{1/2} b; tol 1e-8): each result within 1e-8 of the
    oracle's tol-1e-12 solve (stored at 2048 sampled entries with its 2-norm
    by tests/golden/make_convdiff128_reference.py; Sec. 6 measures errors
    against a reference solution)."""
    op, bd, ref = convdiff128
    op.poly_setup(degree, "cheb")
    m_max = 600 if degree == 0 else 200
    x, st = op.apply(bd, kind=kind, m_max=m_max, tol=1e-8)
    assert st["converged"] == 1
    e_inf, e_rms, e_norm = against_sampled_reference(x, ref, kind)
    assert e_inf <= 1e-8 and e_rms <= 1e-8 and e_norm <= 1e-8, (e_inf, e_rms, e_norm)


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_convdiff_128_tight_solve_against_oracle_reference(convdiff128, kind):
    """Both sides at tol 1e-12 with the same degree (32): agreement to 1e-10."""
    op, bd, ref = convdiff128
    op.poly_setup(ref["degree"], "cheb")
    x, st = op.apply(bd, kind=kind, m_max=60, tol=ref["tol"])
    # checks every step (k = 64 / 33 = 1): an estimate within rounding of
    # 1e-12 may stop one side a step apart
    assert st["converged"] == 1 and abs(st["iters"] - ref[kind]["iters"]) <= 1
    e_inf, e_rms, e_norm = against_sampled_reference(x, ref, kind)
    assert e_inf <= 1e-10 and e_rms <= 1e-10 and e_norm <= 1e-10, (e_inf, e_rms, e_norm)


# --------------------------------------------------------------------------
# the 16^4 Wilson-like workload at full size
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def wilson16():
    """The 16^4 lattice of the configuration: links exp(0.3 i H), m0 = 0.05."""
    L = 16
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    return U, m0, fa().Wilson(U, m0)


def test_wilson_16_ritz_setup_and_chain_against_oracle(wilson16):
    """Full 16^4 size, Ritz degree 16 (Sec. 5.2): the GPU's setup (17 Arnoldi
    steps, Leja order, scaled Newton coefficients) against the oracle's, and
    q(A) x against the oracle's Horner recurrence on the exported nodes."""
    U, m0, op = wilson16
    start = wl.rhs(op.n, seed=11, complex_=True)
    op.poly_setup(16, "ritz", start=dev(start))
    apply_A = lambda v: ops.wilson_apply(U, m0, v)  # noqa: E731
    q = pl.ritz(apply_A, start, 16, real_operator=False)
    p = op.poly()
    key = lambda z: (round(z.real, 6), round(z.imag, 6))  # noqa: E731
    gt = np.array(sorted(p["theta"], key=key))
    rt = np.array(sorted(q.theta, key=key))
    assert p["degree"] == q.degree == 16
    assert np.max(np.abs(gt - rt)) <= 1e-9 * np.max(np.abs(rt))
    x = wl.rhs(op.n, seed=12, complex_=True)
    y = host(op.poly_apply(dev(x)))
    ref, nmv = exported_newton_poly(op, False).apply(apply_A, x)
    assert nmv == 16
    assert_close(y, ref, 1e-12)


def test_wilson_16_fixed_m_solve_against_oracle(wilson16):
    """Full 16^4 size, Ritz degree 16, Algorithm 1 at a fixed Krylov
    dimension m = 2 (c = q(A) b, then two steps of q(A) q(A) A: 82 products
    with A on the host) against the oracle with the exported polynomial."""
    U, m0, op = wilson16
    op.poly_setup(16, "ritz", start=dev(wl.rhs(op.n, seed=11, complex_=True)))
    b = wl.rhs(op.n, seed=0, complex_=True)
    x, st = op.apply(dev(b), kind="invsqrt", m_max=2, tol=0.0)
    apply_A = lambda v: ops.wilson_apply(U, m0, v)  # noqa: E731
    ref = kr.fAb(apply_A, b, exported_newton_poly(op, False), "invsqrt", m_max=2, tol=0.0)
    assert st["iters"] == ref.iters == 2 and st["mvms"] == ref.mvms == 16 + 2 * 33
    assert_close(host(x), ref.x, 1e-10)


# --------------------------------------------------------------------------
# Sec. 6, Example 2: (Q^2)^{-1/2} b with Q = Gamma_5 D(m_w, mu)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mu", [0.0, 0.3])
@pytest.mark.parametrize("Ls", [(4, 4, 4, 4), (4, 3, 5, 4), (8, 2, 8, 8), (8, 3, 8, 8)])
def test_overlap_q2_operator_against_oracle(mu, Ls):
    """D with a chemical potential and Q^2 = (Gamma_5 D)^2 at m_w = -1.4, one
    application each, against the oracle (a lattice whose 240 sites leave the
    last 64-site workgroup partly empty, and two in the t-walk workgroup
    order, with z-blocks of two planes and of one, too)."""
    U = wl.su3_links(Ls, eps=0.5, seed=3)
    m0 = -1.4
    opD = fa().Wilson(U, m0, mu=mu)
    opQ = fa().Wilson(U, m0, mu=mu, squared=True)
    x = wl.rhs(opD.n, seed=5, complex_=True)
    assert_close(host(opD.op_apply(dev(x))), ops.wilson_apply(U, m0, x, mu), 1e-13)
    assert_close(host(opQ.op_apply(dev(x))), ops.wilson_q2_apply(U, m0, x, mu), 1e-13)
    # a squared op takes its scratch vector from the workspace even when the
    # caller asks for none
    assert_close(host(opQ.op_apply(dev(x), split_long_rows=False)),
                 ops.wilson_q2_apply(U, m0, x, mu), 1e-13)


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_overlap_q2_solve_against_oracle(kind):
    """(Q^2)^{-1/2} b and (Q^2)^{1/2} b at m_w = -1.4, mu = 0.3 (non-Hermitian
    Q^2), Ritz degree 7: a fixed m = 3 and a converged solve at tol 1e-12 on
    both sides against the oracle with the exported polynomial."""
    Ls = (4, 4, 4, 4)
    U = wl.su3_links(Ls, eps=0.5, seed=3)
    m0, mu = -1.4, 0.3
    op = fa().Wilson(U, m0, mu=mu, squared=True)
    op.poly_setup(7, "ritz", start=dev(wl.rhs(op.n, seed=11, complex_=True)))
    b = wl.rhs(op.n, seed=0, complex_=True)
    A = lambda v: ops.wilson_q2_apply(U, m0, v, mu)  # noqa: E731
    q = exported_newton_poly(op, False)
    x, st = op.apply(dev(b), kind=kind, m_max=3, tol=0.0)
    ref = kr.fAb(A, b, q, kind, m_max=3, tol=0.0)
    assert st["iters"] == ref.iters == 3 and st["mvms"] == ref.mvms
    assert_close(host(x), ref.x, 1e-10)
    x, st = op.apply(dev(b), kind=kind, m_max=200, tol=1e-12)
    ref = kr.fAb(A, b, q, kind, m_max=200, tol=1e-12)
    assert st["converged"] and st["iters"] == ref.iters
    assert_close(host(x), ref.x, 1e-10)


def test_overlap_q2_free_field_closed_form_and_hermitian_lanczos():
    """Unit links: (Q^2)^{-1/2} b against the momentum-space closed form
    (mu = 0.3, Arnoldi); at mu = 0 Q^2 is Hermitian and Lanczos gives the
    same closed form."""
    Ls = (4, 4, 4, 6)
    U = np.zeros((4, *Ls, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    m0 = -1.4
    b = wl.rhs(int(np.prod(Ls)) * 12, seed=2, complex_=True)
    for mu, herm in ((0.3, False), (0.0, True)):
        op = fa().Wilson(U, m0, mu=mu, squared=True, hermitian=herm)
        op.poly_setup(6, "ritz", start=dev(wl.rhs(op.n, seed=11, complex_=True)))
        x, st = op.apply(dev(b), m_max=300, tol=1e-12)
        assert st["converged"]
        if herm:  # three-term recurrence: two inner products per step
            assert st["inner_products"] == 2 * st["iters"]
        assert_close(host(x), exact.wilson_free_q2_fAb(Ls, m0, b, mu), 1e-10)


def test_overlap_sign_function_squares_to_one():
    """sign(Q) b = Q (Q^2)^{-1/2} b on an 8^4 lattice (m_w = -1.4, mu = 0.3):
    sign(Q)^2 b = b, a property that holds at any size."""
    L = 8
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0, mu = -1.4, 0.3
    opD = fa().Wilson(U, m0, mu=mu)
    opQ = fa().Wilson(U, m0, mu=mu, squared=True)
    opQ.poly_setup(16, "ritz", start=dev(wl.rhs(opQ.n, seed=11, complex_=True)))

    def sign_q(v):
        y, st = opQ.apply(v, m_max=200, tol=1e-12)
        assert st["converged"]
        d = opD.op_apply(y).reshape(-1, 4, 3)
        d[:, 2:, :] *= -1.0  # Gamma_5
        return d.reshape(-1)

    b = dev(wl.rhs(opQ.n, seed=0, complex_=True))
    z = sign_q(sign_q(b))
    assert_close(host(z), host(b), 1e-9)


def test_wilson_16_full_size():
    """16^4 lattice, links exp(0.3 i H), m0 = 0.05, Ritz degree 16, tol 1e-8.

    Converged solves on the full lattice (the oracle pins the setup, the
    chain and a fixed-m solve at this size above): properties that hold at
    any size, agreement with another degree and A^{1/2} (A^{-1/2} b) = b."""
    L = 16
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    op = fa().Wilson(U, m0)
    assert op.n == 786432
    start = dev(wl.rhs(op.n, seed=11, complex_=True))
    b = dev(wl.rhs(op.n, seed=0, complex_=True))
    # one operator application against the oracle on the full lattice
    xv = wl.rhs(op.n, seed=4, complex_=True)
    assert_close(host(op.op_apply(dev(xv))), ops.wilson_apply(U, m0, xv), 1e-14)
    op.poly_setup(16, "ritz", start=start)
    p = op.poly()
    assert min(z.real for z in p["theta"]) > 0
    x16, s16 = op.apply(b, kind="invsqrt", m_max=200, tol=1e-10)
    assert s16["converged"]
    op.poly_setup(8, "ritz", start=start)
    x8, s8 = op.apply(b, kind="invsqrt", m_max=300, tol=1e-10)
    assert s8["converged"] and s8["iters"] > s16["iters"]
    assert_close(host(x16), host(x8), 1e-8)
    op.poly_setup(16, "ritz", start=start)
    y, sy = op.apply(x16, kind="sqrt", m_max=200, tol=1e-10)
    assert_close(host(y), host(b), 1e-8)


def test_powerlaw_csr_apply_full_size():
    """SpMV with a directed power-law graph Laplacian of the shape of
    Example 3 (n = 281,903, ~2.58M stored entries, rows up to ~34k entries)."""
    rp, ci, va = wl.powerlaw_digraph_laplacian_csr(281903, 2594228, seed=5)
    op = fa().CSR(rp, ci, va)
    xv = wl.rhs(op.n, seed=3)
    assert_close(host(op.op_apply(dev(xv))), ops.csr_apply(rp, ci, va, xv), 1e-14)


def test_powerlaw_digraph_sqrt_against_oracle():
    """Sec. 6, Example 3 in shape: L^{1/2} b as L^{-1/2} (L b) for the singular
    in-degree Laplacian of a directed power-law graph (n = 20,000 here),
    b a canonical unit vector, Ritz polynomial of degree 8 from a random start,
    re-orthogonalized Arnoldi, checks every 32 / d = 3 steps.  The oracle runs
    with the GPU's exported polynomial; both at tol 1e-12 (same iterations,
    agreement 1e-10), and at the example's tol 1e-7 the same iterations."""
    n = 20000
    rp, ci, va = wl.powerlaw_digraph_laplacian_csr(n, 184000, seed=5)
    op = fa().CSR(rp, ci, va)
    start = wl.rhs(n, seed=8)
    op.poly_setup(8, "ritz", start=dev(start))
    q = exported_newton_poly(op, True)
    assert np.all(q.theta.real > 0)
    b = np.zeros(n)
    b[int(np.random.default_rng(0).integers(n))] = 1.0
    A = lambda v: ops.csr_apply(rp, ci, va, v)  # noqa: E731
    for tol, bar in ((1e-12, 1e-10), (1e-7, 1e-10)):
        x, st = op.apply(dev(b), kind="sqrt", m_max=300, tol=tol, check_every=3)
        orc = kr.fAb(A, b, q, "sqrt", m_max=300, tol=tol, check_every=3)
        assert st["converged"] == 1 and st["iters"] == orc.iters and st["mvms"] == orc.mvms
        assert_close(host(x), orc.x, bar)


@pytest.mark.parametrize("degree", [0, 4, 8])
def test_singular_digraph_laplacian_sqrt(degree):
    """Sec. 4 (implicit desingularization): L^{1/2} b as L^{-1/2}(L b) for the
    singular in-degree Laplacian of a random digraph; reference from the
    eigendecomposition with sqrt(0) = 0, and the oracle."""
    n = 300
    rp, ci, va = wl.digraph_laplacian_csr(n, p=0.03, seed=3)
    Ld = np.zeros((n, n))
    for i in range(n):
        Ld[i, ci[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
    lam, X = np.linalg.eig(Ld)
    b = wl.rhs(n, seed=6)
    ref = (X @ (np.sqrt(np.where(np.abs(lam) < 1e-10, 0, lam)) * np.linalg.solve(X, b))).real
    op = fa().CSR(rp, ci, va)
    start = wl.rhs(n, seed=8)
    op.poly_setup(degree, "ritz", start=dev(start))
    x, st = op.apply(dev(b), kind="sqrt", m_max=n, tol=1e-10, check_every=2)
    assert st["converged"] and not st["breakdown"]
    assert_close(host(x), ref, 1e-9)
    A = lambda v: ops.csr_apply(rp, ci, va, v)
    q = pl.ritz(A, start, degree, real_operator=True)
    orc = kr.fAb(A, b, q, "sqrt", m_max=n, tol=1e-10, check_every=2)
    assert_close(host(x), orc.x, 1e-9)


@pytest.mark.parametrize("degree", [4, 8])
def test_real_operator_complex_ritz_values(degree):
    """Ritz polynomial of a strongly non-normal real operator whose Ritz values
    include conjugate pairs: evaluated in real arithmetic (real linear and
    quadratic factors) on the GPU, in complex arithmetic by the oracle."""
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 400.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    start = wl.rhs(N ** 3, seed=4)
    q = pl.ritz(A, start, degree, real_operator=True)
    assert np.max(np.abs(q.theta.imag)) > 0.1       # really complex nodes
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "ritz", start=dev(start))
    p = op.poly()
    key = lambda z: (round(z.real, 6), round(z.imag, 6))
    gt = np.array(sorted(p["theta"], key=key))
    rt = np.array(sorted(q.theta, key=key))
    assert np.max(np.abs(gt - rt)) <= 1e-8 * np.max(np.abs(rt))
    x = wl.rhs(N ** 3, seed=5)
    ref, _ = q.apply(A, x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-7)
    b = wl.rhs(N ** 3, seed=0)
    xs, st = op.apply(dev(b), m_max=400, tol=1e-12)
    orc = kr.fAb(A, b, q, "invsqrt", m_max=400, tol=1e-12)
    assert st["converged"]
    assert_close(host(xs), orc.x, 1e-10)


# --------------------------------------------------------------------------
# mixed precision: the polynomial chain in FP32, the rest FP64
# --------------------------------------------------------------------------
@pytest.mark.parametrize("degree", [1, 2, 3, 8, 16])
@pytest.mark.parametrize("fuse", [True, 3, False])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_mixed_precision_against_fp64_oracle(degree, fuse, kind):
    """Per-result error of the mixed mode against the FP64 oracle: <= 1e-6."""
    dims = (40, 33, 29)
    coeffs = wl.convdiff_stencil(40, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    b = wl.rhs(op.n, seed=0)
    x, st = op.apply(dev(b), kind=kind, m_max=300, tol=1e-7, mixed=True, fuse=fuse)
    assert st["converged"]
    a, bb = ops.stencil_interval(coeffs, dims)
    orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, pl.chebyshev(a, bb, degree),
                 kind, m_max=300, tol=1e-12)
    assert_close(host(x), orc.x, 1e-6)


def test_mixed_precision_unsupported_and_degree0():
    rp, ci, va = wl.stencil_csr((8, 8, 8), wl.laplace_stencil(3))
    op = fa().CSR(rp, ci, va)
    op.set_spectral_interval(*ops.stencil_interval(wl.laplace_stencil(3), (8, 8, 8)))
    op.poly_setup(4, "cheb")
    with pytest.raises(fa().FAError) as e:
        op.apply(dev(wl.rhs(512, seed=0)), m_max=50, tol=1e-8, mixed=True)
    assert e.value.status == -9
    st7 = fa().Stencil7((8, 8, 8), wl.laplace_stencil(3))
    st7.poly_setup(0)
    b = dev(wl.rhs(512, seed=0))
    x1, _ = st7.apply(b, m_max=100, tol=1e-10, mixed=True)
    x2, _ = st7.apply(b, m_max=100, tol=1e-10)
    assert torch.equal(x1, x2)


def test_mixed_precision_128_full_size():
    N = 128
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(16, "cheb")
    b = dev(wl.rhs(op.n, seed=0))
    x64, _ = op.apply(b, m_max=200, tol=1e-10)
    x32, st = op.apply(b, m_max=200, tol=1e-7, mixed=True)
    assert st["converged"]
    assert_close(host(x32), host(x64), 1e-6)


# --------------------------------------------------------------------------
# variants of Sec. 5.2 and Sec. 6: harmonic Ritz values, right
# preconditioning (Algorithm 2), two-pass Lanczos
# --------------------------------------------------------------------------
def _sorted_nodes(t):
    key = lambda z: (round(z.real, 6), round(z.imag, 6))
    return np.array(sorted(t, key=key))


def test_harmonic_ritz_wilson():
    L = 4
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    op = fa().Wilson(U, m0)
    start = wl.rhs(op.n, seed=11, complex_=True)
    op.poly_setup(8, "harmonic", start=dev(start))
    p = op.poly()
    assert p["method"] == "harmonic" and p["degree"] == 8
    apply_A = lambda v: ops.wilson_apply(U, m0, v)
    q = pl.ritz(apply_A, start, 8, real_operator=False, harmonic=True)
    gt, rt = _sorted_nodes(p["theta"]), _sorted_nodes(q.theta)
    assert np.max(np.abs(gt - rt)) <= 1e-9 * np.max(np.abs(rt))
    # not the plain Ritz values
    q0 = pl.ritz(apply_A, start, 8, real_operator=False)
    assert np.max(np.abs(rt - _sorted_nodes(q0.theta))) > 1e-3
    x = wl.rhs(op.n, seed=12, complex_=True)
    ref, _ = q.apply(apply_A, x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-8)
    b = wl.rhs(op.n, seed=0, complex_=True)
    xs, st = op.apply(dev(b), m_max=400, tol=1e-12)
    orc = kr.fAb(apply_A, b, q, "invsqrt", m_max=400, tol=1e-12)
    assert st["converged"] and st["iters"] == orc.iters
    assert_close(host(xs), orc.x, 1e-10)


@pytest.mark.parametrize("degree", [4, 8])
def test_harmonic_ritz_real_nonnormal(degree):
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 100.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    start = wl.rhs(N ** 3, seed=4)
    q = pl.ritz(A, start, degree, real_operator=True, harmonic=True)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "harmonic", start=dev(start))
    p = op.poly()
    gt, rt = _sorted_nodes(p["theta"]), _sorted_nodes(q.theta)
    assert np.max(np.abs(gt - rt)) <= 1e-8 * np.max(np.abs(rt))
    b = wl.rhs(N ** 3, seed=0)
    xs, st = op.apply(dev(b), m_max=400, tol=1e-12)
    orc = kr.fAb(A, b, q, "invsqrt", m_max=400, tol=1e-12)
    assert st["converged"]
    assert_close(host(xs), orc.x, 1e-10)


@pytest.mark.parametrize("degree,m", [(0, 30), (3, 12), (8, 6)])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_right_preconditioning_fixed_m(degree, m, kind):
    """Algorithm 2 with Arnoldi (CGS2) on a non-normal operator, fixed m."""
    dims = (20, 18, 16)
    coeffs = wl.convdiff_stencil(20, 50.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(degree, "cheb")
    a, bb = ops.stencil_interval(coeffs, dims)
    b = wl.rhs(op.n, seed=0)
    x, st = op.apply(dev(b), kind=kind, m_max=m, tol=0.0, right=True)
    ref = kr.fAb(A, b, pl.chebyshev(a, bb, degree), kind, m_max=m, tol=0.0, side="right")
    assert st["iters"] == ref.iters == m
    assert st["mvms"] == ref.mvms
    assert_close(host(x), ref.x, 1e-10)


@pytest.mark.parametrize("degree", [4, 15])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_right_preconditioning_lanczos_converged(degree, kind):
    """Algorithm 2 with Lanczos: the stopping estimate over the stored y_j and
    the iteration count agree with the oracle; the result with the closed form."""
    N = 24
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    op = fa().Stencil7(dims, coeffs, hermitian=True)
    op.poly_setup(degree, "cheb")
    a, bb = ops.stencil_interval(coeffs, dims)
    b = wl.rhs(op.n, seed=0)
    x, st = op.apply(dev(b), kind=kind, m_max=300, tol=1e-11, right=True)
    orc = kr.fAb(A, b, pl.chebyshev(a, bb, degree), kind, m_max=300, tol=1e-11,
                 orth="lanczos", side="right")
    assert st["converged"] and st["iters"] == orc.iters
    assert st["mvms"] == orc.mvms and st["inner_products"] == orc.inner_products
    # the estimate is a ratio of small differences: equal up to rounding noise
    assert abs(st["est_rel_change"] - orc.est) <= 0.1 * orc.est + 1e-13
    assert_close(host(x), orc.x, 1e-10)
    assert_close(host(x), exact.stencil_fAb_dst(coeffs, dims, b, kind), 1e-9)


@pytest.mark.parametrize("d", [8, 16])
def test_table1_right_lanczos_100cubed(d):
    """Sec. 6, Example 1, Table 1 at its size (100^3 Laplacian, Chebyshev q
    with d coefficients, right-preconditioned Lanczos): at the printed
    iteration count the true relative error is below 1e-12 and one check
    interval earlier it is not; the operation counts follow the printed rule."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "table1_laplace3d.json")))
    row = next(r for r in g["rows"] if r["d"] == d)
    N = g["N"]
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    op = fa().Stencil7(dims, coeffs, hermitian=True)
    op.poly_setup(d - 1, "cheb")
    b = wl.rhs(N ** 3, seed=0)
    b = b / np.linalg.norm(b)
    xs = exact.stencil_fAb_dst(coeffs, dims, b, "invsqrt")
    k = 64 // d
    m = row["iterations"]
    errs = {}
    for mm in (m - k, m):
        x, st = op.apply(dev(b), m_max=mm, tol=0.0, right=True)
        errs[mm] = np.linalg.norm(host(x) - xs) / np.linalg.norm(xs)
        assert st["mvms"] == mm * (2 * d - 1)
        assert st["inner_products"] == 2 * mm
    assert errs[m] < g["tol_true_error"] < errs[m - k], errs
    assert st["mvms"] == row["mvms"] and st["inner_products"] == row["inner_products"]


@pytest.mark.parametrize("degree", [0, 4])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_two_pass_lanczos(degree, kind):
    """Two-pass Lanczos: the same iterate as one pass (same iteration count),
    the basis regenerated instead of stored, and the oracle's counts."""
    N = 20
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    op = fa().Stencil7(dims, coeffs, hermitian=True)
    op.poly_setup(degree, "cheb")
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    b = wl.rhs(op.n, seed=0)
    x1, s1 = op.apply(dev(b), kind=kind, m_max=300, tol=1e-10)
    x2, s2 = op.apply(dev(b), kind=kind, m_max=300, tol=1e-10, two_pass=True)
    assert s2["converged"] and s2["iters"] == s1["iters"]
    assert_close(host(x2), host(x1), 1e-13)
    orc = kr.fAb(A, b, q, kind, m_max=300, tol=1e-10, orth="lanczos", two_pass=True)
    assert s2["iters"] == orc.iters and s2["mvms"] == orc.mvms
    assert_close(host(x2), orc.x, 1e-10)
    # three basis vectors instead of m_max + 1 (plus the fixed scratch vectors)
    tp = fa().FA_TWO_PASS
    assert op.workspace_bytes(300, tp) < op.workspace_bytes(300) / 10
    # ... and a few scalars per step (H's two diagonals, coefficients)
    assert op.workspace_bytes(3000, tp) - op.workspace_bytes(300, tp) < 64 * (3000 - 300)


@pytest.mark.parametrize("degree", [0, 4])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_two_pass_right_fixed_m(degree, kind):
    """Two-pass with Algorithm 2 (Table 1's 2P column) at a fixed m: the
    oracle's right two-pass iterate, the GPU's one-pass right iterate, and the
    count of two passes plus the final q(A)."""
    N = 20
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    op = fa().Stencil7(dims, coeffs, hermitian=True)
    op.poly_setup(degree, "cheb")
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    b = wl.rhs(op.n, seed=0)
    m = 24
    x1, s1 = op.apply(dev(b), kind=kind, m_max=m, tol=0.0, right=True)
    x2, s2 = op.apply(dev(b), kind=kind, m_max=m, tol=0.0, right=True, two_pass=True)
    assert s1["iters"] == s2["iters"] == m
    assert_close(host(x2), host(x1), 1e-12)
    orc = kr.fAb(A, b, q, kind, m_max=m, tol=0.0, orth="lanczos", side="right", two_pass=True)
    assert s2["mvms"] == orc.mvms
    assert_close(host(x2), orc.x, 1e-10)
    tp = fa().FA_TWO_PASS | fa()._lib.FA_RIGHT_PREC
    assert op.workspace_bytes(300, tp) < op.workspace_bytes(300, fa()._lib.FA_RIGHT_PREC) / 10


def test_variant_flag_errors():
    dims = (8, 8, 8)
    coeffs = wl.convdiff_stencil(8, 10.0)
    op = fa().Stencil7(dims, coeffs)          # not Hermitian
    op.poly_setup(4, "cheb")
    b = dev(wl.rhs(op.n, seed=0))
    with pytest.raises(fa().FAError) as e:
        op.apply(b, two_pass=True)
    assert e.value.status == fa()._lib.FA_ERR_UNSUPPORTED
    with pytest.raises(fa().FAError):
        op.apply(b, right=True, mixed=True)
    oph = fa().Stencil7(dims, wl.laplace_stencil(3), hermitian=True)
    oph.poly_setup(4, "cheb")
    with pytest.raises(fa().FAError) as e:  # right two-pass: a fixed m only
        oph.apply(b, two_pass=True, right=True, tol=1e-8)
    assert e.value.status == fa()._lib.FA_ERR_UNSUPPORTED
    with pytest.raises(fa().FAError):
        oph.apply(b, two_pass=True, force_arnoldi=True)


# --------------------------------------------------------------------------
# Sec. 5.3: least-squares polynomials on a contour around the Ritz values
# --------------------------------------------------------------------------
def _ls_compare(op, q, p, tol_coef):
    assert p["method"] == "ls" and p["degree"] == q.degree and p["npts"] == q.npts
    assert np.max(np.abs(np.array(p["alpha"]) - q.alpha)) <= tol_coef * np.max(np.abs(q.alpha))
    assert np.max(np.abs(np.array(p["h"]) - q.hls)) <= tol_coef * np.max(np.abs(q.hls))


def test_ls_polynomial_real_nonnormal():
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    start = wl.rhs(N ** 3, seed=4)
    q = pl.least_squares(A, start, 6, real_operator=True, ritz_steps=30, step=0.01)
    op = fa().Stencil7(dims, coeffs)
    op.poly_setup(6, "ls", start=dev(start), ritz_steps=30, step=0.01)
    _ls_compare(op, q, op.poly(), 1e-9)
    x = wl.rhs(N ** 3, seed=5)
    ref, _ = q.apply(A, x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-9)
    b = wl.rhs(N ** 3, seed=0)
    for kind in ("invsqrt", "sqrt"):
        xs, st = op.apply(dev(b), kind=kind, m_max=300, tol=1e-12)
        orc = kr.fAb(A, b, q, kind, m_max=300, tol=1e-12)
        assert st["converged"] and st["iters"] == orc.iters and st["mvms"] == orc.mvms
        assert_close(host(xs), orc.x, 1e-10)
        assert_close(host(xs), exact.stencil_fAb_dst(coeffs, dims, b, kind), 1e-9)
    # right preconditioning and a fixed Krylov dimension with the same q
    xr, sr = op.apply(dev(b), m_max=8, tol=0.0, right=True)
    orr = kr.fAb(A, b, q, "invsqrt", m_max=8, tol=0.0, side="right")
    assert_close(host(xr), orr.x, 1e-10)


def test_ls_polynomial_wilson_complex():
    L = 4
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    apply_A = lambda v: ops.wilson_apply(U, m0, v)
    op = fa().Wilson(U, m0)
    start = wl.rhs(op.n, seed=11, complex_=True)
    q = pl.least_squares(apply_A, start, 5, real_operator=False, ritz_steps=24, step=0.01)
    op.poly_setup(5, "ls", start=dev(start), ritz_steps=24, step=0.01)
    _ls_compare(op, q, op.poly(), 1e-8)
    x = wl.rhs(op.n, seed=12, complex_=True)
    ref, _ = q.apply(apply_A, x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-8)
    b = wl.rhs(op.n, seed=0, complex_=True)
    xs, st = op.apply(dev(b), m_max=400, tol=1e-12)
    orc = kr.fAb(apply_A, b, q, "invsqrt", m_max=400, tol=1e-12)
    assert st["converged"] and st["iters"] == orc.iters
    assert_close(host(xs), orc.x, 1e-10)


def test_ls_polynomial_errors():
    N = 8
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 10.0)
    op = fa().Stencil7(dims, coeffs)
    start = dev(wl.rhs(N ** 3, seed=4))
    with pytest.raises(fa().FAError):
        op.poly_setup(64, "ls", start=start, ritz_steps=30, step=0.01)
    op.poly_setup(4, "ls", start=start, ritz_steps=30, step=0.01)
    b = dev(wl.rhs(N ** 3, seed=0))
    with pytest.raises(fa().FAError) as e:
        op.apply(b, mixed=True)
    assert e.value.status == fa()._lib.FA_ERR_UNSUPPORTED
    x, st = op.apply(b, m_max=100, tol=1e-10)
    assert st["converged"]


@pytest.mark.parametrize("complex_", [False, True])
def test_csr_long_rows(complex_):
    """Rows far longer than the mean (a power-law tail) are summed by their own
    one-workgroup-per-row kernel: A x and a Ritz q(A) x (whose Newton terms
    combine A r with v) against the oracle."""
    rng = np.random.default_rng(7)
    n = 3000
    rows, cols = [], []
    for i in range(n):
        k = 3000 if i % 97 == 0 else (1200 if i % 151 == 0 else 4)
        c = rng.choice(n, size=min(k, n), replace=False)
        rows += [i] * len(c)
        cols += list(c)
    rows, cols = np.array(rows), np.array(cols)
    vals = rng.standard_normal(len(rows)) * 0.01
    if complex_:
        vals = vals + 0.01j * rng.standard_normal(len(rows))
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
    op = fa().CSR(rp, ci, va)
    x = wl.rhs(n, seed=3, complex_=complex_)
    assert_close(host(op.op_apply(dev(x))), ops.csr_apply(rp, ci, va, x), 1e-14)
    start = wl.rhs(n, seed=4, complex_=complex_)
    op.poly_setup(6, "ritz", start=dev(start))
    Aop = lambda v: ops.csr_apply(rp, ci, va, v)
    q = pl.ritz(Aop, start, 6, real_operator=not complex_)
    ref, _ = q.apply(Aop, x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-9)


@pytest.mark.parametrize("complex_", [False, True])
def test_csr_very_long_rows_repeats_and_streams(complex_):
    """Rows of 9,000 and 20,000 entries among rows of 3 (each long row cut into
    chunks of 4,096 entries on separate workgroups, the last one adding the
    partial sums in order): A x against the oracle, and the same bits on every
    repeat, on two streams at once (each with its own scratch), and with one
    workgroup per long row (no scratch)."""
    rng = np.random.default_rng(11)
    n = 30000
    rows, cols = [], []
    for i in range(n):
        k = 20000 if i % 1999 == 0 else (9000 if i % 2503 == 0 else 3)
        c = rng.choice(n, size=k, replace=False)
        rows += [i] * len(c)
        cols += list(c)
    rows, cols = np.array(rows), np.array(cols)
    vals = rng.standard_normal(len(rows)) * 0.01
    if complex_:
        vals = vals + 0.01j * rng.standard_normal(len(rows))
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A = A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() + 1.0)
    A = A.tocsr()
    A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
    op = fa().CSR(rp, ci, va)
    x = dev(wl.rhs(n, seed=3, complex_=complex_))
    ref = ops.csr_apply(rp, ci, va, host(x))
    y0 = op.op_apply(x).clone()
    assert_close(host(y0), ref, 1e-14)
    for _ in range(3):
        assert torch.equal(op.op_apply(x), y0)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for _ in range(4):
        for st in (s1, s2):
            with torch.cuda.stream(st):
                outs.append(op.op_apply(x))
    torch.cuda.synchronize()
    for y in outs:
        assert torch.equal(y, y0)
    assert torch.equal(op.op_apply(x, split_long_rows=False), y0)


@pytest.mark.parametrize("complex_", [False, True])
def test_csr_rows_at_the_block_and_chunk_bounds(complex_):
    """Rows of 0, 1, 4095, 4096, 4097, 8192, 8193 and 12,289 entries, runs of
    512 short rows, and the Clenshaw-type epilogue with both extra vectors:
    blocks end at 4,096 entries or 512 rows, longer rows are cut into chunks
    (one entry past a multiple of 4,096 makes a chunk of one); split and
    unsplit long rows give the same bits, and both match the oracle."""
    rng = np.random.default_rng(13)
    lens = [0, 1, 4095, 3, 4096, 0, 4097, 2] + [1] * 600 + [8192, 8193, 12289, 5, 0, 7]
    n = len(lens) + 20000
    lens = lens + list(rng.integers(0, 12, 20000))
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([rng.choice(n, size=k, replace=False) for k in lens]).astype(np.int32)
    va = rng.standard_normal(rp[-1])
    if complex_:
        va = va + 1j * rng.standard_normal(rp[-1])
    op = fa().CSR(rp, ci, va)
    x = wl.rhs(n, seed=3, complex_=complex_)
    y = op.op_apply(dev(x)).clone()
    assert_close(host(y), ops.csr_apply(rp, ci, va, x), 1e-14)
    assert torch.equal(op.op_apply(dev(x), split_long_rows=False), y)
    # out = alpha A x + beta x + g0 y0 + g1 y1 through a Chebyshev q(A) of
    # degree 3 (its middle terms carry both extra vectors)
    lam = np.abs(va).max() * 2e4
    op.set_spectral_interval(1.0, lam)
    op.poly_setup(3, "cheb")
    q = pl.chebyshev(1.0, lam, 3)
    ref, _ = q.apply(lambda v: ops.csr_apply(rp, ci, va, v), x)
    assert_close(host(op.poly_apply(dev(x))), ref, 1e-12)


def test_csr_rejects_bad_row_pointers():
    rp = np.array([0, 2, 1, 3], dtype=np.int32)
    ci = np.array([0, 1, 2], dtype=np.int32)
    va = np.ones(3)
    with pytest.raises(fa().FAError):
        fa().CSR(rp, ci, va)


# --------------------------------------------------------------------------
# small Hermitian problems: the Lanczos steps between checks in one launch
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(32, 32, 1), (12, 11, 10), (7, 5, 3)])
@pytest.mark.parametrize("degree", [0, 3, 8])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
@pytest.mark.parametrize("check_every", [0, 1, 5])
def test_small_lanczos_against_oracle(shape, degree, kind, check_every):
    """n <= 2048 (one or two entries per thread): the one-workgroup Lanczos
    segments against the oracle's Lanczos (both at tol 1e-12: same
    iterations and products with A, agreement 1e-10), against the DST closed
    form, and against the step-by-step launches (fuse=False); CSR for the
    5-point matrix, the stencil for the 3D grids; checks every k steps."""
    coeffs = wl.laplace_stencil(3 if shape[2] > 1 else 2)
    a, bb = ops.stencil_interval(coeffs, shape)
    if shape[2] == 1:
        rp, ci, va = wl.stencil_csr(shape, coeffs)
        op = fa().CSR(rp, ci, va, hermitian=True)
        op.set_spectral_interval(a, bb)
        A = lambda v: ops.csr_apply(rp, ci, va, v)  # noqa: E731
    else:
        op = fa().Stencil7(shape, coeffs, hermitian=True)
        A = lambda v: ops.stencil_apply(coeffs, shape, v)  # noqa: E731
    op.poly_setup(degree, "cheb")
    b = wl.rhs(op.n, seed=0)
    m_max = min(300, op.n)
    x, st = op.apply(dev(b), kind=kind, m_max=m_max, tol=1e-12, check_every=check_every)
    orc = kr.fAb(A, b, pl.chebyshev(a, bb, degree), kind, m_max=m_max, tol=1e-12,
                 check_every=check_every, orth="lanczos")
    assert st["iters"] == orc.iters and st["mvms"] == orc.mvms
    assert st["inner_products"] == orc.inner_products == 2 * orc.iters
    assert st["converged"] == orc.converged
    assert_close(host(x), orc.x, 1e-10)
    assert_close(host(x), exact.stencil_fAb_dst(coeffs, shape, b, kind), 1e-10)
    x1, s1 = op.apply(dev(b), kind=kind, m_max=m_max, tol=1e-12, check_every=check_every,
                      fuse=False)
    assert s1["iters"] == st["iters"]
    assert_close(host(x), host(x1), 1e-12)


def test_small_lanczos_fixed_m_and_breakdown():
    """Fixed Krylov dimension (tol 0: one launch for all m steps) against the
    oracle, and a lucky breakdown in the middle of a launch's steps (a
    diagonal matrix with 4 distinct values: the host finds h_{5,4} ~ 0 and
    keeps 4 steps; the steps computed past it are not used)."""
    coeffs = wl.laplace_stencil(3)
    shape = (9, 8, 7)
    op = fa().Stencil7(shape, coeffs, hermitian=True)
    op.poly_setup(4, "cheb")
    a, bb = ops.stencil_interval(coeffs, shape)
    b = wl.rhs(op.n, seed=2)
    x, st = op.apply(dev(b), m_max=6, tol=0.0)
    orc = kr.fAb(lambda v: ops.stencil_apply(coeffs, shape, v), b, pl.chebyshev(a, bb, 4),
                 "invsqrt", m_max=6, tol=0.0, orth="lanczos")
    assert st["iters"] == 6 and st["mvms"] == orc.mvms
    assert_close(host(x), orc.x, 1e-10)
    d = np.repeat([0.5, 1.5, 4.0, 9.0], 300)
    n = d.size
    op = fa().CSR(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d,
                  hermitian=True)
    op.poly_setup(0)
    bd = wl.rhs(n, seed=3)
    for kind, f in (("invsqrt", d ** -0.5), ("sqrt", d ** 0.5)):
        x, st = op.apply(dev(bd), kind=kind, m_max=50, tol=1e-12, check_every=10)
        assert st["breakdown"] == 1 and st["iters"] == 4
        assert_close(host(x), f * bd, 1e-12)
