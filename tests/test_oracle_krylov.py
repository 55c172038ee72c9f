"""Pins of the oracle's preconditioned Arnoldi / Lanczos (CPU only).

References that are not the oracle: DST closed forms (Laplace and
convection-diffusion), dense scipy.linalg.sqrtm, diagonal matrices, the
Arnoldi relation, algebraic identities between sqrt and invsqrt, and the
iteration / operation counts printed in the paper's Table 1.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import exact, krylov as kr, operators as ops, polynomials as pl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def stencil_problem(coeffs, dims):
    return lambda x: ops.stencil_apply(coeffs, dims, x)


# --------------------------------------------------------------------------
# dense H^{-1/2} e_1
# --------------------------------------------------------------------------
@pytest.mark.parametrize("complex_", [False, True])
def test_hessenberg_invsqrt_against_eigendecomposition(complex_):
    rng = np.random.default_rng(1)
    m = 30
    H = np.triu(rng.standard_normal((m, m)), -1) * 0.1 + 2.0 * np.eye(m)
    if complex_:
        H = H + 1j * np.triu(rng.standard_normal((m, m)), -1) * 0.1
    lam, X = np.linalg.eig(H)
    assert lam.real.min() > 0
    e1 = np.zeros(m)
    e1[0] = 3.0
    ref = X @ (lam ** -0.5 * np.linalg.solve(X, e1))
    z = kr.hessenberg_invsqrt_e1(H, 3.0)
    assert np.allclose(z, ref if complex_ else ref.real, rtol=1e-11, atol=1e-12)


def test_hessenberg_branch_error():
    H = np.diag([2.0, -1.0, 3.0]) + np.diag([0.5, 0.5], -1)
    with pytest.raises(kr.HessenbergError):
        kr.hessenberg_invsqrt_e1(H, 1.0)


def test_tridiagonal_invsqrt_against_dense():
    rng = np.random.default_rng(2)
    a = 2.0 + rng.random(25)
    b = 0.5 * rng.random(24)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    lam, Q = np.linalg.eigh(T)
    ref = Q @ (lam ** -0.5 * Q[0, :]) * 2.0
    assert np.allclose(kr.tridiagonal_invsqrt_e1(a, b, 2.0), ref, rtol=1e-12)


# --------------------------------------------------------------------------
# whole solves against closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("degree,orth", [(0, "lanczos"), (8, "lanczos"), (0, "cgs2"),
                                         (8, "cgs2"), (4, "mgs")])
def test_poisson2d_32_invsqrt_against_dst(degree, orth):
    """The 2D Poisson 32x32 workload (CSR) against the DST closed form."""
    N = 32
    coeffs = wl.laplace_stencil(2)
    rp, ci, va = wl.stencil_csr((N, N, 1), coeffs)
    op = lambda x: ops.csr_apply(rp, ci, va, x)
    b = wl.rhs(N * N, seed=0)
    a, bb = ops.stencil_interval(coeffs, (N, N, 1))
    q = pl.chebyshev(a, bb, degree)
    res = kr.fAb(op, b, q, "invsqrt", m_max=200, tol=1e-10, orth=orth)
    ref = exact.stencil_fAb_dst(coeffs, (N, N, 1), b, "invsqrt")
    assert res.converged
    assert rel(res.x, ref) < 1e-9
    # mvm count: m (2K + 1) products in the iteration plus K for c = q(A) b
    assert res.mvms == res.iters * (2 * degree + 1) + degree


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
@pytest.mark.parametrize("degree", [0, 4, 16])
def test_convdiff_small_peclet_against_similarity_closed_form(kind, degree):
    """Non-symmetric conv-diff (Pe = 10: cond of the similarity is modest)."""
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 10.0)
    op = stencil_problem(coeffs, dims)
    b = wl.rhs(N ** 3, seed=0)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    res = kr.fAb(op, b, q, kind, m_max=300, tol=1e-12, orth="cgs2")
    ref = exact.stencil_fAb_dst(coeffs, dims, b, kind)
    assert res.converged
    assert rel(res.x, ref) < 1e-10


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_convdiff_pe50_tiny_against_dense_sqrtm(kind):
    """At Pe = 50 the similarity is ill-conditioned: pin with dense sqrtm."""
    N = 6
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    A = ops.stencil_matrix(coeffs, dims).toarray()
    b = wl.rhs(N ** 3, seed=0)
    ref = exact.dense_fAb(A, b, kind)
    a, bb = ops.stencil_interval(coeffs, dims)
    for degree in (0, 4):
        res = kr.fAb(stencil_problem(coeffs, dims), b, pl.chebyshev(a, bb, degree), kind,
                     m_max=216, tol=1e-13)
        assert rel(res.x, ref) < 1e-10


def test_wilson_free_and_pure_gauge_against_fourier():
    L = 3
    Ls = (L, L, L, L)
    m0 = 0.1
    n = L ** 4 * 12
    b = wl.rhs(n, seed=0, complex_=True)
    U1 = np.zeros((4, *Ls, 3, 3), dtype=complex)
    U1[...] = np.eye(3)
    Ug, G = wl.pure_gauge_links(L, seed=4)
    for U, ref in ((U1, exact.wilson_free_fAb(Ls, m0, b)),
                   (Ug, exact.wilson_pure_gauge_fAb(G, m0, b))):
        op = lambda x, U=U: ops.wilson_apply(U, m0, x)
        for degree in (0, 6):
            q = pl.ritz(op, wl.rhs(n, seed=1, complex_=True), degree, real_operator=False)
            res = kr.fAb(op, b, q, "invsqrt", m_max=400, tol=1e-12)
            assert res.converged
            assert rel(res.x, ref) < 1e-10


def test_overlap_q2_free_field_against_fourier():
    # Sec. 6, Example 2: (Q^2)^{-1/2} b and (Q^2)^{1/2} b, Q = Gamma_5 D(m_w, mu)
    # at m_w = -1.4, mu = 0.3 (non-Hermitian Q^2), Ritz polynomials of degree
    # 0 and 7, against the momentum-space closed form for unit links
    Ls = (4, 3, 3, 3)
    m0, mu = -1.4, 0.3
    n = int(np.prod(Ls)) * 12
    b = wl.rhs(n, seed=0, complex_=True)
    U1 = np.zeros((4, *Ls, 3, 3), dtype=complex)
    U1[...] = np.eye(3)
    op = lambda x: ops.wilson_q2_apply(U1, m0, x, mu)  # noqa: E731
    for kind in ("invsqrt", "sqrt"):
        ref = exact.wilson_free_q2_fAb(Ls, m0, b, mu, kind)
        for degree in (0, 7):
            q = pl.ritz(op, wl.rhs(n, seed=1, complex_=True), degree, real_operator=False)
            res = kr.fAb(op, b, q, kind, m_max=400, tol=1e-12)
            assert res.converged
            assert rel(res.x, ref) < 1e-10


def test_wilson_random_links_against_dense():
    L = 2
    U = wl.su3_links(L, eps=0.3, seed=1)
    m0 = 0.05
    n = L ** 4 * 12
    op = lambda x: ops.wilson_apply(U, m0, x)
    D = np.zeros((n, n), dtype=complex)
    for i in range(n):
        e = np.zeros(n, dtype=complex)
        e[i] = 1
        D[:, i] = op(e)
    b = wl.rhs(n, seed=0, complex_=True)
    ref = exact.dense_fAb(D, b)
    q = pl.ritz(op, wl.rhs(n, seed=7, complex_=True), 8, real_operator=False)
    res = kr.fAb(op, b, q, "invsqrt", m_max=n, tol=1e-13)
    assert rel(res.x, ref) < 1e-10


# --------------------------------------------------------------------------
# structure: breakdown, Arnoldi relation, identities, variants
# --------------------------------------------------------------------------
def test_diagonal_matrix_lucky_breakdown():
    a = np.repeat([0.5, 1.5, 4.0, 9.0], 25)           # 4 distinct eigenvalues
    b = wl.rhs(100, seed=3)
    for kind, f in (("invsqrt", a ** -0.5), ("sqrt", a ** 0.5)):
        res = kr.fAb(lambda x: a * x, b, None, kind, m_max=50, tol=1e-12)
        assert res.breakdown and res.iters == 4
        assert rel(res.x, f * b) < 1e-12


def test_arnoldi_relation_and_orthogonality_cgs2():
    N = 10
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = stencil_problem(coeffs, dims)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, 6)
    b = wl.rhs(N ** 3, seed=1)
    res = kr.fAb(op, b, q, "invsqrt", m_max=25, tol=0.0, keep_basis=True)
    V, H = res.V, res.H
    m = res.iters
    AQV = np.column_stack([q.apply(op, q.apply(op, op(V[:, j]))[0])[0] for j in range(m)])
    assert np.linalg.norm(AQV - V @ H) / np.linalg.norm(H) < 1e-13
    assert np.linalg.norm(np.eye(m + 1) - V.T @ V) < 1e-13


def test_sqrt_invsqrt_identities():
    N = 10
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = stencil_problem(coeffs, dims)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, 8)
    b = wl.rhs(N ** 3, seed=2)
    run = lambda v, kind: kr.fAb(op, v, q, kind, m_max=200, tol=1e-13).x
    s = run(b, "sqrt")
    assert rel(run(s, "sqrt"), op(b)) < 1e-10          # (A^{1/2})^2 b = A b
    assert rel(run(s, "invsqrt"), b) < 1e-10           # A^{-1/2} A^{1/2} b = b
    assert rel(s, op(run(b, "invsqrt"))) < 1e-10       # A^{1/2} b = A A^{-1/2} b


def test_variants_agree_at_convergence():
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    op = stencil_problem(coeffs, dims)
    a, bb = ops.stencil_interval(coeffs, dims)
    b = wl.rhs(N ** 3, seed=4)
    base = kr.fAb(op, b, None, "invsqrt", m_max=400, tol=1e-13).x
    # single-pass MGS loses orthogonality once the space is nearly invariant,
    # so it is stopped early by checking every 2 steps
    for degree, side, orth, k in ((4, "left", "cgs2", 0), (4, "left", "mgs", 2),
                                  (16, "left", "cgs2", 0), (8, "right", "cgs2", 0),
                                  (16, "right", "cgs2", 0)):
        x = kr.fAb(op, b, pl.chebyshev(a, bb, degree), "invsqrt", m_max=400, tol=1e-13,
                   side=side, orth=orth, check_every=k).x
        assert rel(x, base) < 1e-10


def test_singular_digraph_laplacian_sqrt():
    """Sec. 4 theorem (implicit desingularization): L^{1/2} b as L^{-1/2}(L b).

    L is the in-degree Laplacian of a random digraph (column sums zero, 0 a
    simple eigenvalue).  The reference is the eigendecomposition with the zero
    eigenvalue's square root set to exactly 0 (dense sqrtm of a singular
    matrix is only accurate to ~sqrt(eps)).  In floating point the component
    of L b along the null vector is ~eps, so the iteration must stop before
    the Krylov space resolves it (else H_m gets a near-zero Ritz value): the
    stopping test is run every 2 steps.
    """
    n = 300
    rp, ci, va = wl.digraph_laplacian_csr(n, p=0.03, seed=3)
    op = lambda x: ops.csr_apply(rp, ci, va, x)
    Ld = np.zeros((n, n))
    for i in range(n):
        Ld[i, ci[rp[i]:rp[i + 1]]] = va[rp[i]:rp[i + 1]]
    assert np.allclose(Ld.sum(axis=0), 0)                # singular: column sums 0
    lam, X = np.linalg.eig(Ld)
    assert np.sum(np.abs(lam) < 1e-10) == 1
    b = wl.rhs(n, seed=6)
    s = np.sqrt(np.where(np.abs(lam) < 1e-10, 0, lam))
    ref = (X @ (s * np.linalg.solve(X, b))).real
    for degree in (0, 4, 8):
        q = pl.ritz(op, wl.rhs(n, seed=8), degree, real_operator=True)
        res = kr.fAb(op, b, q, "sqrt", m_max=n, tol=1e-10, check_every=2)
        assert res.converged and not res.breakdown
        assert rel(res.x, ref) < 1e-9


def test_non_principal_root_when_q_changes_sign():
    """Sec. 5 discussion: q < 0 on part of spec(A) yields B b with B^2 = A^{-1},
    B non-principal; the oracle reproduces exactly that root."""
    N = 8
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = ops.stencil_matrix(coeffs, dims).toarray()
    lam, Q = np.linalg.eigh(A)
    a, bb = lam.min(), lam.max()
    # degree 5 on an interval cutting the top of the spectrum: q < 0 there
    c = pl.chebyshev_coefficients(pl.inv_sqrt, a, 0.7 * bb, 5)
    q = pl.Poly(kind="cheb", degree=5, a=a, b=0.7 * bb, c=c)
    qv = q.scalar(lam)
    assert qv.min() < 0 < qv.max()
    b = wl.rhs(N ** 3, seed=1)
    res = kr.fAb(lambda x: A @ x, b, q, "invsqrt", m_max=N ** 3, tol=1e-13, orth="cgs2")
    B_b = Q @ (np.sign(qv) * lam ** -0.5 * (Q.T @ b))
    assert rel(res.x, B_b) < 1e-9
    assert rel(res.x, Q @ (lam ** -0.5 * (Q.T @ b))) > 1e-3


# --------------------------------------------------------------------------
# Table 1 (Sec. 6, Example 1): iteration and operation counts
# --------------------------------------------------------------------------
def _table1_row(d):
    g = json.load(open(os.path.join(GOLDEN, "table1_laplace3d.json")))
    row = next(r for r in g["rows"] if r["d"] == d)
    N = g["N"]
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    op = stencil_problem(coeffs, dims)
    b = wl.rhs(N ** 3, seed=0)
    b = b / np.linalg.norm(b)
    xs = exact.stencil_fAb_dst(coeffs, dims, b, "invsqrt")
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, d - 1)
    # d = 1 (q == 1): right and left preconditioning are the same iteration
    # (c = b, y_j = v_j); left keeps no second basis (half the memory)
    res = kr.fAb(op, b, q, "invsqrt", m_max=row["iterations"] + 64, tol=g["tol_true_error"],
                 check_every=64 // d, orth="lanczos", side="left" if d == 1 else "right",
                 x_true=xs)
    return row, res


def _table1_counts(d):
    from threadpoolctl import threadpool_limits

    with threadpool_limits(2):  # four rows at once share the cores
        row, res = _table1_row(d)
    return row, (res.iters, res.mvms, res.inner_products)


def test_table1_iterations_and_counts():
    """Table 1 rows d = 1, 4, 8, 16 at 100^3 (a minute or two of NumPy each:
    the four rows run in four processes at once)."""
    import concurrent.futures
    import multiprocessing

    ds = (1, 4, 8, 16)
    with concurrent.futures.ProcessPoolExecutor(
            max_workers=len(ds), mp_context=multiprocessing.get_context("fork")) as ex:
        out = list(ex.map(_table1_counts, ds))
    for d, (row, (iters, mvms, ips)) in zip(ds, out):
        assert iters == row["iterations"], d
        assert mvms == row["mvms"] == iters * (2 * d - 1), d
        assert ips == row["inner_products"] == 2 * iters, d


def test_table1_printed_rows_follow_the_count_rule():
    g = json.load(open(os.path.join(GOLDEN, "table1_laplace3d.json")))
    for r in g["rows"]:
        assert r["mvms"] == r["iterations"] * (2 * r["d"] - 1)
        assert r["inner_products"] == 2 * r["iterations"]


@pytest.mark.parametrize("degree", [0, 4])
def test_two_pass_lanczos_equals_one_pass(degree):
    """Two-pass Lanczos (Sec. 6, Example 1): the same iterate as one pass,
    without storing the basis, at twice the products with A."""
    N = 20
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    b = wl.rhs(N ** 3, seed=0)
    one = kr.fAb(A, b, q, "invsqrt", m_max=300, tol=1e-10, orth="lanczos")
    two = kr.fAb(A, b, q, "invsqrt", m_max=300, tol=1e-10, orth="lanczos", two_pass=True)
    assert two.iters == one.iters and two.converged
    assert rel(two.x, one.x) < 1e-13
    # pass 2 repeats c = q(A) b and m - 1 steps of the three-stage product
    assert two.mvms == 2 * one.mvms - (2 * degree + 1)
    assert rel(two.x, exact.stencil_fAb_dst(coeffs, dims, b)) < 1e-9


@pytest.mark.parametrize("degree", [0, 4])
def test_two_pass_right_equals_one_pass_right(degree):
    """Two-pass with Algorithm 2 at a fixed m: the iterate Y_m z_m of the
    one-pass right variant (which stores the y_j), the DST closed form once
    converged, and the operation count of two passes plus one q(A)."""
    N = 20
    dims = (N, N, N)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, degree)
    b = wl.rhs(N ** 3, seed=0)
    m = 120 if degree == 0 else 30
    one = kr.fAb(A, b, q, "invsqrt", m_max=m, tol=0.0, orth="lanczos", side="right")
    two = kr.fAb(A, b, q, "invsqrt", m_max=m, tol=0.0, orth="lanczos", side="right",
                 two_pass=True)
    assert two.iters == one.iters == m
    assert rel(two.x, one.x) < 1e-12
    assert rel(two.x, exact.stencil_fAb_dst(coeffs, dims, b)) < 1e-9
    # pass 1: m steps; pass 2: m - 1 steps and the final q(A)
    assert two.mvms == (2 * m - 1) * (2 * degree + 1) + degree
    # the right variant's stopping estimate needs the stored y_j
    with pytest.raises(ValueError):
        kr.fAb(A, b, q, "invsqrt", m_max=m, tol=1e-8, orth="lanczos", side="right",
               two_pass=True)


# --------------------------------------------------------------------------
# the stopping estimate against the iterates it stands for
# --------------------------------------------------------------------------
def _fixed_m_iterates(run, checkpoints):
    """f_j for each checkpoint j from separate runs that stop at exactly j
    steps (tol <= 0): the returned x, formed by the method's final combination
    (V_j z_j, Y_j z_j, or the second Lanczos pass), not by the check's
    coefficient-vector arithmetic."""
    return {j: run(j) for j in checkpoints}


@pytest.mark.parametrize("variant", ["left", "right", "two_pass", "left_complex"])
def test_stopping_estimate_equals_relative_change_of_iterates(variant):
    """Sec. 3.1 and Sec. 6: at checkpoint j (a multiple of k, and m_max) the
    estimate is ||f_j - f_{j-k}|| / ||f_j||, the first checkpoint comparing with
    f_0 = 0 (estimate 1).  Each recorded estimate is recomputed here from two
    explicitly formed n-vectors, the iterates of runs fixed at j and j - k
    steps.  Comparing with the wrong checkpoint, normalising by the older
    iterate, dropping the zero padding of z_{j-k} or (right variant) using
    ||z_j - z_{j-k}|| although Y is not orthonormal, all fail it."""
    k, m_max = 3, 11
    if variant in ("left", "right"):
        N = 9
        dims = (N, N, N)
        coeffs = wl.convdiff_stencil(N, 50.0)  # non-normal: Y far from orthonormal
        A = stencil_problem(coeffs, dims)
        a, bb = ops.stencil_interval(coeffs, dims)
        q = pl.chebyshev(a, bb, 2)
        b = wl.rhs(N ** 3, seed=3)
        kw = dict(orth="cgs2", side=variant)
    elif variant == "two_pass":
        N = 9
        dims = (N, N, N)
        coeffs = wl.laplace_stencil(3)
        A = stencil_problem(coeffs, dims)
        a, bb = ops.stencil_interval(coeffs, dims)
        q = pl.chebyshev(a, bb, 1)
        b = wl.rhs(N ** 3, seed=3)
        kw = dict(orth="lanczos", two_pass=True)
    else:
        L = (2, 2, 2, 4)
        U = wl.random_su3(4 * int(np.prod(L)), 0.3, np.random.default_rng(5))
        U = U.reshape(4, L[3], L[2], L[1], L[0], 3, 3)
        A = lambda v: ops.wilson_apply(U, 0.4, v)  # noqa: E731
        b = wl.rhs(12 * int(np.prod(L)), seed=3, complex_=True)
        q = None
        kw = dict(orth="cgs2", side="left")
    run = kr.fAb(A, b, q, "invsqrt", m_max=m_max, tol=1e-300, check_every=k, **kw)
    assert not run.converged and run.iters == m_max
    cps = [j for j, _ in run.history]
    assert cps == [3, 6, 9, 11]          # multiples of k, then m_max
    xs = _fixed_m_iterates(
        lambda j: kr.fAb(A, b, q, "invsqrt", m_max=j, tol=0.0, **kw).x, cps)
    prev = np.zeros_like(b, dtype=np.result_type(b, 1.0))
    for j, est in run.history:
        ref = float(np.linalg.norm(xs[j] - prev) / np.linalg.norm(xs[j]))
        assert abs(est - ref) <= 1e-9 * ref + 1e-13, (j, est, ref)
        prev = xs[j]
    assert run.history[0][1] == 1.0
    # the estimate falls as the iterates converge (so the pin is not vacuous)
    assert run.history[-1][1] < 0.1 * run.history[1][1]
