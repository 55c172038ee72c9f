"""Pins of the oracle's preconditioning polynomials (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import exact, krylov as kr, operators as ops, polynomials as pl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _laplace2d_eigs(N):
    k = np.arange(1, N + 1)
    e = 2 - 2 * np.cos(k * math.pi / (N + 1))
    return (e[:, None] + e[None, :]).ravel()


def test_sec32_example_printed_values():
    """Sec. 3.2: epsilon ~ 0.1263 and kappa(A q(A)^2) = 1.5153 for d = 32."""
    g = json.load(open(os.path.join(GOLDEN, "sec32_laplace2d_example.json")))
    N, d = g["grid"], g["d"]
    lam = _laplace2d_eigs(N)
    a, b = lam.min(), lam.max()
    assert abs(b / a - g["kappa_A_approx"]) < 1.0
    q = pl.chebyshev(a, b, d - 1)
    # uniform relative error of q on the spectral interval
    z = np.linspace(a, b, 400001)
    eps = np.max(np.abs((z ** -0.5 - q.scalar(z)) * np.sqrt(z)))
    assert abs(eps - g["epsilon_printed"]) < 3e-4
    pre = lam * q.scalar(lam) ** 2
    kappa_pre = pre.max() / pre.min()
    assert round(kappa_pre, 4) == g["kappa_pre_printed"]
    # the proposition's bound holds and is close to the printed one
    bound = (1 + 2 * eps + eps ** 2) / (1 - 2 * eps - eps ** 2)
    assert kappa_pre <= bound
    assert abs(bound - g["kappa_pre_bound_printed"]) < 3e-3
    # and the eigenvalues of A q^2 lie in [1 - 2 eps - eps^2, 1 + 2 eps + eps^2]
    assert pre.min() >= 1 - 2 * eps - eps ** 2 - 1e-12
    assert pre.max() <= 1 + 2 * eps + eps ** 2 + 1e-12


@pytest.mark.parametrize("degree", [1, 4, 9, 32])
def test_chebyshev_coefficients_match_numpy_interpolant(degree):
    a, b = 0.05, 13.0
    c = pl.chebyshev_coefficients(pl.inv_sqrt, a, b, degree)
    ref = np.polynomial.chebyshev.chebinterpolate(
        lambda t: (0.5 * (a + b) + 0.5 * (b - a) * t) ** -0.5, degree)
    assert np.allclose(c, ref, rtol=1e-12, atol=1e-13)
    zs = np.linspace(a, b, 101)
    t = (2 * zs - (a + b)) / (b - a)
    assert np.allclose(pl.clenshaw_scalar(c, a, b, zs),
                       np.polynomial.chebyshev.chebval(t, c), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("degree", [0, 1, 5, 16])
def test_clenshaw_matrix_form_against_eigenbasis(degree):
    dims = (6, 5, 4)
    coeffs = wl.laplace_stencil(3)
    a, b = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, b, degree)
    v = wl.rhs(120, seed=1)
    y, nmv = q.apply(lambda x: ops.stencil_apply(coeffs, dims, x), v)
    assert nmv == degree
    A = ops.stencil_matrix(coeffs, dims).toarray()
    lam, Q = np.linalg.eigh(A)
    ref = Q @ (q.scalar(lam) * (Q.T @ v))
    assert np.allclose(y, ref, rtol=0, atol=1e-12 * np.linalg.norm(ref))


def test_chebyshev_positive_on_its_interval_but_branch_check_catches_cut_spectrum():
    # the interpolant of z^{-1/2} stays positive on its own interval ...
    for deg in (1, 2, 7, 16, 31):
        q = pl.chebyshev(1e-6, 1.0, deg)
        z = np.geomspace(1e-6, 1.0, 5001)
        assert q.scalar(z).min() > 0
    # ... but built on an interval that cuts off the top of the spectrum, an
    # odd degree turns negative there (alternating coefficients) and the
    # check over the true spectral interval refuses it (Sec. 3, Sec. 5.1)
    with pytest.raises(pl.BranchError):
        pl.chebyshev(0.1, 6.0, 5, check_interval=(0.1, 8.0))
    pl.chebyshev(0.1, 8.0, 5, check_interval=(0.1, 8.0))


def test_newton_coefficients_solve_the_interpolation_system():
    rng = np.random.default_rng(0)
    th = rng.uniform(0.1, 3.0, 7) + 1j * rng.uniform(-1, 1, 7)
    th = pl.leja_order(th, pair_conjugates=False)
    rho = pl.capacity(th)
    eta = pl.newton_coefficients(pl.inv_sqrt, th, rho)
    # lower-triangular Newton basis matrix N[i, j] = prod_{l<j} (th_i - th_l) / rho
    N = np.ones((7, 7), dtype=complex)
    for j in range(1, 7):
        N[:, j] = N[:, j - 1] * (th - th[j - 1]) / rho
    N = np.tril(N)
    assert np.allclose(eta, np.linalg.solve(N, th ** -0.5), rtol=1e-11)
    assert np.allclose(pl.horner_scalar(th, eta, rho, th), th ** -0.5, rtol=1e-11)


def test_leja_order_brute_force():
    rng = np.random.default_rng(3)
    th = rng.uniform(0.1, 5.0, 9) + 1j * rng.uniform(-2, 2, 9)
    o = pl.leja_order(th, pair_conjugates=False)
    assert sorted(np.round(o, 12), key=lambda z: (z.real, z.imag)) == \
        sorted(np.round(th, 12), key=lambda z: (z.real, z.imag))
    assert abs(o[0]) == np.max(np.abs(th))
    for j in range(1, len(o)):
        prods = [np.prod(np.abs(z - o[:j])) for z in o[j:]]
        assert np.isclose(prods[0], max(prods))


def test_leja_keeps_conjugate_pairs_adjacent():
    th = np.array([1.0 + 0.5j, 1.0 - 0.5j, 3.0, 0.2, 2.0 + 1.0j, 2.0 - 1.0j])
    o = pl.leja_order(th, pair_conjugates=True)
    for j, z in enumerate(o):
        if z.imag > 0:
            assert o[j + 1] == np.conj(z)


def test_ritz_polynomial_is_exact_on_small_diagonal_matrix():
    # n = d distinct eigenvalues: the d Ritz values are the eigenvalues, so
    # q interpolates z^{-1/2} on the whole spectrum and q(A) v = A^{-1/2} v
    a = np.array([0.3, 0.7, 1.1, 2.0, 3.5, 5.0])
    v = wl.rhs(6, seed=2)
    q = pl.ritz(lambda x: a * x, wl.rhs(6, seed=9), degree=5, real_operator=True)
    assert np.allclose(np.sort(q.theta.real), a, rtol=1e-10)
    y, nmv = q.apply(lambda x: a * x, v)
    assert nmv == 5
    assert np.allclose(y, a ** -0.5 * v, rtol=1e-9)


def test_ritz_real_operator_with_complex_ritz_values_gives_real_q():
    dims = (6, 6, 6)
    coeffs = wl.convdiff_stencil(6, 400.0)      # strongly non-normal
    op = lambda x: ops.stencil_apply(coeffs, dims, x)
    q = pl.ritz(op, wl.rhs(216, seed=4), degree=8, real_operator=True)
    v = wl.rhs(216, seed=5)
    yc, _ = pl.horner_apply(op, q.theta, q.eta, q.rho, v)
    assert np.max(np.abs(yc.imag)) <= 1e-10 * np.max(np.abs(yc.real))
    assert np.allclose(q.scalar(q.theta), q.theta ** -0.5, rtol=1e-8)


def test_ritz_rejects_left_half_plane():
    a = np.array([-0.5, 1.0, 2.0, 3.0])
    with pytest.raises(pl.BranchError):
        pl.ritz(lambda x: a * x, np.ones(4), degree=3, real_operator=True)


def test_ritz_polynomial_preconditions_wilson():
    # the Ritz polynomial makes A q(A)^2 close to I on the free Wilson operator
    L = (2, 2, 2, 4)
    U = np.zeros((4, *L, 3, 3), dtype=complex)
    U[...] = np.eye(3)
    m0 = 0.2
    op = lambda x: ops.wilson_apply(U, m0, x)
    n = int(np.prod(L)) * 12
    q = pl.ritz(op, wl.rhs(n, seed=1, complex_=True), degree=6, real_operator=False)
    v = wl.rhs(n, seed=2, complex_=True)
    y, _ = q.apply(op, v)
    ref = exact.wilson_free_fAb(L, m0, v)
    assert np.linalg.norm(y - ref) / np.linalg.norm(ref) < 0.5


def test_harmonic_ritz_values_solve_the_petrov_galerkin_problem():
    """Harmonic Ritz values (Sec. 5.2) against the generalized eigenproblem
    (A V)^H (A V) y = theta (A V)^H V y that defines them, via the Arnoldi
    relation A V_d = V_{d+1} Hbar_d, solved by scipy.linalg.eig."""
    import scipy.linalg as sla
    dims = (6, 5, 4)
    coeffs = wl.convdiff_stencil(6, 80.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    start = wl.rhs(120, seed=3)
    d = 7
    H, h = pl.arnoldi_hessenberg(A, start, d, with_next=True)
    Hbar = np.vstack([H, np.zeros((1, d))])
    Hbar[d, d - 1] = h
    ref = sla.eig(Hbar.conj().T @ Hbar, H.conj().T, right=False)
    got = pl.harmonic_ritz_values(H, h)
    key = lambda z: (round(z.real, 8), round(z.imag, 8))
    assert np.allclose(sorted(got, key=key), sorted(ref, key=key), rtol=1e-10)


def test_harmonic_ritz_values_spd_lie_in_the_spectral_interval():
    # for SPD A the harmonic Ritz values are real and inside [lmin, lmax]
    dims = (9, 8, 7)
    coeffs = wl.laplace_stencil(3)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    lo, hi = ops.stencil_interval(coeffs, dims)
    H, h = pl.arnoldi_hessenberg(A, wl.rhs(504, seed=1), 10, with_next=True)
    th = pl.harmonic_ritz_values(H, h)
    assert np.max(np.abs(th.imag)) < 1e-10
    assert th.real.min() >= lo - 1e-10 and th.real.max() <= hi + 1e-10
    # and they are at least the standard Ritz values' lower end (bounded away from 0)
    assert th.real.min() >= np.linalg.eigvalsh((H + H.T) / 2).min() - 1e-10


def test_harmonic_ritz_polynomial_preconditions():
    N = 10
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 20.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    q = pl.ritz(A, wl.rhs(N ** 3, seed=2), 6, real_operator=True, harmonic=True)
    assert np.allclose(q.scalar(q.theta), q.theta ** -0.5, rtol=1e-8)


# --------------------------------------------------------------------------
# Sec. 5.3: least-squares polynomials on a contour
# --------------------------------------------------------------------------
def test_ls_on_a_circle_is_the_truncated_taylor_series():
    """On N equispaced points of a circle |z - c| = r the monomials (z - c)^j,
    j < N, are orthogonal, so the discrete least-squares fit of degree K is the
    degree-K Taylor polynomial of z^{-1/2} at c up to aliasing of order
    (r / c)^(N - K)."""
    from scipy.special import binom
    c, r, N = 2.0, 1.0, 400
    pts = c + r * np.exp(2j * np.pi * np.arange(N) / N)
    zt = np.array([1.5, 2.3 + 0.4j, 2.0 - 0.7j, 2.9])
    for K in (1, 5, 12):
        q = pl.ls_polynomial(pts, K)
        taylor = sum(binom(-0.5, j) * c ** (-0.5 - j) * (zt - c) ** j for j in range(K + 1))
        assert np.max(np.abs(q.scalar(zt) - taylor)) < 1e-13


def test_ls_fit_equals_lstsq_on_a_scaled_vandermonde():
    """The fitted values P_d alpha are the orthogonal projection of f onto the
    polynomials of degree <= K on the points: compare with numpy's least
    squares on a scaled Vandermonde basis (independent of the Arnoldi basis)."""
    th = np.array([0.3 + 1j, 0.3 - 1j, 6 + 2j, 6 - 2j, 9.0, 2 + 0.1j, 2 - 0.1j])
    pts = pl.ls_contour(th, 0.1, 0.05, symmetric=True)
    f = pl.inv_sqrt(pts)
    cen, sc = 5.0, 6.0
    for K in (2, 5, 8):
        q = pl.ls_polynomial(pts, K, real_operator=True)
        Vd = np.vander((pts - cen) / sc, K + 1, increasing=True)
        coef, *_ = np.linalg.lstsq(Vd, f, rcond=None)
        assert np.max(np.abs(q.scalar(pts) - Vd @ coef)) < 1e-10 * np.max(np.abs(f))
        # real recurrence and coefficients for a conjugate-symmetric point set
        assert not np.iscomplexobj(q.hls) and not np.iscomplexobj(q.alpha)


def test_ls_matrix_recurrence_on_a_diagonal_matrix():
    th = np.array([0.5 + 0.5j, 0.5 - 0.5j, 4.0 + 1j, 4.0 - 1j])
    q = pl.ls_polynomial(pl.ls_contour(th, 0.1, 0.02, symmetric=True), 6, real_operator=True)
    lam = np.linspace(0.6, 3.9, 50)
    v = np.cos(np.arange(50.0))
    y, nmv = q.apply(lambda x: lam * x, v)
    assert nmv == 6
    assert np.max(np.abs(y - q.scalar(lam) * v)) < 1e-13 * np.max(np.abs(y))
    # complex operator, complex point set
    lamc = lam + 0.3j
    qc = pl.ls_polynomial(pl.ls_contour(th + 0.3j, 0.1, 0.02, symmetric=False), 6)
    yc, _ = qc.apply(lambda x: lamc * x, v.astype(complex))
    assert np.max(np.abs(yc - qc.scalar(lamc) * v)) < 1e-13 * np.max(np.abs(yc))


def test_ls_contour_geometry_rectangle_with_min_radius():
    """Hull = rectangle [0.05, 10] x [-1, 1]; the disk |z| < 0.1 cuts its left
    edge, which is replaced by the arc |z| = 0.1 through z = 0.1."""
    th = np.array([0.05 + 1j, 0.05 - 1j, 10 + 1j, 10 - 1j, 3 + 0.2j, 3 - 0.2j])
    step, r = 0.005, 0.1
    pts = pl.ls_contour(th, r, step, symmetric=False)
    chord = 2 * math.sqrt(r * r - 0.05 ** 2)
    length = 2 * 9.95 + 2 * 2.0 - chord + r * 2 * math.acos(0.05 / r)
    N = math.ceil(length / step)
    assert len(pts) == N
    gaps = np.abs(np.diff(np.concatenate([pts, pts[:1]])))
    assert np.max(gaps) <= length / N * (1 + 1e-12)
    assert np.min(np.abs(pts)) >= r * (1 - 1e-14)
    on_arc = np.abs(np.abs(pts) - r) < 1e-12
    assert on_arc.sum() >= 2 and np.min(pts[on_arc].real) >= 0.05 - 1e-15
    assert np.all(pts.real >= 0.05 - 1e-15) and np.all(pts.real <= 10 + 1e-15)
    assert np.all(np.abs(pts.imag) <= 1 + 1e-15)
    on_edges = ((np.abs(pts.real - 0.05) < 1e-12) | (np.abs(pts.real - 10) < 1e-12)
                | (np.abs(np.abs(pts.imag) - 1) < 1e-12) | on_arc)
    assert np.all(on_edges)
    sym = pl.ls_contour(th, r, step, symmetric=True)
    assert len(sym) == 2 * N and np.allclose(np.sort_complex(sym), np.sort_complex(sym.conj()))


def test_ls_contour_of_real_ritz_values_is_a_segment():
    th = np.array([0.05, 0.7, 2.0, 5.0])
    pts = pl.ls_contour(th, 0.1, 0.01, symmetric=True)
    assert np.all(pts.imag == 0.0)
    assert abs(np.min(pts.real) - 0.1) < 1e-12 and np.max(pts.real) <= 5.0
    # forth and back: 2 * 4.9 / 0.01 points, doubled by the symmetric union
    assert len(pts) == 2 * math.ceil(2 * 4.9 / 0.01)


def test_ls_branch_check():
    """A low degree on points reaching close to the branch point cannot stay
    in the right half-plane: the fit is refused."""
    z = np.linspace(1e-4, 1.0, 500).astype(complex)
    with pytest.raises(pl.BranchError):
        pl.ls_polynomial(z, 1)
    assert np.min(pl.ls_polynomial(z, 2).scalar(z).real) > 0


def test_ls_preconditioned_solve_matches_closed_form():
    """Sec. 5.3 polynomial (Ritz values from 60 Arnoldi steps, contour with
    minimum radius 0.1) preconditioning a non-normal conv-diff operator."""
    N = 12
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, 50.0)
    A = lambda v: ops.stencil_apply(coeffs, dims, v)
    start = wl.rhs(N ** 3, seed=4)
    q = pl.least_squares(A, start, 6, real_operator=True, ritz_steps=30, step=0.01)
    assert q.kind == "ls" and q.degree == 6
    b = wl.rhs(N ** 3, seed=0)
    res = kr.fAb(A, b, q, "invsqrt", m_max=300, tol=1e-12)
    assert res.converged
    ref = exact.stencil_fAb_dst(coeffs, dims, b, "invsqrt")
    assert np.linalg.norm(res.x - ref) / np.linalg.norm(ref) < 1e-10
    plain = kr.fAb(A, b, None, "invsqrt", m_max=300, tol=1e-12)
    assert res.iters < plain.iters
