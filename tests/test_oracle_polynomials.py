"""Pins of the oracle's preconditioning polynomials (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import exact, operators as ops, polynomials as pl

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
