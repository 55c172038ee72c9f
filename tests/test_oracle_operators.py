"""Pins of the oracle's operators (CPU only).

Each check compares the oracle with something that is not the oracle: an
assembled sparse matrix, dense eigenvalues, algebraic identities of the Dirac
matrices, or the Fourier symbol of the free Wilson operator.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import exact, operators as ops


@pytest.mark.parametrize("dims", [(5, 4, 3), (7, 6, 1), (1, 1, 9)])
def test_stencil_matches_assembled_csr(dims):
    c = wl.convdiff_stencil(8, 50.0)
    x = wl.rhs(int(np.prod(dims)), seed=3)
    rp, ci, va = wl.stencil_csr(dims, c)
    y_csr = ops.csr_apply(rp, ci, va, x)
    y_st = ops.stencil_apply(c, dims, x)
    y_sp = ops.stencil_matrix(c, dims) @ x
    assert np.allclose(y_st, y_csr, rtol=0, atol=1e-14)
    assert np.allclose(y_st, y_sp, rtol=0, atol=1e-14)


def test_csr_counts_poisson32():
    # the 2D Poisson 32x32 CSR: 5 n - 4 N entries
    rp, ci, va = wl.stencil_csr((32, 32, 1), wl.laplace_stencil(2))
    assert rp[-1] == 5 * 1024 - 4 * 32 == 4992
    assert np.all(np.diff(rp) > 0)


@pytest.mark.parametrize("coeffs,dims", [
    (wl.laplace_stencil(2), (9, 7, 1)),
    (wl.laplace_stencil(3), (5, 6, 4)),
    (wl.convdiff_stencil(6, 50.0), (6, 6, 6)),
    (wl.convdiff_stencil(6, 10.0), (6, 5, 4)),
])
def test_stencil_interval_is_dense_spectrum(coeffs, dims):
    A = ops.stencil_matrix(coeffs, dims).toarray()
    ev = np.linalg.eigvals(A)
    assert np.max(np.abs(ev.imag)) < 1e-8
    lo, hi = ops.stencil_interval(coeffs, dims)
    assert abs(lo - ev.real.min()) < 1e-10 and abs(hi - ev.real.max()) < 1e-10


def test_laplace3d_interval_matches_example1_formula():
    # Sec. 6, Example 1 states [6(1 - cos(pi/(N+1))), 12 - 6(1 - cos(pi/(N+1)))]
    N = 100
    lo, hi = ops.stencil_interval(wl.laplace_stencil(3), (N, N, N))
    s = 6 * (1 - math.cos(math.pi / (N + 1)))
    assert lo == pytest.approx(s, rel=1e-13) and hi == pytest.approx(12 - s, rel=1e-13)


def test_laplace2d_condition_number_sec32():
    # Sec. 3.2 example: kappa(A) ~ 1054 for the 50 x 50 Laplacian
    lo, hi = ops.stencil_interval(wl.laplace_stencil(2), (50, 50, 1))
    assert round(hi / lo) == 1053 or round(hi / lo) == 1054
    assert abs(hi / lo - 1054) < 1.0


def test_gamma_algebra():
    g, g5 = ops.gamma_matrices()
    I4 = np.eye(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        assert np.allclose(g[mu] @ g[mu], I4)
        for nu in range(mu + 1, 4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 0)
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0)
    assert np.allclose(g[0] @ g[1] @ g[2] @ g[3], g5)


def _dense(apply, n, dtype=np.complex128):
    M = np.zeros((n, n), dtype=dtype)
    for i in range(n):
        e = np.zeros(n, dtype=dtype)
        e[i] = 1
        M[:, i] = apply(e)
    return M


def test_wilson_gamma5_hermiticity_and_field_of_values():
    L = 2
    U = wl.su3_links(L, eps=1.5, seed=11)
    m0 = 0.05
    n = L ** 4 * 12
    D = _dense(lambda v: ops.wilson_apply(U, m0, v), n)
    G5 = _dense(ops.gamma5_apply, n)
    assert np.allclose(G5 @ D @ G5, D.conj().T, atol=1e-13)
    # Hermitian part >= m0, hence spec(D) in Re z >= m0
    herm = 0.5 * (D + D.conj().T)
    assert np.linalg.eigvalsh(herm).min() >= m0 - 1e-12
    assert np.linalg.eigvals(D).real.min() >= m0 - 1e-12


def test_device_link_generator_matches_host():
    # the torch matrix exponential used for the 64 x 32^3 lattice gives the
    # host generator's links (eigendecomposition) to rounding
    U = wl.su3_links_device((2, 2, 2, 3), eps=0.3, seed=1, device="cpu").numpy()
    assert np.abs(U - wl.su3_links((2, 2, 2, 3), eps=0.3, seed=1)).max() < 1e-13


def test_links_are_su3():
    U = wl.su3_links(2, eps=0.3, seed=1).reshape(-1, 3, 3)
    assert np.allclose(U @ U.conj().transpose(0, 2, 1), np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-13)


def test_wilson_free_field_symbol():
    # D b through the stencil equals (D^{1/2})^2 b through the Fourier symbol
    L = (4, 2, 3, 4)
    m0 = 0.3
    U = np.zeros((4, *L, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    b = wl.rhs(int(np.prod(L)) * 12, seed=2, complex_=True)
    y = ops.wilson_apply(U, m0, b)
    s = exact.wilson_free_fAb(L, m0, exact.wilson_free_fAb(L, m0, b, "sqrt"), "sqrt")
    assert np.allclose(y, s, atol=1e-12)


def test_wilson_chemical_potential_free_symbol():
    # unit links: D(mu) acts in momentum space as (m0 + a) + i sum gamma s at
    # the complex temporal momentum p_t - i mu (a plane wave picks up e^{+mu}
    # from the forward temporal hop and e^{-mu} from the backward one)
    L = (4, 2, 3, 4)
    m0, mu = -1.4, 0.3
    U = np.zeros((4, *L, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    b = wl.rhs(int(np.prod(L)) * 12, seed=6, complex_=True)
    y = ops.wilson_apply(U, m0, b, mu)
    g, _ = ops.gamma_matrices()
    a, s = exact.wilson_free_symbol(L, mu)
    bh = np.fft.fftn(b.reshape(*L, 4, 3), axes=(0, 1, 2, 3))
    yh = (m0 + a)[..., None, None] * bh + 1j * sum(
        s[nu][..., None, None] * np.einsum("st,...tc->...sc", g[nu], bh) for nu in range(4))
    assert np.allclose(y, np.fft.ifftn(yh, axes=(0, 1, 2, 3)).reshape(-1), atol=1e-12)


def test_wilson_chemical_potential_gamma5_relation_and_q2():
    # D(mu)^H = G5 D(-mu) G5; Q = G5 D(0) is Hermitian and Q^2 positive
    # semidefinite; Q^2 for mu != 0 is not Hermitian
    L = 2
    U = wl.su3_links(L, eps=1.5, seed=11)
    m0, mu = -1.4, 0.3
    n = L ** 4 * 12
    G5 = _dense(ops.gamma5_apply, n)
    Dp = _dense(lambda v: ops.wilson_apply(U, m0, v, mu), n)
    Dm = _dense(lambda v: ops.wilson_apply(U, m0, v, -mu), n)
    assert np.allclose(Dp.conj().T, G5 @ Dm @ G5, atol=1e-13)
    D0 = _dense(lambda v: ops.wilson_apply(U, m0, v), n)
    Q0 = G5 @ D0
    assert np.allclose(Q0, Q0.conj().T, atol=1e-13)
    Q2 = _dense(lambda v: ops.wilson_q2_apply(U, m0, v), n)
    assert np.allclose(Q2, Q0 @ Q0, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (Q2 + Q2.conj().T)).min() > -1e-12
    Q2m = _dense(lambda v: ops.wilson_q2_apply(U, m0, v, mu), n)
    assert np.allclose(Q2m, (G5 @ Dp) @ (G5 @ Dp), atol=1e-12)
    assert not np.allclose(Q2m, Q2m.conj().T, atol=1e-3)


def test_wilson_free_q2_closed_form_against_dense():
    # the scalar symbol of Q^2 against the dense principal square root of the
    # assembled Q^2 (unit links, mu = 0.3)
    L = (2, 2, 2, 2)
    m0, mu = -1.4, 0.3
    U = np.zeros((4, *L, 3, 3), dtype=np.complex128)
    U[...] = np.eye(3)
    n = 16 * 12
    Q2 = _dense(lambda v: ops.wilson_q2_apply(U, m0, v, mu), n)
    b = wl.rhs(n, seed=9, complex_=True)
    for kind in ("invsqrt", "sqrt"):
        ref = exact.dense_fAb(Q2, b, kind)
        assert np.allclose(exact.wilson_free_q2_fAb(L, m0, b, mu, kind), ref, atol=1e-11)


def test_wilson_pure_gauge_equivalence():
    L = 3
    U, G = wl.pure_gauge_links(L, seed=4)
    m0 = 0.1
    n = L ** 4 * 12
    b = wl.rhs(n, seed=5, complex_=True)
    U1 = np.zeros_like(U)
    U1[...] = np.eye(3)
    G4 = G
    gb = np.einsum("...ba,...sb->...sa", G4.conj(), b.reshape(L, L, L, L, 4, 3))
    ref = np.einsum("...ab,...sb->...sa", G4,
                    ops.wilson_apply(U1, m0, gb.reshape(-1)).reshape(L, L, L, L, 4, 3))
    assert np.allclose(ops.wilson_apply(U, m0, b), ref.reshape(-1), atol=1e-12)


@pytest.mark.parametrize("coeffs,dims", [
    (wl.laplace_stencil(2), (7, 6, 1)),
    (wl.laplace_stencil(3), (4, 5, 3)),
    (wl.convdiff_stencil(5, 10.0), (5, 4, 6)),
])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_dst_closed_form_against_dense_sqrtm(coeffs, dims, kind):
    A = ops.stencil_matrix(coeffs, dims).toarray()
    b = wl.rhs(A.shape[0], seed=8)
    ref = exact.dense_fAb(A, b, kind)
    y = exact.stencil_fAb_dst(coeffs, dims, b, kind)
    assert np.allclose(y, ref, rtol=0, atol=1e-11 * np.linalg.norm(ref))
