"""Pins of the block Arnoldi oracle (several right-hand sides)."""
import numpy as np
import pytest

import workloads as wl
from oracle import block as bk, exact, krylov as kr, operators as ops, polynomials as pl


def rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def _stencil(N, pe=50.0):
    dims = (N, N - 2, N - 3)
    coeffs = wl.convdiff_stencil(N, pe)
    a, b = ops.stencil_interval(coeffs, dims)
    return dims, coeffs, (lambda v: ops.stencil_apply(coeffs, dims, v)), a, b


@pytest.mark.parametrize("degree", [0, 3])
@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_one_column_is_the_single_vector_method(degree, kind):
    dims, coeffs, A, a, b = _stencil(10)
    q = pl.chebyshev(a, b, degree)
    bv = wl.rhs(int(np.prod(dims)), seed=0)
    blk = bk.block_fAB(A, bv[:, None], q, kind, m_max=12, tol=0.0)
    one = kr.fAb(A, bv, q, kind, m_max=12, tol=0.0)
    assert blk.iters == one.iters == 12 and blk.mvms == one.mvms
    assert rel(blk.X[:, 0], one.x) < 1e-12


@pytest.mark.parametrize("kind", ["invsqrt", "sqrt"])
def test_columns_match_the_closed_form(kind):
    dims, coeffs, A, a, b = _stencil(12)
    n = int(np.prod(dims))
    B = np.stack([wl.rhs(n, seed=s) for s in range(4)], 1)
    res = bk.block_fAB(A, B, pl.chebyshev(a, b, 4), kind, m_max=60, tol=1e-12)
    assert res.converged and np.max(res.est) <= 1e-12
    for c in range(4):
        ref = exact.stencil_fAb_dst(coeffs, dims, B[:, c], kind)
        assert rel(res.X[:, c], ref) < 1e-10
    # a block space holds each column's own Krylov space: no more steps than one column
    single = kr.fAb(A, B[:, 0], pl.chebyshev(a, b, 4), kind, m_max=60, tol=1e-12)
    assert res.iters <= single.iters


def test_block_arnoldi_relation_and_orthonormality():
    dims, coeffs, A, a, b = _stencil(9)
    n = int(np.prod(dims))
    q = pl.chebyshev(a, b, 2)
    B = np.stack([wl.rhs(n, seed=s) for s in range(3)], 1)
    res = bk.block_fAB(A, B, q, "invsqrt", m_max=6, tol=0.0, keep_basis=True)
    V, H = res.V, res.H
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) < 1e-13
    AqqV = np.stack([q.apply(A, q.apply(A, A(V[:, c]))[0])[0] for c in range(18)], 1)
    assert np.max(np.abs(AqqV - V @ H)) < 1e-12 * np.max(np.abs(H))
    # block upper Hessenberg: zero below the first block subdiagonal
    for j in range(6):
        assert np.all(H[(j + 2) * 3:, j * 3:(j + 1) * 3] == 0.0)


def test_exact_when_the_block_space_is_everything():
    lam = np.linspace(0.5, 7.0, 12)
    A = lambda v: lam * v
    B = np.stack([wl.rhs(12, seed=s) for s in range(4)], 1)
    res = bk.block_fAB(A, B, None, "invsqrt", m_max=3, tol=0.0)
    assert rel(res.X, lam[:, None] ** -0.5 * B) < 1e-12
    # one more step finds the invariant space: a lucky breakdown
    res2 = bk.block_fAB(A, B, None, "invsqrt", m_max=5, tol=0.0)
    assert res2.breakdown and res2.iters == 3
    assert rel(res2.X, lam[:, None] ** -0.5 * B) < 1e-12


def test_column_permutation_equivariance():
    dims, coeffs, A, a, b = _stencil(8)
    n = int(np.prod(dims))
    B = np.stack([wl.rhs(n, seed=s) for s in range(4)], 1)
    q = pl.chebyshev(a, b, 3)
    perm = [2, 0, 3, 1]
    r1 = bk.block_fAB(A, B, q, "invsqrt", m_max=5, tol=0.0)
    r2 = bk.block_fAB(A, B[:, perm], q, "invsqrt", m_max=5, tol=0.0)
    assert rel(r2.X, r1.X[:, perm]) < 1e-11


def test_partial_rank_loss_is_refused():
    dims, coeffs, A, a, b = _stencil(8)
    n = int(np.prod(dims))
    b0 = wl.rhs(n, seed=0)
    with pytest.raises(bk.DeflationError):
        bk.block_fAB(A, np.stack([b0, 2.0 * b0], 1), None, "invsqrt", m_max=4, tol=0.0)
