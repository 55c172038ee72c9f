"""Block Arnoldi for f(A) B with several right-hand sides (B is n x s).

Test infrastructure only (see the package header).

The paper treats one right-hand side at a time.  Right-hand sides that share
A can instead be run together in one block Krylov space
K_m(A q(A)^2, C) = span{C, (A q^2) C, ..., (A q^2)^{m-1} C},  C = q(A) B'
(B' = B, or A B for the square root, Sec. 4): the natural block form of
Algorithm 1, with the scalars of the single-vector method replaced by s x s
blocks.  Steps, in order:

* C = V_1 R (thin QR, R upper triangular with a non-negative diagonal);
* for j = 1, 2, ...: W = q(A) (q(A) (A V_j)) (three stages, as Algorithm 1);
  classical block Gram-Schmidt twice, H_{ij} = V_i^H W summed over both
  passes; W = V_{j+1} H_{j+1,j} (thin QR);
* F_j = [V_1 .. V_j] H_j^{-1/2} E_1 R with the block upper Hessenberg H_j
  (js x js) and E_1 the first s columns of the identity (principal square
  root by Schur, then a solve);
* stop every k steps when, for every column c, ||Z_j e_c - [Z_{j-k} e_c; 0]||
  / ||Z_j e_c|| <= tol (V orthonormal: the relative change of column c of the
  iterate).

A step whose new block W is numerically zero (every diagonal entry of
H_{j+1,j} <= 1e-12 times the largest column norm of H seen) is a lucky
breakdown; a partial rank loss would need deflation, which is not part of
this method: it raises DeflationError.

Pins (tests/test_oracle_block.py): s = 1 against the single-vector oracle,
columns against the DST closed form, the block Arnoldi relation and
orthonormality, exactness once the block Krylov space is the whole space,
and equivariance under column permutations.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .krylov import HessenbergError, default_check_every
from .polynomials import Poly, one


class DeflationError(ValueError):
    """The new block lost rank partially (block Arnoldi would need deflation)."""


@dataclass
class BlockResult:
    X: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    mvms: int          # products of A with single vectors
    est: np.ndarray    # per-column estimate at the last check
    checks: int
    H: np.ndarray = None
    V: np.ndarray = None


def thin_qr(W):
    """W = Q R with R's diagonal made non-negative."""
    Qm, R = np.linalg.qr(W)
    d = np.diag(R)
    sg = np.where(d < 0, -1.0, 1.0).astype(R.dtype)
    return Qm * sg, (R.T * sg).T


def block_invsqrt_E1R(H, R):
    """Z = H^{-1/2} E_1 R (principal square root by Schur, then a solve)."""
    ev = np.linalg.eigvals(H)
    scale = max(1.0, float(np.max(np.abs(ev))))
    if np.any((ev.real <= 0.0) & (np.abs(ev.imag) <= 1e-12 * scale)):
        raise HessenbergError("H has an eigenvalue on (-inf, 0]")
    S = sla.sqrtm(H)
    s = R.shape[0]
    rhs = np.zeros((H.shape[0], s), dtype=np.result_type(S, R, 1.0))
    rhs[:s, :] = R
    Z = sla.solve(S, rhs)
    if not np.iscomplexobj(H):
        Z = Z.real
    return Z


def block_fAB(apply_A, B, poly: Poly | None = None, kind="invsqrt", m_max=30, tol=1e-10,
              check_every=0, keep_basis=False):
    """Approximate A^{-1/2} B (kind "invsqrt") or A^{1/2} B (kind "sqrt")."""
    poly = poly or one()
    B = np.asarray(B)
    n, s = B.shape
    dt = np.result_type(B, 1.0)
    mvms = 0

    def A(X):
        nonlocal mvms
        mvms += X.shape[1]
        return np.stack([np.asarray(apply_A(X[:, c]), dtype=dt) for c in range(X.shape[1])], 1)

    def Q(X):
        nonlocal mvms
        cols = []
        for c in range(X.shape[1]):
            y, k = poly.apply(apply_A, X[:, c])
            mvms += k
            cols.append(np.asarray(y, dtype=dt))
        return np.stack(cols, 1)

    if kind == "sqrt":
        B = A(B)
    elif kind != "invsqrt":
        raise ValueError("kind must be 'sqrt' or 'invsqrt'")
    C = Q(B)
    V1, R = thin_qr(C)
    if np.min(np.abs(np.diag(R))) <= 1e-12 * max(np.max(np.abs(R)), 1e-300):
        raise DeflationError("the start block is rank deficient")
    k = check_every if check_every > 0 else default_check_every(poly.degree)
    Vs = [V1]
    H = np.zeros(((m_max + 1) * s, m_max * s), dtype=dt)
    Zprev = np.zeros((0, s))
    est = np.ones(s)
    checks = 0
    m = m_max
    converged = breakdown = False
    colmax = 0.0
    for j in range(m_max):
        W = Q(Q(A(Vs[j])))
        Vall = np.concatenate(Vs, 1)
        for _ in range(2):
            P = Vall.conj().T @ W
            W = W - Vall @ P
            H[:(j + 1) * s, j * s:(j + 1) * s] += P
        Vn, Rn = thin_qr(W)
        H[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Rn
        colmax = max(colmax, float(np.max(np.linalg.norm(H[:(j + 2) * s, j * s:(j + 1) * s],
                                                         axis=0))))
        small = np.abs(np.diag(Rn)) <= 1e-12 * colmax
        if np.all(small):
            m, breakdown, converged = j + 1, True, True
            break
        if np.any(small):
            raise DeflationError("partial rank loss of the new block")
        Vs.append(Vn)
        jj = j + 1
        if tol > 0.0 and (jj % k == 0 or jj == m_max):
            Z = block_invsqrt_E1R(H[:jj * s, :jj * s], R)
            checks += 1
            Zp = np.zeros_like(Z)
            Zp[:Zprev.shape[0], :] = Zprev
            est = np.linalg.norm(Z - Zp, axis=0) / np.linalg.norm(Z, axis=0)
            Zprev = Z
            if np.max(est) <= tol:
                m, converged = jj, True
                break
    Z = block_invsqrt_E1R(H[:m * s, :m * s], R)
    Vall = np.concatenate(Vs[:m], 1)
    X = Vall @ Z
    return BlockResult(X=X, iters=m, converged=converged, breakdown=breakdown, mvms=mvms,
                       est=est, checks=checks,
                       H=H[:(m + 1) * s, :m * s].copy() if keep_basis else None,
                       V=np.concatenate(Vs[:m + 1], 1) if keep_basis else None)
