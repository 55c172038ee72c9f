"""Polynomially preconditioned Arnoldi / Lanczos for A^{-1/2} b and A^{1/2} b.

Test infrastructure only (see the package header).

Follows Sec. 3.1 of the paper:

* Algorithm 1 (left preconditioning): c = q(A) b, v_1 = c / ||c||; each step
  forms w = q(A) (q(A) (A v_j)) in three stages (A once, q(A) twice, never a
  representation of q^2), orthogonalizes w against v_1..v_j (h_ij = <w, v_i>,
  i.e. v_i^H w), h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}; the approximation is
  f_m = V_m H_m^{-1/2} e_1 ||c||.
* Algorithm 2 (right preconditioning): v_1 = b / ||b||; each step stores
  y_j = q(A) v_j and forms w = A (q(A) y_j); f_m = Y_m H_m^{-1/2} e_1 ||b||.
* Orthogonalization: classical Gram-Schmidt applied twice ("cgs2"), modified
  Gram-Schmidt as printed in the algorithms ("mgs"), or the three-term Lanczos
  recurrence for Hermitian A q(A)^2 ("lanczos", used in the paper's Example 1).
* H_m^{-1/2} e_1: Schur-based principal square root of H_m, then a linear
  solve (Sec. 3.1); for Lanczos the eigendecomposition of the tridiagonal T_m.
  The principal branch must exist: H_m may have no eigenvalue on (-inf, 0].
* Stopping (Sec. 3.1, Sec. 6): every k iterations the coefficient vector z_j is
  formed and the relative change ||f_j - f_{j-k}|| / ||f_j|| of the iterate is
  estimated; with left preconditioning this equals ||z_j - [z_{j-k}; 0]|| / ||z_j||
  because V is orthonormal.  k defaults to max(1, floor(64 / d)) (Examples 1, 2).
* Square root (Sec. 4): A^{1/2} b = A^{-1/2} (A b); a singular A with a
  semisimple eigenvalue 0 needs no change (theorem on implicit
  desingularization).

A (lucky) breakdown is declared when h_{j+1,j} <= 1e-12 times the largest
column norm of H seen so far (the norm of column i equals ||A q(A)^2 v_i|| when
the basis is orthonormal, so this is a lower estimate of ||A q(A)^2||); the
Krylov space is then invariant to that accuracy and the iterate is exact in it.

Pins (tests/test_oracle_krylov.py): DST closed forms, dense sqrtm for tiny n,
diagonal A, the Arnoldi relation and orthogonality, sqrt/invsqrt identities,
agreement of plain and preconditioned and of left and right variants, the
Sec. 6 Example 1 iteration counts (Table 1) and operation-count rules.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .polynomials import Poly, one


class HessenbergError(ValueError):
    """H_m has an eigenvalue on (-inf, 0]: no principal H_m^{-1/2}."""


@dataclass
class Result:
    x: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    mvms: int
    inner_products: int
    est: float
    checks: int
    H: np.ndarray = None
    V: np.ndarray = None
    history: list = field(default_factory=list)


def default_check_every(degree):
    """k = 64 / d with d = degree + 1 (Sec. 6, Examples 1 and 2), at least 1."""
    return max(1, 64 // (degree + 1))


# --------------------------------------------------------------------------
# dense H^{-1/2} e_1
# --------------------------------------------------------------------------
def hessenberg_invsqrt_e1(H, beta):
    """z = H^{-1/2} (beta e_1): principal square root by Schur, then solve."""
    H = np.asarray(H)
    m = H.shape[0]
    ev = np.linalg.eigvals(H)
    scale = max(1.0, float(np.max(np.abs(ev))))
    bad = (ev.real <= 0.0) & (np.abs(ev.imag) <= 1e-12 * scale)
    if np.any(bad):
        raise HessenbergError("H has an eigenvalue on (-inf, 0]")
    S = sla.sqrtm(H)
    rhs = np.zeros(m, dtype=np.result_type(S, 1.0))
    rhs[0] = beta
    z = sla.solve(S, rhs)
    if not np.iscomplexobj(H):
        z = z.real
    return z


def tridiagonal_invsqrt_e1(alpha, beta_off, beta):
    """z = T^{-1/2} (beta e_1) for symmetric tridiagonal T by eigendecomposition."""
    lam, Q = sla.eigh_tridiagonal(np.asarray(alpha, dtype=np.float64),
                                  np.asarray(beta_off, dtype=np.float64))
    if np.min(lam) <= 0.0:
        raise HessenbergError("T has an eigenvalue <= 0")
    return Q @ (lam ** -0.5 * (Q[0, :] * beta))


# --------------------------------------------------------------------------
# the preconditioned Krylov method
# --------------------------------------------------------------------------
def fAb(apply_A, b, poly: Poly | None = None, kind="invsqrt", m_max=100, tol=1e-10,
        check_every=0, orth="cgs2", side="left", x_true=None, keep_basis=False,
        two_pass=False):
    """Approximate A^{-1/2} b (kind "invsqrt") or A^{1/2} b (kind "sqrt").

    apply_A: callable x -> A x.  poly: preconditioning polynomial (None: q == 1).
    orth: "cgs2" | "mgs" | "lanczos".  side: "left" (Algorithm 1) | "right"
    (Algorithm 2, with the y_j stored).  tol: stopping threshold on the
    difference-of-iterates estimate; with x_true given the true relative error
    ||f_j - x_true|| / ||x_true|| is tested instead (as in Example 1's tables).
    tol <= 0 runs exactly m_max steps.
    two_pass (Lanczos): the first pass keeps only the three-term
    coefficients (and the two latest vectors); after it stops, a second pass
    regenerates the basis with the same coefficients and accumulates
    x = V_m z_m, so no basis is stored and the products with A double (the
    two-pass Lanczos of Sec. 6, Example 1).  With side "right" the iterate
    Y_m z_m is q(A) (V_m z_m), one more q(A) after pass 2; there the
    stopping estimate would need the y_j, so only a fixed m (tol <= 0) is run.
    """
    if two_pass:
        return _two_pass_lanczos(apply_A, b, poly or one(), kind, m_max, tol, check_every, side)
    poly = poly or one()
    b = np.asarray(b)
    dt = np.result_type(b, 1.0)
    mvms = 0
    ips = 0

    def A(x):
        nonlocal mvms
        mvms += 1
        return apply_A(x)

    def Q(x):
        nonlocal mvms
        y, k = poly.apply(apply_A, x)
        mvms += k
        return y.astype(dt, copy=False)

    # Sec. 4: the square root through the inverse square root
    if kind == "sqrt":
        b = A(b).astype(dt, copy=False)
    elif kind != "invsqrt":
        raise ValueError("kind must be 'sqrt' or 'invsqrt'")

    n = b.size
    start = Q(b) if side == "left" else np.array(b, dtype=dt)
    beta = float(np.linalg.norm(start))
    if beta == 0.0:
        return Result(x=np.zeros(n, dtype=dt), iters=0, converged=True, breakdown=False,
                      mvms=mvms, inner_products=0, est=0.0, checks=0)

    k = check_every if check_every > 0 else default_check_every(poly.degree)
    V = np.zeros((n, m_max + 1), dtype=dt)
    Y = np.zeros((n, m_max), dtype=dt) if side == "right" else None
    H = np.zeros((m_max + 1, m_max), dtype=dt)
    V[:, 0] = start / beta

    def coeffs(m):
        if orth == "lanczos":
            return tridiagonal_invsqrt_e1(np.real(np.diag(H[:m, :m])),
                                          np.real(np.diag(H[:m, :m], -1)), beta)
        return hessenberg_invsqrt_e1(H[:m, :m], beta)

    def iterate(m, z):
        B = V[:, :m] if side == "left" else Y[:, :m]
        return B @ z

    z_prev = np.zeros(0)
    est = 1.0
    checks = 0
    converged = False
    breakdown = False
    m = m_max
    history = []
    colmax = 0.0
    for j in range(m_max):
        # three-stage preconditioned product (Algorithm 1 / Algorithm 2)
        if side == "left":
            w = Q(Q(A(V[:, j])))
        else:
            Y[:, j] = Q(V[:, j])
            w = A(Q(Y[:, j])).astype(dt, copy=False)
        w = np.array(w, dtype=dt)
        # orthogonalization; h[i] = v_i^H w
        if orth == "cgs2":
            h = np.zeros(j + 1, dtype=dt)
            for _ in range(2):
                g = V[:, :j + 1].conj().T @ w
                w = w - V[:, :j + 1] @ g
                h += g
                ips += j + 1
        elif orth == "mgs":
            h = np.zeros(j + 1, dtype=dt)
            for i in range(j + 1):
                h[i] = np.vdot(V[:, i], w)
                w = w - V[:, i] * h[i]
                ips += 1
        elif orth == "lanczos":
            h = np.zeros(j + 1, dtype=dt)
            if j > 0:
                h[j - 1] = H[j, j - 1]
                w = w - H[j, j - 1] * V[:, j - 1]
            h[j] = np.vdot(V[:, j], w)
            w = w - h[j] * V[:, j]
            ips += 1
        else:
            raise ValueError("orth must be 'cgs2', 'mgs' or 'lanczos'")
        H[:j + 1, j] = h
        hn = float(np.linalg.norm(w))
        ips += 1
        H[j + 1, j] = hn
        colmax = max(colmax, math.sqrt(float(np.linalg.norm(h)) ** 2 + hn ** 2))
        if hn <= 1e-12 * colmax:
            m = j + 1
            breakdown = True
            converged = True
            break
        V[:, j + 1] = w / hn
        # stopping test every k steps and at m_max
        jj = j + 1
        if tol > 0.0 and (jj % k == 0 or jj == m_max):
            z = coeffs(jj)
            checks += 1
            if x_true is not None:
                fj = iterate(jj, z)
                est = float(np.linalg.norm(fj - x_true) / np.linalg.norm(x_true))
            else:
                zp = np.zeros_like(z)
                zp[:z_prev.size] = z_prev
                if side == "left":
                    est = float(np.linalg.norm(z - zp) / np.linalg.norm(z))
                else:
                    est = float(np.linalg.norm(iterate(jj, z - zp))
                                / np.linalg.norm(iterate(jj, z)))
            history.append((jj, est))
            z_prev = z
            if est <= tol:
                m = jj
                converged = True
                break
    z = coeffs(m)
    x = iterate(m, z)
    return Result(x=x, iters=m, converged=converged, breakdown=breakdown, mvms=mvms,
                  inner_products=ips, est=est, checks=checks,
                  H=H[:m + 1, :m].copy() if keep_basis else None,
                  V=V[:, :m + 1].copy() if keep_basis else None, history=history)


def _two_pass_lanczos(apply_A, b, poly, kind, m_max, tol, check_every, side="left"):
    """Two-pass Lanczos for Hermitian A q(A)^2 (Sec. 6, Example 1), with
    the start vector and product of Algorithm 1 (left) or Algorithm 2 (right)."""
    if side not in ("left", "right"):
        raise ValueError("side must be 'left' or 'right'")
    if side == "right" and tol > 0.0:
        raise ValueError("two-pass with right preconditioning runs a fixed m (tol <= 0)")
    b = np.asarray(b)
    dt = np.result_type(b, 1.0)
    mvms = 0

    def A(x):
        nonlocal mvms
        mvms += 1
        return apply_A(x)

    def Q(x):
        nonlocal mvms
        y, k = poly.apply(apply_A, x)
        mvms += k
        return y.astype(dt, copy=False)

    def start():  # Algorithm 1: c = q(A) b; Algorithm 2: b itself
        return Q(b) if side == "left" else np.array(b, dtype=dt)

    def product(v):  # Algorithm 1: q(A) q(A) A v; Algorithm 2: A q(A) q(A) v
        return Q(Q(A(v))) if side == "left" else A(Q(Q(v))).astype(dt, copy=False)

    if kind == "sqrt":
        b = A(b).astype(dt, copy=False)
    c = start()
    beta = float(np.linalg.norm(c))
    n = b.size
    if beta == 0.0:
        return Result(x=np.zeros(n, dtype=dt), iters=0, converged=True, breakdown=False,
                      mvms=mvms, inner_products=0, est=0.0, checks=0)
    k = check_every if check_every > 0 else default_check_every(poly.degree)
    alpha = np.zeros(m_max)
    off = np.zeros(m_max)   # off[j] = beta_{j+1} = h_{j+1,j}
    # pass 1: coefficients only
    v_prev = np.zeros(n, dtype=dt)
    v = c / beta
    z_prev = np.zeros(0)
    m, est, checks, converged, breakdown = m_max, 1.0, 0, False, False
    colmax = 0.0
    ips = 0
    history = []
    for j in range(m_max):
        w = product(v)
        if j > 0:
            w = w - off[j - 1] * v_prev
        alpha[j] = np.real(np.vdot(v, w))
        w = w - alpha[j] * v
        off[j] = float(np.linalg.norm(w))
        ips += 2
        colmax = max(colmax, math.sqrt(alpha[j] ** 2 + off[j] ** 2 + (off[j - 1] ** 2 if j else 0)))
        if off[j] <= 1e-12 * colmax:
            m, breakdown, converged = j + 1, True, True
            break
        v_prev, v = v, w / off[j]
        jj = j + 1
        if tol > 0.0 and (jj % k == 0 or jj == m_max):
            z = tridiagonal_invsqrt_e1(alpha[:jj], off[:jj - 1], beta)
            checks += 1
            zp = np.zeros_like(z)
            zp[:z_prev.size] = z_prev
            est = float(np.linalg.norm(z - zp) / np.linalg.norm(z))
            history.append((jj, est))
            z_prev = z
            if est <= tol:
                m, converged = jj, True
                break
    z = tridiagonal_invsqrt_e1(alpha[:m], off[:m - 1], beta)
    # pass 2: regenerate v_1..v_m with the stored coefficients and combine
    c = start()
    v_prev = np.zeros(n, dtype=dt)
    v = c / beta
    x = z[0] * v
    for j in range(m - 1):
        w = product(v)
        if j > 0:
            w = w - off[j - 1] * v_prev
        w = w - alpha[j] * v
        v_prev, v = v, w / off[j]
        x = x + z[j + 1] * v
    if side == "right":
        x = Q(x)  # Y_m z_m = q(A) V_m z_m
    return Result(x=x, iters=m, converged=converged, breakdown=breakdown, mvms=mvms,
                  inner_products=ips, est=est, checks=checks, history=history)
