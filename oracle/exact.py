"""Exact references for f(A) b, f(z) = z^{-1/2} or z^{1/2}, in FP64.

Test infrastructure only (see the package header).

These compute the quantity the method approximates (its plain definition,
Sec. 1: the action of the principal matrix square root or inverse square root
on a vector) without any Krylov iteration, so they pin the iterative oracle:

* ``stencil_fAb_dst``: separable stencils whose 1D factors are similar to
  symmetric tridiagonal Toeplitz matrices (the Laplacian of Sec. 3.2 and of
  Example 1; the convection-diffusion operator at moderate Peclet number).
  f(A) b = S F f(Lambda) F S^{-1} b with F the orthonormal DST-I in every
  direction and S the diagonal similarity.
* ``wilson_free_fAb``: the Wilson-like operator with unit links, diagonal in
  momentum space: D(p) = (m0 + sum(1 - cos p_mu)) I + i sum gamma_mu sin p_mu, a
  4x4 matrix a I + i S with S^2 = |s|^2 I, whose function is
  (f(a + i|s|) + f(a - i|s|))/2 I + (f(a + i|s|) - f(a - i|s|))/(2 i |s|) (i S).
* ``wilson_free_q2_fAb``: Q^2 with Q = Gamma_5 D for unit links and a
  chemical potential mu (the temporal momentum becomes p_t - i mu): Gamma_5
  anticommutes with every gamma_nu, so Q^2 = (a - i S)(a + i S) = a^2 + S^2,
  and S^2 = sum_nu s_nu^2 (complex s_nu when mu != 0) is a multiple of the
  identity: f(Q^2) is the scalar f(a^2 + sum s_nu^2) in momentum space
  (Sec. 6, Example 2 computes (Q^2)^{-1/2} b).
* ``wilson_pure_gauge_fAb``: links U_mu(x) = G(x) G(x + mu)^H make the
  operator G D_free G^H, so f(D) b = G f(D_free) (G^H b).
* ``dense_fAb``: scipy.linalg.sqrtm of a dense matrix (Schur method), for
  tiny n.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from .operators import gamma_matrices


def _f(kind):
    if kind == "invsqrt":
        return lambda z: 1.0 / np.sqrt(z)
    if kind == "sqrt":
        return np.sqrt
    raise ValueError(kind)


def stencil_fAb_dst(coeffs, dims, b, kind="invsqrt"):
    """f(A) b for a 7-coefficient stencil with c_dm * c_dp > 0 in every direction.

    Direction d is tridiag(c_dm, ., c_dp) = D_d T_d D_d^{-1}, D_d = diag(delta_d^i),
    delta_d = sqrt(c_dm / c_dp), T_d symmetric with off-diagonal
    t_d = sign(c_dm) sqrt(c_dm c_dp), eigenvalues 2 t_d cos(k pi / (N_d + 1)).
    Accuracy degrades like cond(S) = prod_d delta_d^{max(N_d - 1, 0)}.
    """
    nx, ny, nz = (int(d) for d in dims)
    c = [float(t) for t in coeffs]
    f = _f(kind)
    shape = (nz, ny, nx)
    lam = np.full(shape, c[0])
    scale = np.ones(shape)
    for ax, N, cm, cp in ((2, nx, c[1], c[2]), (1, ny, c[3], c[4]), (0, nz, c[5], c[6])):
        if N == 1:
            continue
        if cm * cp <= 0.0:
            raise ValueError("direction without real similarity")
        t = math.copysign(math.sqrt(cm * cp), cm)
        delta = math.sqrt(cm / cp)
        k = np.arange(1, N + 1)
        ev = 2.0 * t * np.cos(k * math.pi / (N + 1))
        sh = [1, 1, 1]
        sh[ax] = N
        lam = lam + ev.reshape(sh)
        scale = scale * (delta ** np.arange(N)).reshape(sh)
    axes = [ax for ax, N in ((2, nx), (1, ny), (0, nz)) if N > 1]
    u = np.asarray(b).reshape(shape) / scale
    uh = sfft.dstn(u, type=1, axes=axes, norm="ortho")
    uh = f(lam.astype(np.result_type(uh, lam))) * uh
    return (sfft.idstn(uh, type=1, axes=axes, norm="ortho") * scale).reshape(-1)


def _fourier_symbol_apply(L, m0, bh, kind):
    g, _ = gamma_matrices()
    f = _f(kind)
    # site axes are [t][z][y][x]; direction mu = x, y, z, t
    Lt, Lz, Ly, Lx = L
    pt, pz, py, px = np.meshgrid(*(2.0 * math.pi * np.arange(n) / n for n in (Lt, Lz, Ly, Lx)),
                                 indexing="ij")
    pm = (px, py, pz, pt)
    a = m0 + sum(1.0 - np.cos(q) for q in pm)
    s = [np.sin(q) for q in pm]
    snorm = np.sqrt(sum(si ** 2 for si in s))
    fp = f(a + 1j * snorm)
    fm = f(a - 1j * snorm)
    c0 = 0.5 * (fp + fm)
    with np.errstate(invalid="ignore", divide="ignore"):
        c1 = np.where(snorm > 0.0, (fp - fm) / (2j * np.where(snorm > 0, snorm, 1.0)), 0.0)
    # S chi = sum_mu gamma_mu s_mu chi (spin matmul), applied to bh[..., s, c]
    Sb = sum(np.einsum("st,...tc->...sc", g[mu], bh) * s[mu][..., None, None]
             for mu in range(4))
    return c0[..., None, None] * bh + (c1[..., None, None] * 1j) * Sb


def wilson_free_fAb(L, m0, b, kind="invsqrt"):
    """f(D) b for unit links on an L = (L_t, L_z, L_y, L_x) periodic lattice."""
    b4 = np.asarray(b, dtype=np.complex128).reshape(*L, 4, 3)
    bh = np.fft.fftn(b4, axes=(0, 1, 2, 3))
    # a plane wave e^{i p x} picks up e^{+i p_mu} from psi(x + mu): the forward
    # transform here uses e^{-i p x}, i.e. a mode b(x) = e^{+i p x} lands on p.
    yh = _fourier_symbol_apply(L, m0, bh, kind)
    return np.fft.ifftn(yh, axes=(0, 1, 2, 3)).reshape(-1)


def wilson_free_symbol(L, mu=0.0):
    """(a, s) of D(p) = a I + i sum_nu gamma_nu s_nu for unit links on an
    L = (L_t, L_z, L_y, L_x) lattice: a = sum_nu (1 - cos q_nu) (without the
    mass shift), s_nu = sin q_nu, q = p except q_t = p_t - i mu.  Arrays over
    the momentum grid in the layout of numpy's fftn of a [t][z][y][x] field;
    s ordered x, y, z, t."""
    Lt, Lz, Ly, Lx = L
    pt, pz, py, px = np.meshgrid(*(2.0 * math.pi * np.arange(n) / n for n in (Lt, Lz, Ly, Lx)),
                                 indexing="ij")
    q = (px.astype(complex), py.astype(complex), pz.astype(complex), pt - 1j * mu)
    a = sum(1.0 - np.cos(qi) for qi in q)
    s = [np.sin(qi) for qi in q]
    return a, s


def wilson_free_q2_fAb(L, m0, b, mu=0.0, kind="invsqrt"):
    """f(Q^2) b, Q = Gamma_5 D, for unit links with chemical potential mu."""
    a, s = wilson_free_symbol(L, mu)
    a = a + m0
    lam = a * a + sum(si * si for si in s)
    b4 = np.asarray(b, dtype=np.complex128).reshape(*L, 4, 3)
    bh = np.fft.fftn(b4, axes=(0, 1, 2, 3))
    yh = _f(kind)(lam)[..., None, None] * bh
    return np.fft.ifftn(yh, axes=(0, 1, 2, 3)).reshape(-1)


def wilson_pure_gauge_fAb(G, m0, b, kind="invsqrt"):
    """f(D) b for links U_mu(x) = G(x) G(x + mu)^H, G of shape (L_t, L_z, L_y, L_x, 3, 3)."""
    G = np.asarray(G)
    L = G.shape[:4]
    b4 = np.asarray(b, dtype=np.complex128).reshape(*L, 4, 3)
    gb = np.einsum("...ba,...sb->...sa", G.conj(), b4)      # G^H b
    y = wilson_free_fAb(L, m0, gb.reshape(-1), kind).reshape(*L, 4, 3)
    return np.einsum("...ab,...sb->...sa", G, y).reshape(-1)  # G y


def dense_fAb(A, b, kind="invsqrt"):
    """f(A) b from the dense principal square root (scipy's Schur method)."""
    A = np.asarray(A)
    S = sla.sqrtm(A)
    if kind == "sqrt":
        y = S @ b
    else:
        y = sla.solve(S, b)
    if not np.iscomplexobj(A) and not np.iscomplexobj(b):
        y = y.real
    return y
