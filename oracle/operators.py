"""Operators A of the paper's experiments, applied to vectors in FP64.

Test infrastructure only (see the package header).

* 7-point (3D) / 5-point (2D) stencils with zero Dirichlet boundary: the
  discrete Laplacian of Sec. 3.2's example and of Sec. 6 Example 1, and a
  first-order upwind convection-diffusion operator standing in for the
  non-Hermitian matrices of Examples 2 and 3.
* CSR matrices (the sparse matrix-vector product of Examples 1 and 3).
* A Wilson-Dirac-like operator on a periodic 4D lattice with 12 complex
  degrees of freedom per site (Example 2 describes the Wilson-Dirac operator
  and its spinor layout: 4 spins x 3 colours), with an optional chemical
  potential, and the square Q^2 of Q = Gamma_5 D whose inverse square root
  Example 2 computes.

Pins: ``stencil_apply`` against the assembled CSR and the DST eigenbasis
(tests/test_oracle_operators.py); ``wilson_apply`` against gamma-5
hermiticity (with a chemical potential: D(mu)^H = Gamma_5 D(-mu) Gamma_5),
the free-field Fourier symbol (at a complex temporal momentum for mu != 0)
and the pure-gauge equivalence; ``wilson_q2_apply`` against the Hermitian
positive semidefinite Q^2 at mu = 0; ``*_interval`` against dense
eigenvalues on small grids.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# --------------------------------------------------------------------------
# stencils
# --------------------------------------------------------------------------
def stencil_apply(coeffs, dims, x):
    """y = A x for a 7-coefficient stencil on an nx*ny*nz grid, x fastest.

    coeffs = [c0, c_xm, c_xp, c_ym, c_yp, c_zm, c_zp]:

        (A u)_p = c0 u_p + c_xm u_{p-ex} + c_xp u_{p+ex} + ... ,

    with neighbours outside the grid taken as zero (Dirichlet).  A 2D
    operator is the case nz = 1.
    """
    nx, ny, nz = (int(d) for d in dims)
    c = [float(t) for t in coeffs]
    u = np.asarray(x).reshape(nz, ny, nx)
    y = c[0] * u
    y[:, :, 1:] += c[1] * u[:, :, :-1]
    y[:, :, :-1] += c[2] * u[:, :, 1:]
    y[:, 1:, :] += c[3] * u[:, :-1, :]
    y[:, :-1, :] += c[4] * u[:, 1:, :]
    y[1:, :, :] += c[5] * u[:-1, :, :]
    y[:-1, :, :] += c[6] * u[1:, :, :]
    return y.reshape(-1)


def stencil_interval(coeffs, dims):
    """Exact real eigenvalue interval [lo, hi] of a stencil operator.

    The operator is a Kronecker sum of 1D tridiagonal Toeplitz matrices
    tridiag(c_dm, ., c_dp) (plus c0 on the diagonal).  When c_dm * c_dp > 0 for
    every direction each factor is diagonally similar to a symmetric one with
    off-diagonal sqrt(c_dm c_dp), whose eigenvalues are
    2 sqrt(c_dm c_dp) cos(k pi / (N_d + 1)), k = 1..N_d.  For the Laplacian this
    is the interval the paper states in Sec. 6, Example 1.
    Returns None when some direction has c_dm * c_dp < 0 (complex spectrum).
    """
    nx, ny, nz = (int(d) for d in dims)
    c = [float(t) for t in coeffs]
    spread = 0.0
    for N, cm, cp in ((nx, c[1], c[2]), (ny, c[3], c[4]), (nz, c[5], c[6])):
        prod = cm * cp
        if N == 1 or prod == 0.0:
            continue
        if prod < 0.0:
            return None
        spread += 2.0 * math.sqrt(prod) * math.cos(math.pi / (N + 1))
    return c[0] - spread, c[0] + spread


def stencil_matrix(coeffs, dims):
    """The stencil assembled as a scipy CSR matrix (for dense checks)."""
    nx, ny, nz = (int(d) for d in dims)

    def T(N, cm, cp):
        return sp.diags([np.full(N - 1, cm), np.full(N - 1, cp)], [-1, 1],
                        shape=(N, N), format="csr")

    c = [float(t) for t in coeffs]
    Ix, Iy, Iz = (sp.identity(k, format="csr") for k in (nx, ny, nz))
    A = c[0] * sp.identity(nx * ny * nz, format="csr")
    A = A + sp.kron(Iz, sp.kron(Iy, T(nx, c[1], c[2])))
    A = A + sp.kron(Iz, sp.kron(T(ny, c[3], c[4]), Ix))
    A = A + sp.kron(T(nz, c[5], c[6]), sp.kron(Iy, Ix))
    return A.tocsr()


# --------------------------------------------------------------------------
# CSR
# --------------------------------------------------------------------------
def csr_apply(rowptr, colind, vals, x):
    """y = A x for A in CSR form (row pointers, column indices, values)."""
    n = len(rowptr) - 1
    A = sp.csr_matrix((np.asarray(vals), np.asarray(colind), np.asarray(rowptr)),
                      shape=(n, n))
    return A @ np.asarray(x)


# --------------------------------------------------------------------------
# Wilson-Dirac-like operator on a periodic 4D lattice
# --------------------------------------------------------------------------
_SIGMA = (np.array([[0, 1], [1, 0]], dtype=np.complex128),
          np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
          np.array([[1, 0], [0, -1]], dtype=np.complex128))


def gamma_matrices():
    """Euclidean Dirac matrices in the chiral basis.

    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x, y, z),
    gamma_t = [[0, I], [I, 0]], gamma_5 = diag(I, -I): Hermitian, square to I
    and anticommute.  gamma_5 acts as +1 on spins 1, 2 and -1 on spins 3, 4,
    as the paper describes Gamma_5 in Example 2.
    Returns (g, g5) with g of shape (4, 4, 4) indexed [mu][s][s'], mu = x,y,z,t.
    """
    Z = np.zeros((2, 2), dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    g = np.empty((4, 4, 4), dtype=np.complex128)
    for k in range(3):
        g[k] = np.block([[Z, -1j * _SIGMA[k]], [1j * _SIGMA[k], Z]])
    g[3] = np.block([[Z, I2], [I2, Z]])
    g5 = np.diag([1, 1, -1, -1]).astype(np.complex128)
    return g, g5


# the lattice array is [t][z][y][x]; direction mu = x, y, z, t lives on axis:
_AXIS = (3, 2, 1, 0)


def wilson_apply(links, m0, psi, mu=0.0):
    """y = D psi for the Wilson-Dirac-like operator with mass shift m0:

        (D psi)(x) = (4 + m0) psi(x)
                     - 1/2 sum_nu [ e^{+mu d_nu,t} (I - gamma_nu) U_nu(x) psi(x + nu)
                                    + e^{-mu d_nu,t} (I + gamma_nu) U_nu(x - nu)^H psi(x - nu) ].

    links: (4, L_t, L_z, L_y, L_x, 3, 3) complex; psi: flat complex vector of
    length V*12 in [t][z][y][x][spin][colour] order.  Periodic boundaries.
    mu: the chemical potential of Sec. 6, Example 2, as the factors e^{+-mu}
    on the temporal hops (the usual lattice form; the paper gives no formula,
    it only says that mu != 0 makes Gamma_5 D non-Hermitian).  For mu = 0 the
    Hermitian part is m0 + 1/2 sum_nu (I - X_nu)^H (I - X_nu) >= m0 with X_nu
    the (unitary) gauge-covariant forward shift, so spec(D) lies in the
    half-plane Re z >= m0.
    """
    g, _ = gamma_matrices()
    U = np.asarray(links)
    shp = U.shape[1:5]
    p = np.asarray(psi, dtype=np.complex128).reshape(*shp, 4, 3)
    out = (4.0 + m0) * p
    for nu in range(4):
        ax = _AXIS[nu]
        ef, eb = (math.exp(mu), math.exp(-mu)) if nu == 3 else (1.0, 1.0)
        fwd = np.roll(p, -1, axis=ax)                         # psi(x + nu)
        up = ef * np.einsum("...ab,...sb->...sa", U[nu], fwd)  # U_nu(x) psi(x+nu)
        Ub = np.roll(U[nu], 1, axis=ax)                       # U_nu(x - nu)
        bwd = np.roll(p, 1, axis=ax)                          # psi(x - nu)
        dn = eb * np.einsum("...ba,...sb->...sa", Ub.conj(), bwd)  # U^H psi(x-nu)
        gup = np.einsum("st,...tc->...sc", g[nu], up)
        gdn = np.einsum("st,...tc->...sc", g[nu], dn)
        out = out - 0.5 * ((up - gup) + (dn + gdn))
    return out.reshape(-1)


def wilson_q2_apply(links, m0, psi, mu=0.0):
    """y = Q^2 psi with Q = Gamma_5 D (Sec. 6, Example 2: the sign function
    of Q through (Q^2)^{-1/2}; Q^2 is applied as two products with Q, never
    formed)."""
    q = gamma5_apply(wilson_apply(links, m0, psi, mu))
    return gamma5_apply(wilson_apply(links, m0, q, mu))


def gamma5_apply(psi):
    """Gamma_5 psi: +psi on spins 1, 2, -psi on spins 3, 4."""
    p = np.asarray(psi).reshape(-1, 4, 3).copy()
    p[:, 2:, :] *= -1.0
    return p.reshape(-1)
