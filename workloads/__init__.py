"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only *generates data*: right-hand sides, sparse matrices, stencil
coefficient vectors, lattice gauge links and start vectors.  It contains none
of the method's arithmetic (no Krylov step, no polynomial, no matrix
function), so both the HIP path and the CPU oracle may consume what it makes
without sharing any of the computation.

Problem shapes follow the paper's workloads (section 6 and the 2D example of
section 3.2):

* 2D / 3D discrete Laplacians on a grid of N^dim interior points, zero
  Dirichlet boundary, unscaled (the diagonal is 2*dim), x the fastest index;
* a 3D first-order upwind convection-diffusion operator, the non-Hermitian
  stand-in for the directed-graph Laplacian of Example 3;
* a 4D Wilson-Dirac-like operator with random SU(3) links, the stand-in for
  the lattice-QCD operator of Example 2 (whose gauge field is not public);
* directed-graph in-degree Laplacians (Example 3's structure: L = D_in - A).

Stencil operators are described by seven coefficients
``[c0, c_xm, c_xp, c_ym, c_yp, c_zm, c_zp]`` with

    (A u)_p = c0 u_p + c_xm u_{p-ex} + c_xp u_{p+ex} + c_ym u_{p-ey}
              + c_yp u_{p+ey} + c_zm u_{p-ez} + c_zp u_{p+ez},

neighbours outside the grid being zero (Dirichlet).  Vectors are stored with
x fastest, i.e. a C-ordered array of shape (nz, ny, nx).
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rhs",
    "laplace_stencil",
    "convdiff_stencil",
    "laplace2d_csr",
    "stencil_csr",
    "digraph_laplacian_csr",
    "powerlaw_digraph_laplacian_csr",
    "su3_links",
    "pure_gauge_links",
    "random_su3",
    "CONFIGS",
]


# --------------------------------------------------------------------------
# right-hand sides and start vectors
# --------------------------------------------------------------------------
def rhs(n: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """b ~ N(0,1) entrywise, unnormalised (relative errors are scale-free).

    For complex vectors the real and imaginary parts are independent N(0,1)
    draws: first all real parts, then all imaginary parts.
    """
    rng = np.random.default_rng(seed)
    if not complex_:
        return rng.standard_normal(n)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


# --------------------------------------------------------------------------
# stencil operators
# --------------------------------------------------------------------------
def laplace_stencil(dim: int) -> np.ndarray:
    """Unscaled 5-point (dim=2) or 7-point (dim=3) negative Laplacian."""
    if dim == 2:
        return np.array([4.0, -1.0, -1.0, -1.0, -1.0, 0.0, 0.0])
    if dim == 3:
        return np.array([6.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0])
    raise ValueError("dim must be 2 or 3")


def convdiff_stencil(N: int, pe: float, direction=(1.0, 0.5, 0.25)) -> np.ndarray:
    """First-order upwind convection-diffusion on the unit cube, times h^2.

    h = 1/(N+1), gamma_d = h * Pe * direction_d, and

        (A u)_p = (6 + sum gamma) u_p - sum_d [(1+gamma_d) u_{p-e_d} + u_{p+e_d}].
    """
    h = 1.0 / (N + 1)
    g = [h * pe * float(t) for t in direction]
    return np.array([6.0 + sum(g),
                     -(1.0 + g[0]), -1.0,
                     -(1.0 + g[1]), -1.0,
                     -(1.0 + g[2]), -1.0])


def stencil_csr(dims, coeffs):
    """CSR (int32 row pointers / column indices, float64 values) of a stencil.

    dims = (nx, ny, nz); column indices are sorted within each row.
    """
    nx, ny, nz = (int(d) for d in dims)
    c = np.asarray(coeffs, dtype=np.float64)
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    # (offset_z, offset_y, offset_x, coefficient index)
    for dz, dy, dx, k in ((-1, 0, 0, 5), (0, -1, 0, 3), (0, 0, -1, 1), (0, 0, 0, 0),
                          (0, 0, 1, 2), (0, 1, 0, 4), (1, 0, 0, 6)):
        if c[k] == 0.0:
            continue
        zs = slice(max(0, -dz), nz - max(0, dz))
        ys = slice(max(0, -dy), ny - max(0, dy))
        xs = slice(max(0, -dx), nx - max(0, dx))
        r = idx[zs, ys, xs]
        col = idx[zs.start + dz:zs.stop + dz, ys.start + dy:ys.stop + dy,
                  xs.start + dx:xs.stop + dx]
        rows.append(r.ravel())
        cols.append(col.ravel())
        vals.append(np.full(r.size, c[k]))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), cols.astype(np.int32), vals


def laplace2d_csr(N: int):
    """CSR of the unscaled 5-point Laplacian on an N x N interior grid."""
    return stencil_csr((N, N, 1), laplace_stencil(2))


def _csr_from_coo(n, rows, cols, vals):
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64)


def digraph_laplacian_csr(n: int, p: float = 0.08, seed: int = 3):
    """In-degree Laplacian L = D_in - A of a random directed graph.

    A_ij = 1 for an edge i -> j drawn with probability p (no self loops);
    D_in holds the in-degrees (column sums of A), so every column of L sums
    to zero and L is singular.  Returned as CSR.
    """
    rng = np.random.default_rng(seed)
    adj = (rng.random((n, n)) < p).astype(np.float64)
    np.fill_diagonal(adj, 0.0)
    # adj[i, j] = 1 for an edge i -> j; column j collects the in-edges of j
    L = np.diag(adj.sum(axis=0)) - adj
    rows, cols = np.nonzero(L)
    return _csr_from_coo(n, rows, cols, L[rows, cols])


def powerlaw_digraph_laplacian_csr(n: int, nnz_target: int, exponent: float = 2.2,
                                   seed: int = 5):
    """In-degree Laplacian of a synthetic directed power-law graph.

    Out-degrees follow a discrete power law with the given exponent, edge
    heads are drawn with probability proportional to a second power-law
    weight, duplicates and self loops are dropped.  The number of stored
    entries of L (off-diagonals plus the diagonal) is close to nnz_target.
    """
    rng = np.random.default_rng(seed)
    m_edges = max(1, nnz_target - n)
    w_out = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (exponent - 1.0))
    w_in = rng.permutation(w_out)
    w_out = w_out / w_out.sum()
    w_in = w_in / w_in.sum()
    src = rng.choice(n, size=int(m_edges * 1.15), p=w_out)
    dst = rng.choice(n, size=src.size, p=w_in)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = np.unique(src.astype(np.int64) * n + dst)[:m_edges]
    src, dst = key // n, key % n
    # L = D_in - A with A[src, dst] = 1 for an edge src -> dst, so that
    # column j of L sums to in-degree(j) - in-degree(j) = 0
    indeg = np.bincount(dst, minlength=n).astype(np.float64)
    rows = np.concatenate([src, np.arange(n)])
    cols = np.concatenate([dst, np.arange(n)])
    vals = np.concatenate([-np.ones(dst.size), indeg])
    keep = vals != 0.0
    return _csr_from_coo(n, rows[keep], cols[keep], vals[keep])


# --------------------------------------------------------------------------
# lattice gauge fields
# --------------------------------------------------------------------------
def _gell_mann() -> np.ndarray:
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / math.sqrt(3)
    l[7][2, 2] = -2 / math.sqrt(3)
    return l


def _expi_hermitian(H: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for a stack of Hermitian traceless 3x3 matrices."""
    w, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", Q, ph, Q.conj())


def random_su3(count: int, eps: float, rng) -> np.ndarray:
    """count matrices exp(i eps H), H = sum_a xi_a lambda_a / 2, xi_a ~ N(0,1)."""
    xi = rng.standard_normal((count, 8))
    H = np.einsum("na,aij->nij", xi, _gell_mann()) / 2.0
    return _expi_hermitian(H, eps)


def su3_links(L, eps: float = 0.3, seed: int = 1) -> np.ndarray:
    """Random SU(3) links near the identity on a periodic 4D lattice: L^4
    for an int L, else L = (L_t, L_z, L_y, L_x).

    Returned shape (4, L_t, L_z, L_y, L_x, 3, 3) = [mu][t][z][y][x][a][b],
    i.e. one 3x3 complex matrix per direction and site, sites with x fastest.
    Direction mu = 0, 1, 2, 3 is x, y, z, t.
    """
    dims = (L, L, L, L) if np.isscalar(L) else tuple(int(d) for d in L)
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    U = random_su3(4 * V, eps, rng)
    return U.reshape(4, *dims, 3, 3)


def su3_links_device(L, eps: float = 0.3, seed: int = 1, device="cuda"):
    """su3_links for lattices where the host eigendecompositions would take
    long (a 64 x 32^3 lattice has 8.4 M links): the same H from the same
    seeded stream, exp(i eps H) taken by torch's matrix exponential on
    `device` (equal to su3_links' result to rounding).  Returns a complex128
    tensor on `device` of shape (4, L_t, L_z, L_y, L_x, 3, 3)."""
    import torch

    dims = (L, L, L, L) if np.isscalar(L) else tuple(int(d) for d in L)
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    xi = torch.from_numpy(rng.standard_normal((4 * V, 8))).to(device)
    lam = torch.from_numpy(_gell_mann()).to(device)
    H = torch.einsum("na,aij->nij", xi.to(torch.complex128), lam) / 2.0
    del xi
    U = torch.linalg.matrix_exp((1j * eps) * H)
    return U.reshape(4, *dims, 3, 3)


def pure_gauge_links(L: int, seed: int = 7, eps: float = 2.0):
    """Links U_mu(x) = G(x) G(x+mu)^H of a random gauge transformation G.

    Returns (links, G) with G of shape (L, L, L, L, 3, 3).  The operator built
    on such links is unitarily equivalent to the free operator.
    """
    rng = np.random.default_rng(seed)
    G = random_su3(L ** 4, eps, rng).reshape(L, L, L, L, 3, 3)
    links = np.empty((4, L, L, L, L, 3, 3), dtype=np.complex128)
    # axis of direction mu in the (t, z, y, x) site array
    for mu, ax in enumerate((3, 2, 1, 0)):
        Gf = np.roll(G, -1, axis=ax)  # G(x + mu)
        links[mu] = np.einsum("...ab,...cb->...ac", G, Gf.conj())
    return links, G


# --------------------------------------------------------------------------
# the benchmark workloads, described by their parameters
# --------------------------------------------------------------------------
CONFIGS = {
    # 2D Poisson 32x32, CSR, Hermitian, Chebyshev degrees 0 and 8
    "poisson2d_32": dict(kind="csr_laplace2d", N=32, degrees=(0, 8), tol=1e-10,
                         m_max=200, f="invsqrt", hermitian=True),
    # 3D convection-diffusion 128^3 at Pe = 50, Chebyshev degrees 0/4/16/32
    "convdiff3d_128": dict(kind="convdiff3d", N=128, pe=50.0, degrees=(0, 4, 16, 32),
                           tol=1e-8, f=("sqrt", "invsqrt")),
    # 4D Wilson-like 16^4 with links exp(0.3 i H), mass shift 0.05, Ritz degree 16
    "wilson4d_16": dict(kind="wilson4d", L=16, eps=0.3, m0=0.05, degrees=(0, 16),
                        tol=1e-8, f="invsqrt"),
}


# --------------------------------------------------------------------------
# serving: a stream of requests (arrival times and request parameters only)
# --------------------------------------------------------------------------
SERVING_TYPES = (
    # name, weight in the mix
    ("laplace2d_256", 0.30),
    ("convdiff3d_64", 0.25),
    ("convdiff3d_96", 0.15),
    ("convdiff3d_128", 0.10),
    ("wilson4d_16", 0.20),
)


def poisson_arrivals(qps: float, count: int, seed: int = 11) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate qps:
    cumulative sums of exponential gaps with mean 1/qps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / qps, size=count))


def serving_mix(count: int, seed: int = 12):
    """Request parameters of the serving workload: operator type (by weight),
    f in {sqrt, invsqrt} and tol in {1e-6, 1e-10}, each half and half, and the
    seed of the request's right-hand side."""
    rng = np.random.default_rng(seed)
    names = [t[0] for t in SERVING_TYPES]
    w = np.array([t[1] for t in SERVING_TYPES])
    typ = rng.choice(len(names), size=count, p=w / w.sum())
    kind = rng.integers(0, 2, size=count)
    tol = rng.integers(0, 2, size=count)
    return [dict(type=names[typ[i]], kind=("sqrt", "invsqrt")[kind[i]],
                 tol=(1e-6, 1e-10)[tol[i]], seed=1000 + i) for i in range(count)]
