"""Preconditioning polynomials q ~ z^{-1/2} and their action q(A) v, in FP64.

Test infrastructure only (see the package header).

The method needs a polynomial q with q(A) ~ A^{-1/2}, so that A q(A)^2 is
close to the identity (Sec. 3, eq. prec_identity).  Degree convention: a
polynomial of degree K uses d = K + 1 coefficients or nodes (the paper's d,
Sec. 6), and degree 0 means the plain, unpreconditioned method, q == 1.

Three constructions from Sec. 5 are implemented:

* Sec. 5.1, Chebyshev: q is the Chebyshev polynomial approximation of z^{-1/2}
  on a real interval [a, b] containing spec(A).  The paper states the weighted
  projection integral; this oracle evaluates it with the d-point
  Gauss-Chebyshev rule, which makes q the interpolant of z^{-1/2} at the d
  first-kind Chebyshev points of [a, b] (reading recorded in the design notes;
  it reproduces the Sec. 3.2 example's printed kappa(A q^2) = 1.5153).  q(A) v is
  evaluated with the matrix-vector form of the Clenshaw recurrence.  The
  branch condition of Sec. 3 (spec(q(A)) in the right half-plane) is checked
  numerically by testing q > 0 on a fine grid of [a, b], as Sec. 5.1 suggests.
* Sec. 5.2, Ritz values: d steps of Arnoldi on A give a Hessenberg H_d whose
  eigenvalues (Ritz values) theta are the interpolation nodes.  The
  interpolant of z^{-1/2} is stored in Newton form on Leja-ordered nodes and
  evaluated with a Horner-type recurrence.  Nodes with Re theta <= 0 are
  rejected (the Ritz values must lie in the right half-plane for the
  principal branch to be plausible, Sec. 5.2).

* Sec. 5.3, least squares: the boundary of the convex hull of Ritz values,
  kept at distance >= r_min from 0 by an arc, discretized at equal arc
  length; Arnoldi on diag(z_1..z_N) gives orthonormal polynomials p_j and
  alpha = P_d^H z^{-1/2}; q(A) v is evaluated with the same recurrence in A.

Pins (tests/test_oracle_polynomials.py): the Sec. 3.2 example's epsilon and
kappa(A q^2); Clenshaw against the Chebyshev-polynomial power form and the
DST eigenbasis; interpolation property q(theta) = theta^{-1/2} at the nodes;
exactness of q(A) v when A is diagonal; Leja ordering against brute force;
least squares on a circle against the truncated Taylor series, against
numpy's least squares on a Vandermonde basis, and the contour's geometry
against closed-form lengths.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def inv_sqrt(z):
    """Principal branch z^{-1/2}, branch cut on (-inf, 0] (Sec. 3)."""
    return 1.0 / np.sqrt(np.asarray(z))


class BranchError(ValueError):
    """q would not give the principal inverse square root (Sec. 3, Sec. 5)."""


@dataclass
class Poly:
    """A preconditioning polynomial in one of three representations.

    kind == "one":    q == 1 (degree 0, the plain method).
    kind == "cheb":   q(z) = sum_i c[i] T_i((2 z - (a + b)) / (b - a)).
    kind == "newton": q(z) = sum_j eta[j] prod_{i<j} (z - theta[i]) / rho.
    kind == "ls":     q(z) = sum_j alpha[j] p_j(z), p_j the orthonormal
                      polynomials of the discrete inner product on `npts`
                      contour points, given by their Arnoldi recurrence
                      hls (d x (d - 1), Hessenberg).
    """
    kind: str
    degree: int
    a: float = 0.0
    b: float = 0.0
    c: np.ndarray = field(default_factory=lambda: np.zeros(0))
    theta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    eta: np.ndarray = field(default_factory=lambda: np.zeros(0))
    rho: float = 1.0
    real_operator: bool = True
    hls: np.ndarray = field(default_factory=lambda: np.zeros((0, 0)))
    alpha: np.ndarray = field(default_factory=lambda: np.zeros(0))
    npts: int = 0

    # ---- scalar evaluation ------------------------------------------------
    def scalar(self, z):
        z = np.asarray(z)
        if self.kind == "one":
            return np.ones_like(z, dtype=np.result_type(z, 1.0))
        if self.kind == "cheb":
            return clenshaw_scalar(self.c, self.a, self.b, z)
        if self.kind == "ls":
            return ls_scalar(self.hls, self.alpha, self.npts, z)
        return horner_scalar(self.theta, self.eta, self.rho, z)

    # ---- action on a vector -----------------------------------------------
    def apply(self, apply_A, v):
        """Return (q(A) v, number of products with A)."""
        if self.kind == "one":
            return np.array(v, copy=True), 0
        if self.kind == "cheb":
            return clenshaw_apply(apply_A, self.c, self.a, self.b, v)
        if self.kind == "ls":
            return ls_apply(apply_A, self.hls, self.alpha, self.npts, v)
        y, nmv = horner_apply(apply_A, self.theta, self.eta, self.rho, v)
        if self.real_operator and not np.iscomplexobj(v):
            y = y.real.copy()
        return y, nmv


def one() -> Poly:
    return Poly(kind="one", degree=0)


# --------------------------------------------------------------------------
# Sec. 5.1: Chebyshev approximation on [a, b]
# --------------------------------------------------------------------------
def chebyshev_coefficients(f, a, b, degree):
    """Coefficients c_0..c_K of the Chebyshev approximation of f on [a, b].

    Sec. 5.1 defines c_i = (2 / pi) * int_a^b w f T_i^{[a,b]} (c_0 with 1/pi),
    w = ((x - a)(b - x))^{-1/2}.  With x = (a + b)/2 + (b - a)/2 cos(t) the
    integral is (2 / pi) int_0^pi f(x(t)) cos(i t) dt, evaluated here with the
    d = K + 1 point midpoint (Gauss-Chebyshev) rule t_k = pi (k + 1/2) / d.
    """
    d = degree + 1
    t = math.pi * (np.arange(d) + 0.5) / d
    x = 0.5 * (a + b) + 0.5 * (b - a) * np.cos(t)
    fx = f(x)
    c = np.array([2.0 / d * np.sum(fx * np.cos(i * t)) for i in range(d)])
    c[0] *= 0.5
    return c


def clenshaw_scalar(c, a, b, z):
    """sum_i c_i T_i(zhat) at scalar points by the Clenshaw recurrence."""
    z = np.asarray(z, dtype=np.result_type(z, 1.0))
    zh = (2.0 * z - (a + b)) / (b - a)
    b1 = np.zeros_like(zh)
    b2 = np.zeros_like(zh)
    for k in range(len(c) - 1, 0, -1):
        b1, b2 = c[k] + 2.0 * zh * b1 - b2, b1
    return c[0] + zh * b1 - b2


def clenshaw_apply(apply_A, c, a, b, v):
    """q(A) v by the matrix-vector Clenshaw recurrence (Sec. 5.1).

    With Ahat = (2 A - (a + b) I) / (b - a):
        b_{K+1} = b_{K+2} = 0,
        b_k = c_k v + 2 Ahat b_{k+1} - b_{k+2},   k = K, ..., 1,
        q(A) v = c_0 v + Ahat b_1 - b_2.
    The first step has b_{K+1} = 0, so the recurrence costs K products with A.
    Returns (q(A) v, number of products with A).
    """
    K = len(c) - 1
    s = 2.0 / (b - a)
    t = -(a + b) / (b - a)
    nmv = 0

    def Ahat(x):
        nonlocal nmv
        nmv += 1
        return s * apply_A(x) + t * x

    v = np.asarray(v)
    if K == 0:
        return c[0] * v, 0
    b2 = np.zeros_like(v)
    b1 = c[K] * v
    for k in range(K - 1, 0, -1):
        b1, b2 = c[k] * v + 2.0 * Ahat(b1) - b2, b1
    return c[0] * v + Ahat(b1) - b2, nmv


def chebyshev(a, b, degree, check_points=10000, check_interval=None):
    """Sec. 5.1 polynomial for z^{-1/2} on [a, b] with the positivity check.

    Degree 0 is the plain method (q == 1).  q must be positive on the
    interval that holds spec(A) (then spec(q(A)) lies in the right
    half-plane and the principal branch is obtained, Sec. 3).  That interval
    is [a, b] unless check_interval is given (a polynomial built on a
    narrower interval than the spectrum).  q is tested on check_points
    equispaced points plus the interpolation nodes; a BranchError is raised
    if it is not positive there.
    """
    if degree == 0:
        return one()
    if not (0.0 < a < b):
        raise ValueError("need 0 < a < b")
    c = chebyshev_coefficients(inv_sqrt, a, b, degree)
    d = degree + 1
    t = math.pi * (np.arange(d) + 0.5) / d
    lo, hi = check_interval if check_interval is not None else (a, b)
    pts = np.concatenate([np.linspace(lo, hi, check_points),
                          0.5 * (a + b) + 0.5 * (b - a) * np.cos(t)])
    if np.min(clenshaw_scalar(c, a, b, pts)) <= 0.0:
        raise BranchError("Chebyshev q is not positive on [a, b]")
    return Poly(kind="cheb", degree=degree, a=float(a), b=float(b), c=c)


# --------------------------------------------------------------------------
# Sec. 5.2: interpolation at Ritz values, Newton form on Leja points
# --------------------------------------------------------------------------
def arnoldi_hessenberg(apply_A, start, steps, with_next=False):
    """H_d from `steps` Arnoldi steps on A (classical Gram-Schmidt, twice).

    Returns the square Hessenberg H (j x j) where j <= steps is the number of
    steps completed before a (lucky) breakdown, declared with the same rule as
    in the Krylov solver (h_{j+1,j} <= 1e-12 times the largest column norm).
    With with_next, returns (H, h_{j+1,j}) (0 after a breakdown).
    """
    v = np.asarray(start)
    dt = np.result_type(v, 1.0)
    n = v.size
    V = np.zeros((n, steps + 1), dtype=dt)
    H = np.zeros((steps + 1, steps), dtype=dt)
    V[:, 0] = v / np.linalg.norm(v)
    colmax = 0.0
    for j in range(steps):
        w = apply_A(V[:, j]).astype(dt)
        h = np.zeros(j + 1, dtype=dt)
        for _ in range(2):
            g = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ g
            h += g
        H[:j + 1, j] = h
        hn = np.linalg.norm(w)
        H[j + 1, j] = hn
        colmax = max(colmax, math.sqrt(np.linalg.norm(h) ** 2 + hn ** 2))
        if hn <= 1e-12 * colmax:
            return (H[:j + 1, :j + 1], 0.0) if with_next else H[:j + 1, :j + 1]
        V[:, j + 1] = w / hn
    return (H[:steps, :steps], float(np.real(H[steps, steps - 1]))) if with_next else H[:steps, :steps]


def harmonic_ritz_values(H, h_next):
    """Harmonic Ritz values (Sec. 5.2): eigenvalues of
    H_d + h_{d+1,d}^2 H_d^{-*} e_d e_d^*."""
    d = H.shape[0]
    ed = np.zeros(d)
    ed[-1] = 1.0
    y = np.linalg.solve(np.asarray(H).conj().T, ed)
    Ht = np.array(H, dtype=np.result_type(H, y, 1.0), copy=True)
    Ht[:, -1] += h_next ** 2 * y
    return np.linalg.eigvals(Ht)


def leja_order(theta, pair_conjugates):
    """Leja ordering of the nodes.

    The first node has the largest modulus (ties: larger real part, then
    non-negative imaginary part first); each following node maximises the
    product of distances to the nodes already chosen (compared through the sum
    of logarithms).  With pair_conjugates (real operators, whose Ritz values
    come in conjugate pairs) a node with nonzero imaginary part is followed
    directly by its conjugate.
    """
    th = list(np.asarray(theta, dtype=np.complex128))
    order = []
    key0 = max(range(len(th)), key=lambda i: (abs(th[i]), th[i].real, th[i].imag >= 0))
    order.append(th.pop(key0))

    def take_partner():
        z = order[-1]
        if pair_conjugates and z.imag != 0.0 and th:
            j = min(range(len(th)), key=lambda i: abs(th[i] - z.conjugate()))
            if abs(th[j] - z.conjugate()) <= 1e-10 * max(1.0, abs(z)):
                order.append(th.pop(j))

    take_partner()
    while th:
        def score(i):
            return sum(math.log(abs(th[i] - s)) if th[i] != s else -math.inf
                       for s in order)
        i = max(range(len(th)), key=lambda i: (score(i), th[i].imag >= 0))
        order.append(th.pop(i))
        take_partner()
    return np.array(order)


def capacity(theta):
    """rho = (prod_{i<d-1} |theta_{d-1} - theta_i|)^{1/(d-1)} of Leja nodes."""
    d = len(theta)
    if d < 2:
        return 1.0
    logs = [math.log(abs(theta[-1] - theta[i])) for i in range(d - 1)]
    return math.exp(sum(logs) / (d - 1))


def newton_coefficients(f, theta, rho):
    """Scaled Newton divided differences eta_j = f[theta_0..theta_j] * rho^j.

    The table recursion f[t_i..t_{i+j}] = (f[t_{i+1}..] - f[t_i..]) / (t_{i+j} - t_i)
    is carried out with every denominator divided by rho, which gives the
    coefficients of q in the scaled Newton basis prod_{i<j} (z - theta_i)/rho.
    """
    th = np.asarray(theta, dtype=np.complex128)
    dd = np.array(f(th), dtype=np.complex128)
    d = len(th)
    for j in range(1, d):
        for i in range(d - 1, j - 1, -1):
            dd[i] = (dd[i] - dd[i - 1]) / ((th[i] - th[i - j]) / rho)
    return dd


def horner_scalar(theta, eta, rho, z):
    z = np.asarray(z, dtype=np.complex128)
    r = np.full_like(z, eta[-1])
    for j in range(len(eta) - 2, -1, -1):
        r = (z - theta[j]) / rho * r + eta[j]
    return r


def horner_apply(apply_A, theta, eta, rho, v):
    """q(A) v for q in scaled Newton form by the Horner-type recurrence:

        r = eta_K v;   r = (A - theta_j I) r / rho + eta_j v,  j = K-1, ..., 0.

    Carried out in complex arithmetic.  Returns (q(A) v, products with A).
    """
    v = np.asarray(v).astype(np.complex128)
    K = len(eta) - 1
    r = eta[K] * v
    nmv = 0
    for j in range(K - 1, -1, -1):
        r = (apply_A(r) - theta[j] * r) / rho + eta[j] * v
        nmv += 1
    return r, nmv


def ritz(apply_A, start, degree, real_operator, harmonic=False):
    """Sec. 5.2 polynomial of the given degree from Ritz values of A.

    d = degree + 1 Arnoldi steps from `start`; the Ritz values are the
    eigenvalues of H_d (harmonic: of H_d + h_{d+1,d}^2 H_d^{-*} e_d e_d^*).  If
    Arnoldi breaks down after j < d steps, the j Ritz values found are used
    (degree j - 1).  Raises BranchError if a Ritz value has Re <= 0.
    """
    if degree == 0:
        return one()
    H, h_next = arnoldi_hessenberg(apply_A, start, degree + 1, with_next=True)
    theta = harmonic_ritz_values(H, h_next) if harmonic else np.linalg.eigvals(H)
    if np.min(theta.real) <= 0.0:
        raise BranchError("a Ritz value lies outside the open right half-plane")
    if real_operator:
        # Ritz values of a real H come in exact conjugate pairs
        theta = np.where(np.abs(theta.imag) <= 1e-14 * np.abs(theta), theta.real, theta)
    th = leja_order(theta, pair_conjugates=real_operator)
    rho = capacity(th)
    eta = newton_coefficients(inv_sqrt, th, rho)
    return Poly(kind="newton", degree=len(th) - 1, theta=th, eta=eta, rho=rho,
                real_operator=real_operator)


# --------------------------------------------------------------------------
# Sec. 5.3: least-squares polynomial on a contour around the Ritz values
# --------------------------------------------------------------------------
def convex_hull(points):
    """Vertices of the convex hull of complex points, counter-clockwise
    (Andrew's monotone chain; collinear points dropped)."""
    pts = sorted(set((float(z.real), float(z.imag)) for z in np.asarray(points).ravel()))
    if len(pts) <= 2:
        return np.array([complex(x, y) for x, y in pts])

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    hull = lower[:-1] + upper[:-1]
    return np.array([complex(x, y) for x, y in hull])


def ls_contour(theta, r_min, step, symmetric):
    """Discretized contour Gamma around the Ritz values theta (Sec. 5.3, and
    the choices of Sec. 6, Example 3).

    Gamma is the boundary of the convex hull of theta with the part closer to
    0 than r_min replaced by the arc |z| = r_min (the boundary of
    hull minus the open disk of radius r_min).  It is discretized by points
    at equal arc-length spacing of at most `step`, starting at the first hull
    vertex.  symmetric=True (real operators): the returned set is the points
    together with their complex conjugates, so that the least-squares
    polynomial has real coefficients.

    A hull of collinear points (real Ritz values) is a segment, traversed
    forth and back.
    """
    hull = convex_hull(theta)
    if len(hull) < 2:
        raise ValueError("the contour needs at least two distinct Ritz values")
    if np.min(hull.real) <= 0.0:
        raise BranchError("a Ritz value lies outside the open right half-plane")
    # pieces of the boundary: ("seg", p, q) and ("arc", angle0, span) with
    # span < 0 meaning clockwise
    pieces = []
    entry = None
    nv = len(hull)
    for i in range(nv):
        p, q = hull[i], hull[(i + 1) % nv]
        d = q - p
        # |p + t d|^2 = r^2  ->  |d|^2 t^2 + 2 Re(conj(p) d) t + |p|^2 - r^2 = 0
        A2 = abs(d) ** 2
        B2 = 2.0 * (p.conjugate() * d).real
        C2 = abs(p) ** 2 - r_min ** 2
        disc = B2 * B2 - 4.0 * A2 * C2
        cuts = [0.0, 1.0]
        if disc > 0.0:
            sq = math.sqrt(disc)
            for t in ((-B2 - sq) / (2.0 * A2), (-B2 + sq) / (2.0 * A2)):
                if 0.0 < t < 1.0:
                    cuts.append(t)
        cuts.sort()
        for t0, t1 in zip(cuts[:-1], cuts[1:]):
            a, b = p + t0 * d, p + t1 * d
            mid = p + 0.5 * (t0 + t1) * d
            if abs(mid) >= r_min:
                if entry is not None:
                    pieces.append(("arc_to", entry, a))
                    entry = None
                pieces.append(("seg", a, b))
            elif entry is None:
                entry = a
    if entry is not None:
        # the walk ended inside the disk: close with the arc to the first kept point
        first = next(pc for pc in pieces if pc[0] == "seg")[1] if pieces else None
        if first is None:
            raise ValueError("the whole hull lies within r_min of the origin")
        pieces.append(("arc_to", entry, first))
    if not any(pc[0] == "seg" for pc in pieces):
        raise ValueError("the whole hull lies within r_min of the origin")
    # arcs: from the entry point to the exit point, clockwise about 0 (the
    # region lies outside the disk, to the left of the walk)
    geo = []
    for pc in pieces:
        if pc[0] == "seg":
            geo.append(("seg", pc[1], pc[2], abs(pc[2] - pc[1])))
        else:
            a0 = math.atan2(pc[1].imag, pc[1].real)
            a1 = math.atan2(pc[2].imag, pc[2].real)
            span = (a0 - a1) % (2.0 * math.pi)
            if span > math.pi:  # rounding around a zero-length arc
                span = 0.0
            geo.append(("arc", a0, -span, r_min * span))
    total = sum(g[3] for g in geo)
    N = max(int(math.ceil(total / step)), 2)
    h = total / N
    pts = []
    s0 = 0.0   # arc length at the start of the current piece
    k = 0
    for g in geo:
        while k < N and k * h < s0 + g[3]:
            t = (k * h - s0) / g[3] if g[3] > 0 else 0.0
            if g[0] == "seg":
                pts.append(g[1] + t * (g[2] - g[1]))
            else:
                ang = g[1] + t * g[2]
                pts.append(r_min * complex(math.cos(ang), math.sin(ang)))
            k += 1
        s0 += g[3]
    pts = np.array(pts)
    if symmetric:
        pts = np.concatenate([pts, pts.conj()])
    return pts


def ls_polynomial(points, degree, f=inv_sqrt, real_operator=False):
    """Least-squares polynomial of the given degree for f on the points
    (Sec. 5.3).

    Arnoldi on diag(z_1..z_N) from [1..1]/sqrt(N) (classical Gram-Schmidt,
    twice) gives the orthonormal basis polynomials p_0..p_{d-1} as the
    vectors P_d and their recurrence hls; alpha = P_d^H f(z).  Raises
    BranchError unless Re q(z_i) > 0 at every point (the check of Sec. 5.3).
    real_operator: the point set is conjugate-symmetric, so hls and alpha are
    real up to rounding; they are stored real.
    """
    z = np.asarray(points, dtype=np.complex128)
    N = z.size
    d = degree + 1
    if d > N:
        raise ValueError("need more points than coefficients")
    P = np.zeros((N, d), dtype=np.complex128)
    Hs = np.zeros((d, max(d - 1, 0)), dtype=np.complex128)
    P[:, 0] = 1.0 / math.sqrt(N)
    for j in range(d - 1):
        w = z * P[:, j]
        h = np.zeros(j + 1, dtype=np.complex128)
        for _ in range(2):
            g = P[:, :j + 1].conj().T @ w
            w = w - P[:, :j + 1] @ g
            h += g
        Hs[:j + 1, j] = h
        Hs[j + 1, j] = np.linalg.norm(w)
        P[:, j + 1] = w / Hs[j + 1, j]
    alpha = P.conj().T @ f(z)
    qz = P @ alpha
    if np.min(qz.real) <= 0.0:
        raise BranchError("Re q(z) <= 0 at a contour point")
    if real_operator:
        scale = max(np.max(np.abs(Hs)) if Hs.size else 0.0, np.max(np.abs(alpha)))
        if max(np.max(np.abs(Hs.imag)) if Hs.size else 0.0,
               np.max(np.abs(alpha.imag))) > 1e-10 * scale:
            raise ValueError("the point set is not conjugate-symmetric")
        Hs, alpha = Hs.real.copy(), alpha.real.copy()
    return Poly(kind="ls", degree=degree, hls=Hs, alpha=alpha, npts=N,
                real_operator=real_operator)


def ls_scalar(hls, alpha, npts, z):
    """q(z) = sum_j alpha_j p_j(z) with p_0 = N^{-1/2} and
    p_k = (z p_{k-1} - sum_{i<k} h_{i,k-1} p_i) / h_{k,k-1}."""
    z = np.asarray(z)
    p = [np.full(z.shape, 1.0 / math.sqrt(npts), dtype=np.result_type(z, hls, 1.0))]
    for k in range(1, len(alpha)):
        w = z * p[k - 1]
        for i in range(k):
            w = w - hls[i, k - 1] * p[i]
        p.append(w / hls[k, k - 1])
    return sum(a * pk for a, pk in zip(alpha, p))


def ls_apply(apply_A, hls, alpha, npts, v):
    """q(A) v by the same recurrence with A for z (the Arnoldi-like evaluation
    of Sec. 5.3): d - 1 products with A, O(d^2) vector updates, no inner
    products.  Returns (q(A) v, number of products with A)."""
    v = np.asarray(v)
    dt = np.result_type(v, hls, alpha, 1.0)
    W = [np.asarray(v, dtype=dt) / math.sqrt(npts)]
    for k in range(1, len(alpha)):
        w = np.asarray(apply_A(W[k - 1]), dtype=dt)
        for i in range(k):
            w = w - hls[i, k - 1] * W[i]
        W.append(w / hls[k, k - 1])
    y = sum(a * wk for a, wk in zip(alpha, W))
    return y, len(alpha) - 1


def least_squares(apply_A, start, degree, real_operator, ritz_steps=60, r_min=0.1,
                  step=0.005):
    """Sec. 5.3 polynomial as used in Sec. 6, Example 3: `ritz_steps` Arnoldi
    steps on A give Ritz values, the contour around them (ls_contour) is
    discretized, and q is the least-squares fit of z^{-1/2} there."""
    if degree == 0:
        return one()
    H = arnoldi_hessenberg(apply_A, start, ritz_steps)
    theta = np.linalg.eigvals(H)
    if np.min(theta.real) <= 0.0:
        raise BranchError("a Ritz value lies outside the open right half-plane")
    pts = ls_contour(theta, r_min, step, symmetric=real_operator)
    return ls_polynomial(pts, degree, real_operator=real_operator)
