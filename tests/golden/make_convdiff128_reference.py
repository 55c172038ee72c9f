"""Write convdiff128_reference.json: oracle results for the 3D
convection-diffusion workload at 128^3 (Pe = 50, b ~ N(0,1) seed 0), sampled.

The stand-in for the non-Hermitian operator of Sec. 6, Example 3: the error of
a result is measured against a reference solution (as in Example 1).  The
references here are the oracle's own solves (Algorithm 1, Chebyshev degree 32,
tol 1e-12), for A^{-1/2} b and A^{1/2} b; a full vector (2^21 doubles) is too
large to keep, so the file holds the values at 2048 seeded indices and the
2-norm of each reference.  Only the oracle and the input generator are used.

    python tests/golden/make_convdiff128_reference.py     (a few minutes)
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import krylov as kr, operators as ops, polynomials as pl  # noqa: E402

N, PE, DEGREE, TOL, SAMPLES, SAMPLE_SEED = 128, 50.0, 32, 1e-12, 2048, 2024


def sample_indices(n):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(n, SAMPLES, replace=False))


def main():
    dims = (N, N, N)
    coeffs = wl.convdiff_stencil(N, PE)
    b = wl.rhs(N ** 3, seed=0)
    a, bb = ops.stencil_interval(coeffs, dims)
    q = pl.chebyshev(a, bb, DEGREE)
    idx = sample_indices(N ** 3)
    out = {
        "what": "oracle f(A)b for the 128^3 convection-diffusion operator (Pe 50), Algorithm 1 "
                "with the Chebyshev interpolant of degree 32 on the exact interval, tol 1e-12; "
                "values at sampled indices and the 2-norm",
        "N": N, "Pe": PE, "rhs_seed": 0, "degree": DEGREE, "tol": TOL,
        "sample_seed": SAMPLE_SEED, "indices": idx.tolist(),
    }
    for kind in ("invsqrt", "sqrt"):
        t0 = time.time()
        r = kr.fAb(lambda v: ops.stencil_apply(coeffs, dims, v), b, q, kind, m_max=60, tol=TOL)
        assert r.converged, kind
        out[kind] = {"iters": r.iters, "est": r.est, "norm2": float(np.linalg.norm(r.x)),
                     "values": [float(v) for v in r.x[idx]]}
        print(f"{kind}: m = {r.iters}, est = {r.est:.2e}, {time.time() - t0:.1f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "convdiff128_reference.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
        f.write("\n")


if __name__ == "__main__":
    main()
