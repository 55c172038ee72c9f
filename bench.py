"""Benchmark: f(A)b solves/s on one MI355X, polynomially preconditioned vs plain.

Workload (the metric's configuration): 3D convection-diffusion, 7-point
first-order upwind stencil on a 128^3 grid (n = 2,097,152), Pe = 50 with
convection direction (1, 0.5, 0.25), real FP64; b ~ N(0, 1) (seed 0);
f = A^{-1/2}; Chebyshev polynomial of degree 16 on the exact spectral interval;
stopping tolerance 1e-8 on the difference-of-iterates estimate.

A step is one fa_apply solve (setup of the operator and polynomial excluded,
inputs resident in HBM).  Printed as one JSON line with a roofline object for
the dominant kernel (the stencil chain launch that evaluates four Clenshaw
terms, timed by its own dispatch events in every tenth timed solve) and the
oracle leg: the CPU oracle's reference solve (degree 32, tol 1e-12), against
which every GPU result's true error is taken, and the median of 3 timed
oracle solves of the headline configuration.  Extra fields: every degree of
the configuration (0 = plain Arnoldi, 4, 16, 32) for A^{-1/2} b and A^{1/2} b,
one launch per term, mixed precision, the chain at 256^3 (beyond the 256 MB
Infinity Cache), the 2D Poisson 32 x 32 configuration, Table 1's workload
(the 3D Laplacian on 100^3, right preconditioning, one and two passes at the
printed iteration counts, true errors against the closed form), the Wilson
16^4 leg, Example 2's shape ((Q^2)^{-1/2} b, Q = Gamma_5 D at m_w = -1.4,
mu = 0.3 on 64 x 32^3, Ritz d = 8..64 and the plain method), the CSR legs, the batched leg (64 right-hand sides) and the serving workload: Poisson
arrivals of a request mix (2D Laplacian 256^2, convection-diffusion 64^3 /
96^3 / 128^3, Wilson 16^4; f in {sqrt, invsqrt}, tol in {1e-6, 1e-10}) through
the library's request loop, with solves/s and p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "f(A)b solves/s at rel err 1e-8, poly-precond vs plain Arnoldi; SpMV HBM GB/s"
HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the dominant kernel (the multi-term middle launch
# st7_multi<..., NT, 64, 8, true, true> at 128^3 with the LDS pitch padded
# by 2 and paired slabs, keyed by NT): FETCH_SIZE x 2 + WRITE_SIZE, from the rocprofv3 counter
# runs in profiles/st7_multi_convdiff128_deg16_hbm_counters.md (FETCH_SIZE
# counts gfx950's 128-byte L2 read requests at 64 bytes: the 2 GiB copy and
# the raw request-size counters there both give the factor 2); only the
# current build's kernels are listed (others report null)
MULTI_TRAFFIC_BYTES = {4: (87254 + 32768) * 1024}
# the same at the larger grid of the chain leg beyond the 256 MB Infinity
# Cache, keyed by (N, NT), from profiles/st7_multi_convdiff256_deg16_hbm_counters.md
BIG_TRAFFIC_BYTES = {(256, 4): (276520 * 2 + 262144) * 1024}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--degree", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-Arnoldi leg")
    ap.add_argument("--big-N", type=int, default=256,
                    help="grid of the chain leg beyond the Infinity Cache (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--chain-only", type=int, default=0, metavar="R",
                    help="only run R applications of q(A) (for hardware counters) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB (counter calibration) and exit")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (block) leg")
    ap.add_argument("--batch-only", action="store_true", help="only run the batched leg")
    ap.add_argument("--csr-only", action="store_true", help="only run the CSR SpMV leg")
    ap.add_argument("--wilson-only", action="store_true", help="only run the Wilson leg")
    ap.add_argument("--serve-only", action="store_true", help="only run the serving leg")
    ap.add_argument("--poisson-only", action="store_true",
                    help="only run the 2D Poisson 32 x 32 leg (no oracle)")
    ap.add_argument("--overlap-only", action="store_true",
                    help="only run Example 2's 64 x 32^3 overlap leg")
    ap.add_argument("--table1-only", action="store_true",
                    help="only run Table 1's 100^3 Laplacian rows (no closed-form errors)")
    ap.add_argument("--plain-only", action="store_true",
                    help="only run two plain Arnoldi solves each on the 128^3 "
                         "convection-diffusion and the 16^4 Wilson operators (Gram-Schmidt "
                         "sweeps over bases of up to 448 and 192 vectors)")
    ap.add_argument("--qps", type=float, default=2000.0, help="serving arrival rate")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-pool-gb", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(one GPU's share of a row-sharded operator is what it measures)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2401_06684_amd as fa
    import workloads as wl

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        # a plain copy kernel of known size: 2^28 doubles (2 GiB) read + written
        src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 copies of 2 GiB done")
        return
    if args.wilson_only:
        print(json.dumps({"wilson4d_16": wilson_leg(fa, torch, wl, dev)}), flush=True)
        return
    if args.csr_only:
        print(json.dumps({"csr_spmv": csr_leg(fa, torch, wl, dev)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched": batched_leg(fa, torch, wl, dev)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": serving_leg(args, fa, torch, wl, dev)}), flush=True)
        return
    if args.poisson_only:
        print(json.dumps({"poisson2d_32": poisson_leg(fa, torch, wl, dev, None)}), flush=True)
        return
    if args.overlap_only:
        print(json.dumps({"overlap_64x32cubed": overlap_leg(fa, torch, wl, dev)}), flush=True)
        return
    if args.table1_only:
        print(json.dumps({"table1_laplace3d_100": table1_leg(fa, torch, wl, dev, None)}),
              flush=True)
        return
    if args.plain_only:
        print(json.dumps({"plain": plain_leg(fa, torch, wl, dev)}), flush=True)
        return
    N = args.N
    dims = (N, N, N)
    pe = 50.0
    coeffs = wl.convdiff_stencil(N, pe)
    b = torch.from_numpy(wl.rhs(N ** 3, seed=0)).to(dev)
    tol = 1e-8

    def make(degree):
        op = fa.Stencil7(dims, coeffs, device=dev)
        op.poly_setup(degree, "cheb")
        return op

    if args.chain_only:
        op = make(args.degree)
        y = torch.empty_like(b)
        for _ in range(args.chain_only):
            op.poly_apply(b, out=y)
        torch.cuda.synchronize()
        log(f"chain only: {args.chain_only} x q(A) b at degree {args.degree} done")
        return

    # ---- the oracle: references for the true errors, and the CPU baseline ---
    # (run first, on the host; every GPU result below is compared with it)
    orc = None
    if not args.no_cpu:
        orc = cpu_baseline(coeffs, dims, args.degree, tol)
        x_ref = torch.from_numpy(orc.pop("x_ref_invsqrt")).to(dev)
        x_ref_sqrt = torch.from_numpy(orc.pop("x_ref_sqrt")).to(dev)
        ref_name = "oracle solve (degree 32, tol 1e-12, same b)"
    else:
        # no oracle requested: a GPU reference, named as such in the output
        op_ref = make(32)
        x_ref, _ = op_ref.apply(b, m_max=100, tol=1e-12)
        x_ref = x_ref.clone()
        x_ref_sqrt = op_ref.op_apply(x_ref)
        op_ref.release_workspace()
        del op_ref
        ref_name = "GPU solve (degree 32, tol 1e-12); run without the oracle leg"

    def rel_err(x, kind="invsqrt"):
        r = x_ref if kind == "invsqrt" else x_ref_sqrt
        return float(torch.linalg.vector_norm(x - r) / torch.linalg.vector_norm(r))

    def timed(op, steps, warmup, kind="invsqrt", m_max=200, profile=False, fuse=True,
              mixed=False, tol_=None, profile_every=1):
        t_ = tol if tol_ is None else tol_
        x = torch.empty_like(b)
        for _ in range(warmup):
            op.apply(b, kind=kind, m_max=m_max, tol=t_, out=x, fuse=fuse, mixed=mixed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats = []
        for i in range(steps):
            _, st = op.apply(b, kind=kind, m_max=m_max, tol=t_, out=x,
                             profile=profile and i % profile_every == 0, fuse=fuse, mixed=mixed)
            stats.append(st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return x, dt, stats

    def launch_stats(stats):
        """Mean duration, algorithmic bytes and terms of the timed chain
        launches (only the profiled solves carry them)."""
        prof = [s_ for s_ in stats if s_["n_chain"] > 0]
        n_ = sum(s_["n_chain"] for s_ in prof)
        ms_ = sum(s_["ms_chain"] for s_ in prof)
        by_ = sum(s_["chain_bytes"] * s_["n_chain"] for s_ in prof) / max(n_, 1)
        te_ = sum(s_["n_chain_terms"] for s_ in prof) / max(n_, 1)
        avg_ = ms_ / max(n_, 1)
        return {"launches": n_, "avg_ms": avg_, "bytes": by_, "terms": te_,
                "GBs": by_ / (avg_ * 1e-3) / 1e9 if n_ else 0.0}

    # ---- headline: degree-K polynomially preconditioned solve ------------
    K = args.degree
    log(f"headline: degree {K}, {args.warmup} warmup + {args.steps} timed solves")
    op = make(K)
    # the dominant kernel's launches are timed by their own dispatch (a start
    # and an end event per launch) in every tenth timed solve: each timed
    # launch costs the solve about 5 us, and two solves in twenty already give
    # 172 launches
    x, dt, stats = timed(op, args.steps, args.warmup, profile=True, profile_every=10)
    err = rel_err(x)
    value = args.steps / dt
    st0 = stats[-1]
    ls = launch_stats(stats)
    n_chain, avg_ms, bytes_avg, terms = ls["launches"], ls["avg_ms"], ls["bytes"], ls["terms"]
    traffic = MULTI_TRAFFIC_BYTES.get(int(round(terms)))  # None: not measured for this kernel
    # algorithmic bytes of one timed launch as designed: x, v, b_(k+2) read
    # once and the two terms the next launch needs written once (5 vectors,
    # bytes_avg from the solve's statistics)
    achieved = ls["GBs"]
    log(f"degree {K}: {value:.2f} solves/s, m = {st0['iters']}, err vs {ref_name} = {err:.2e}, "
        f"chain launch {avg_ms * 1e3:.1f} us ({terms:.0f} terms), {achieved:.0f} GB/s of the "
        f"launch's 5 vectors")
    op.release_workspace()
    del op

    extra = {"iters": st0["iters"], "mvms": st0["mvms"], "inner_products": st0["inner_products"],
             "rel_err_vs_ref": err, "reference": ref_name, "est": st0["est_rel_change"],
             "ms_host_fH_per_solve": st0["ms_host_fH"],
             "chain_per_term_accounting": {
                 "note": "each of the launch's terms counted at the 4 vectors a one-term launch "
                         "moves; the fused launch keeps most of them on chip, so this rate is "
                         "not an HBM rate",
                 "bytes_per_launch": terms * 4 * (N ** 3) * 8,
                 "GBs": terms * 4 * (N ** 3) * 8 / (avg_ms * 1e-3) / 1e9 if n_chain else 0.0}}

    # ---- the same chain beyond the 256 MB Infinity Cache: 256^3 -----------
    if args.big_N:
        Nb = args.big_N
        log(f"chain at {Nb}^3 (one launch's working set {5 * 8 * Nb ** 3 / 1e6:.0f} MB)")
        ob = fa.Stencil7((Nb, Nb, Nb), wl.convdiff_stencil(Nb, pe), device=dev)
        ob.poly_setup(K, "cheb")
        bb_ = torch.from_numpy(wl.rhs(Nb ** 3, seed=0)).to(dev)
        ob.apply(bb_, m_max=200, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sb = [ob.apply(bb_, m_max=200, tol=tol, profile=True)[1] for _ in range(2)]
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / 2
        lb = launch_stats(sb)
        extra["convdiff3d_%d" % Nb] = {
            "n": Nb ** 3, "solves_per_s": 1.0 / dtb, "iters": sb[-1]["iters"],
            "chain_launch_us": lb["avg_ms"] * 1e3, "chain_bytes_per_launch": lb["bytes"],
            "chain_GBs": lb["GBs"], "chain_frac": lb["GBs"] / HBM_PEAK_GBS,
            "chain_traffic_bytes": BIG_TRAFFIC_BYTES.get((Nb, int(round(lb["terms"])))),
            "launches_timed": lb["launches"]}
        log(f"{Nb}^3: {1.0 / dtb:.2f} solves/s, m = {sb[-1]['iters']}, chain launch "
            f"{lb['avg_ms'] * 1e3:.1f} us, {lb['GBs']:.0f} GB/s")
        ob.release_workspace()
        del ob, bb_

    # ---- the same solve with one launch per recurrence term ---------------
    o = make(K)
    xu, dtu, stu = timed(o, 5, 1, profile=True, fuse=False)
    lu = launch_stats(stu)
    extra["single_term_launches"] = {
        "solves_per_s": 5 / dtu, "rel_err": rel_err(xu), "kernel": "st7_chain<true,true>",
        "avg_launch_us": lu["avg_ms"] * 1e3, "bytes_per_launch": lu["bytes"],
        "achieved_GBs": lu["GBs"]}
    log(f"single-term launches: {5 / dtu:.2f} solves/s, chain launch {lu['avg_ms'] * 1e3:.1f} us")
    o.release_workspace()
    del o

    # ---- mixed precision: the chain in FP32 (tolerance 1e-7) ---------------
    o = make(K)
    xm, dtm, stm = timed(o, 5, 1, profile=True, mixed=True, tol_=1e-7, profile_every=5)
    lm = launch_stats(stm)
    extra["mixed_fp32_chain"] = {
        "solves_per_s": 5 / dtm, "iters": stm[-1]["iters"], "rel_err": rel_err(xm),
        "tol": 1e-7, "kernel": f"st7_multi<float, {lm['terms']:.0f} terms>",
        "avg_launch_us": lm["avg_ms"] * 1e3, "bytes_per_launch": lm["bytes"],
        "achieved_GBs": lm["GBs"], "frac": lm["GBs"] / HBM_PEAK_GBS,
        "launches_timed": lm["launches"]}
    log(f"mixed precision: {5 / dtm:.2f} solves/s, m = {stm[-1]['iters']}, "
        f"err {rel_err(xm):.2e}, chain launch {lm['avg_ms'] * 1e3:.1f} us, {lm['GBs']:.0f} GB/s")
    o.release_workspace()
    del o

    # ---- every degree of the configuration, both functions -----------------
    others = {}
    for deg in (0, 4, 16, 32):
        if deg == 0 and args.no_plain:
            continue
        for kind in ("invsqrt", "sqrt"):
            if deg == K and kind == "invsqrt":
                continue  # the headline
            o = make(deg)
            reps = 1 if deg == 0 else 3
            m_max = 1000 if deg == 0 else 200
            xo, dto, sto = timed(o, reps, 1 if deg else 0, kind=kind, m_max=m_max)
            e = rel_err(xo, kind)
            others[f"{kind}_deg{deg}"] = {"solves_per_s": reps / dto, "iters": sto[-1]["iters"],
                                          "mvms": sto[-1]["mvms"], "rel_err": e,
                                          "ms_host_fH": sto[-1]["ms_host_fH"]}
            log(f"{kind} degree {deg}: {reps / dto:.3f} solves/s, m = {sto[-1]['iters']}, "
                f"err {e:.2e}")
            o.release_workspace()
            del o
    extra["every_degree"] = others
    if "invsqrt_deg0" in others:
        p0 = others["invsqrt_deg0"]
        extra["plain"] = {"solves_per_s": p0["solves_per_s"], "iters": p0["iters"],
                          "rel_err": p0["rel_err"], "ms_host_fH": p0["ms_host_fH"],
                          "speedup_poly_over_plain": value / p0["solves_per_s"]}

    # ---- 2D Poisson 32 x 32 (CSR, Lanczos), the small configuration ---------
    extra["poisson2d_32"] = poisson_leg(fa, torch, wl, dev, orc)

    # ---- Table 1's workload: the 3D Laplacian on 100^3 ------------------------
    extra["table1_laplace3d_100"] = table1_leg(fa, torch, wl, dev, orc)

    # ---- Wilson 16^4 (the lattice operator) --------------------------------
    extra["wilson4d_16"] = wilson_leg(fa, torch, wl, dev)

    # ---- Example 2's shape: (Q^2)^{-1/2} b on 64 x 32^3 ---------------------
    extra["overlap_64x32cubed"] = overlap_leg(fa, torch, wl, dev)

    # ---- CSR SpMV (the operator of the directed-graph example) ------------
    extra["csr_spmv"] = csr_leg(fa, torch, wl, dev)

    # ---- batched: 64 right-hand sides as one block Arnoldi ------------------
    if not args.no_batch:
        extra["batched"] = batched_leg(fa, torch, wl, dev)

    # ---- serving: Poisson arrivals of a request mix ------------------------
    if not args.no_serve:
        extra["serving"] = serving_leg(args, fa, torch, wl, dev)

    cpu = None
    if orc is not None:
        orc.pop("poisson2d_32_ref", None)
        orc.pop("table1_ref", None)
        cpu = orc

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"convdiff3d_{N}^3 Pe=50 invsqrt chebyshev degree {K} tol 1e-8",
                   "n": N ** 3, "degree": K, "tol": tol, "kind": "invsqrt",
                   "orthogonalization": "CGS2", "preconditioning": "left"},
        "roofline": {"bound": "hbm",
                     "kernel": f"st7_multi<double, {terms:.0f} terms> ({terms:.0f} Clenshaw "
                               "terms per launch)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_avg,
                     "algorithmic_unit": f"one launch = {terms:.0f} Clenshaw middle terms: x, v, "
                                         "b_k+2 read and the last two terms written (5 vectors)",
                     "traffic_frac": (traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None),
                     "avg_launch_us": avg_ms * 1e3, "launches_timed": n_chain,
                     "working_set_MB": bytes_avg / 1e6},
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


def plain_leg(fa, torch, wl, dev):
    """Two plain Arnoldi solves (degree 0, tol 1e-8) each on the 128^3
    convection-diffusion operator (m = 448, real) and the 16^4 Wilson
    operator (m = 192, complex): the delayed-CGS2 sweeps at every basis size
    up to those (the first solve of each warms up)."""
    out = {}
    N = 128
    op = fa.Stencil7((N, N, N), wl.convdiff_stencil(N, 50.0), device=dev)
    op.poly_setup(0)
    b = torch.from_numpy(wl.rhs(N ** 3, seed=0)).to(dev)
    for _ in range(2):
        _, st = op.apply(b, m_max=1000, tol=1e-8)
    out["convdiff3d_128"] = {"iters": st["iters"], "ms": st["ms_total"]}
    op.release_workspace()
    del op, b
    op = fa.Wilson(wl.su3_links(16, eps=0.3, seed=1), 0.05, device=dev)
    op.poly_setup(0)
    b = torch.from_numpy(wl.rhs(op.n, seed=0, complex_=True)).to(dev)
    for _ in range(2):
        _, st = op.apply(b, m_max=1000, tol=1e-8)
    out["wilson4d_16"] = {"iters": st["iters"], "ms": st["ms_total"]}
    op.release_workspace()
    for k, v in out.items():
        log(f"plain {k}: m = {v['iters']}, {v['ms']:.1f} ms")
    return out


def poisson_leg(fa, torch, wl, dev, orc):
    """2D Poisson 32 x 32 (5-point, CSR int32, Hermitian: Lanczos), b ~ N(0, 1)
    seed 0, f = A^{-1/2}, Chebyshev degrees 0 and 8 on the exact interval,
    tol 1e-10, m_max 200.  The whole problem is under 100 KB (cache-resident,
    launch-bound): microseconds per solve; errors against the oracle's
    tol-1e-12 solve when the oracle leg ran."""
    import numpy as np
    N = 32
    coeffs = wl.laplace_stencil(2)
    rp, ci, va = wl.stencil_csr((N, N, 1), coeffs)
    op = fa.CSR(rp, ci, va, hermitian=True, device=dev)
    # the exact interval of the 5-point Laplacian (Sec. 6, Example 1's formula)
    h = np.pi / (N + 1)
    op.set_spectral_interval(4.0 * (1.0 - np.cos(h)), 8.0 - 4.0 * (1.0 - np.cos(h)))
    b = torch.from_numpy(wl.rhs(N * N, seed=0)).to(dev)
    x = torch.empty_like(b)
    out = {}
    for deg in (0, 8):
        op.poly_setup(deg, "cheb")
        for _ in range(3):
            op.apply(b, m_max=200, tol=1e-10, out=x)
        torch.cuda.synchronize()
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            _, st = op.apply(b, m_max=200, tol=1e-10, out=x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        d = {"us_per_solve": dt * 1e6, "solves_per_s": 1.0 / dt, "iters": st["iters"],
             "mvms": st["mvms"], "inner_products": st["inner_products"]}
        if orc is not None:
            ref = torch.from_numpy(orc["poisson2d_32_ref"][deg]).to(dev)
            d["rel_err_vs_oracle_tol1e-12"] = float(torch.linalg.vector_norm(x - ref)
                                                    / torch.linalg.vector_norm(ref))
            d["oracle_s_per_solve"] = orc["poisson2d_32"][f"degree_{deg}"]["s_per_solve"]
            d["speedup_vs_oracle"] = d["oracle_s_per_solve"] / dt
        out[f"degree_{deg}"] = d
        log(f"Poisson 32^2 degree {deg}: {dt * 1e6:.0f} us per solve, m = {st['iters']}"
            + (f", err {d['rel_err_vs_oracle_tol1e-12']:.1e}, oracle {d['oracle_s_per_solve']:.3f} s"
               if orc is not None else ""))
    op.release_workspace()
    return out


def table1_leg(fa, torch, wl, dev, orc):
    """Sec. 6, Example 1, Table 1's workload: the 3D Laplacian on 100^3
    interior points (n = 10^6, Hermitian: Lanczos), b ~ N(0, 1) seed 0 scaled
    to unit norm, Chebyshev q with d coefficients on the exact interval, right
    preconditioning (Algorithm 2).  Each row runs the printed iteration count
    as a fixed m (the same mvms and inner products as the printed row), one
    pass (1P, y_j stored) and two passes (2P, O(n) memory), median of 3;
    the true error is against the DST closed form the oracle leg computed.
    The printed times are context (MATLAB on an 8-core laptop CPU)."""
    import numpy as np
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                                    "golden", "table1_laplace3d.json")))
    N = g["N"]
    op = fa.Stencil7((N, N, N), wl.laplace_stencil(3), hermitian=True, device=dev)
    b = wl.rhs(N ** 3, seed=0)
    b = torch.from_numpy(b / np.linalg.norm(b)).to(dev)
    x = torch.empty_like(b)
    ref = torch.from_numpy(orc["table1_ref"]).to(dev) if orc is not None else None
    rows = []
    for r in g["rows"]:
        d, m = r["d"], r["iterations"]
        op.poly_setup(d - 1, "cheb")
        row = {"d": d, "iterations": m}
        for name, tp in (("1P", False), ("2P", True)):
            op.apply(b, m_max=m, tol=0.0, right=True, two_pass=tp, out=x)
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                _, st = op.apply(b, m_max=m, tol=0.0, right=True, two_pass=tp, out=x)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = float(np.median(ts))
            row[f"ms_{name}"] = t * 1e3
            row[f"mvms_{name}"] = st["mvms"]
            row[f"inner_products_{name}"] = st["inner_products"]
            row[f"printed_s_{name}"] = r[f"time_{name}_s"]
            if ref is not None:
                row[f"rel_err_{name}_vs_closed_form"] = float(
                    torch.linalg.vector_norm(x - ref) / torch.linalg.vector_norm(ref))
        rows.append(row)
        log(f"Table 1 d = {d:2d}, m = {m:3d}: 1P {row['ms_1P']:7.2f} ms, 2P {row['ms_2P']:7.2f} ms"
            + (f", error {row['rel_err_1P_vs_closed_form']:.1e} / "
               f"{row['rel_err_2P_vs_closed_form']:.1e}" if ref is not None else ""))
        op.release_workspace()
    return {"workload": "laplace3d_100^3 invsqrt, Chebyshev, right preconditioning, fixed m = "
                        "the printed iterations", "rows": rows}


def overlap_leg(fa, torch, wl, dev, with_plain=True):
    """Sec. 6, Example 2's shape: (Q^2)^{-1/2} b with Q = Gamma_5 D(m_w, mu),
    m_w = -1.4, mu = 0.3, on a 64 x 32^3 lattice (n = 25,165,824 complex, one
    vector 403 MB).  The paper's gauge field is not available: links
    exp(0.3 i H) (seed 1), so the iteration counts are not Table 2's.  b
    complex N(0, 1) seed 0; Ritz polynomials with d = 8, 16, 32, 64
    coefficients (start vector seed 11) and the plain method, tol 4e-5 (the
    error level Table 2 stops at), checks every 64/d steps.  Errors against a
    tight GPU solve (d = 32, tol 1e-10); mvms count products with Q (two per
    product with Q^2), as Table 2 does.  Times exclude the polynomial setup
    (reported apart); Table 2's exclude the stopping checks, which are
    included here."""
    import numpy as np
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests",
                                    "golden", "table2_overlap.json")))
    dims = tuple(g["dims_t_z_y_x"])
    t0 = time.perf_counter()
    U = wl.su3_links_device(dims, eps=0.3, seed=1, device=dev)
    op = fa.Wilson(U, g["m_w"], mu=g["mu"], squared=True, device=dev)
    del U
    b = torch.from_numpy(wl.rhs(op.n, seed=0, complex_=True)).to(dev)
    start = torch.from_numpy(wl.rhs(op.n, seed=11, complex_=True)).to(dev)
    torch.cuda.synchronize()
    log(f"overlap 64x32^3: links and operator in {time.perf_counter() - t0:.1f} s")
    vec_gb = op.n * 16 / 1e9
    op.poly_setup(31, "ritz", start=start)
    xref, sref = op.apply(b, m_max=80, tol=1e-10)
    xref = xref.clone()
    op.release_workspace()
    printed = {r["d"]: r for r in g["rows"]}
    rows = []
    for d in (8, 16, 32, 64):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        op.poly_setup(d - 1, "ritz", start=start)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, st = op.apply(b, m_max=100, tol=g["tol"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(x - xref) / torch.linalg.vector_norm(xref))
        rows.append({"d": d, "iterations": st["iters"], "mvms_Q": 2 * st["mvms"],
                     "inner_products": st["inner_products"], "s_per_solve": dt,
                     "s_setup": ts, "rel_err_vs_reference": err,
                     "basis_GB": (st["iters"] + 1) * vec_gb,
                     "printed_iterations": printed[d]["iterations"],
                     "printed_s_64_nodes": printed[d]["time_64_nodes_s"]})
        log(f"overlap d = {d:2d}: {dt:.2f} s per solve (setup {ts:.2f} s), m = {st['iters']}, "
            f"{2 * st['mvms']} products with Q, error {err:.1e}")
        del x
        op.release_workspace()
    out = {"workload": "overlap_q2_64x32^3 m_w=-1.4 mu=0.3 invsqrt, Ritz, tol 4e-5",
           "n": op.n, "vector_GB": vec_gb,
           "reference": {"d": 32, "tol": 1e-10, "iterations": sref["iters"]},
           "rows": rows}
    if with_plain:
        # the plain method; its basis is the memory Table 2's d = 1 row needs
        op.poly_setup(0, "ritz", start=start)
        t0 = time.perf_counter()
        x, st = op.apply(b, m_max=300, tol=g["tol"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = float(torch.linalg.vector_norm(x - xref) / torch.linalg.vector_norm(xref))
        out["plain"] = {"iterations": st["iters"], "converged": bool(st["converged"]),
                        "mvms_Q": 2 * st["mvms"], "inner_products": st["inner_products"],
                        "s_per_solve": dt, "rel_err_vs_reference": err,
                        "basis_GB": (st["iters"] + 1) * vec_gb,
                        "printed_basis_GB_at_m_1600": 1601 * vec_gb}
        log(f"overlap plain: {dt:.2f} s, m = {st['iters']}, error {err:.1e}, basis "
            f"{(st['iters'] + 1) * vec_gb:.0f} GB (Table 2's m = 1600 would need "
            f"{1601 * vec_gb:.0f} GB)")
        del x
        op.release_workspace()
    return out


def wilson_leg(fa, torch, wl, dev):
    """The 4D Wilson-Dirac-like operator on 16^4 (links exp(0.3 i H), m0 =
    0.05), A^{-1/2} b with a Ritz polynomial of degree 16, tol 1e-8, and
    the same with q == 1.  The Newton middle terms (read r with its 8
    neighbours, the links, v; write r') are timed with HIP events: 3 spinor
    fields + the links, which are special unitary and kept as two rows per
    3 x 3 matrix (the third rebuilt in the kernel) = 62.9 MB per launch."""
    L = 16
    op = fa.Wilson(wl.su3_links(L, eps=0.3, seed=1), 0.05, device=dev)
    start = torch.from_numpy(wl.rhs(op.n, seed=11, complex_=True)).to(dev)
    b = torch.from_numpy(wl.rhs(op.n, seed=0, complex_=True)).to(dev)
    out = {}
    for deg, m_max in ((16, 200), (0, 1000)):
        op.poly_setup(deg, "ritz", start=start)
        op.apply(b, m_max=m_max, tol=1e-8)
        torch.cuda.synchronize()
        reps = 3 if deg else 1
        t0 = time.perf_counter()
        sts = [op.apply(b, m_max=m_max, tol=1e-8, profile=deg > 0)[1] for _ in range(reps)]
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        d = {"solves_per_s": 1.0 / dt, "iters": sts[-1]["iters"], "mvms": sts[-1]["mvms"]}
        if deg:
            nch = sum(s_["n_chain"] for s_ in sts)
            ms = sum(s_["ms_chain"] for s_ in sts)
            d["chain_launch_us"] = ms / nch * 1e3
            d["chain_bytes"] = sts[-1]["chain_bytes"]
            d["chain_GBs"] = sts[-1]["chain_bytes"] / (ms / nch * 1e-3) / 1e9
        out[f"degree_{deg}"] = d
        log(f"Wilson 16^4 degree {deg}: {1.0 / dt:.2f} solves/s, m = {sts[-1]['iters']}"
            + (f", chain launch {d['chain_launch_us']:.1f} us, {d['chain_GBs']:.0f} GB/s" if deg else ""))
    op.release_workspace()
    return out


def csr_leg(fa, torch, wl, dev):
    """The CSR kernel.  (1) The paper's graph example in shape (Sec. 6,
    Example 3): L^{1/2} b = L^{-1/2} (L b) for the singular in-degree Laplacian
    of a synthetic directed power-law graph (n = 281,903, about 2.58M stored
    entries), b a canonical unit vector, tol 1e-7, checks every 32 / d steps:
    Ritz polynomial of degree 8 against the plain method (degree 0); the Newton
    middle terms of the degree-8 solve (CSR product of r fused with v: row
    pointers, column indices, values, r, v and the output once = the
    algorithmic bytes) are timed by HIP events; both results are compared
    with a plain solve at tol 1e-9.  (2) y = A x through fa_op_apply on the
    same matrix and on the 2D Poisson 32 x 32 matrix, timed per call from the
    host (so including each call's host overhead)."""
    import numpy as np
    out = {}
    rp, ci, va = wl.powerlaw_digraph_laplacian_csr(281903, 2594228, seed=5)
    op = fa.CSR(rp, ci, va, device=dev)
    b = torch.zeros(op.n, dtype=torch.float64, device=dev)
    b[int(np.random.default_rng(0).integers(op.n))] = 1.0
    start = torch.from_numpy(wl.rhs(op.n, seed=8)).to(dev)
    op.poly_setup(0)
    x_ref, st_ref = op.apply(b, kind="sqrt", m_max=1500, tol=1e-9, check_every=32)
    x_ref = x_ref.clone()

    def diff(x):
        return float(torch.linalg.vector_norm(x - x_ref) / torch.linalg.vector_norm(x_ref))

    d = {"workload": "powerlaw digraph Laplacian n=281903, L^(1/2) e_i, tol 1e-7, k = 32/d",
         "reference": f"plain solve, tol 1e-9 (m = {st_ref['iters']})"}
    for deg, k in ((8, 3), (0, 32)):
        op.poly_setup(deg, "ritz", start=start)
        op.apply(b, kind="sqrt", m_max=1500, tol=1e-7, check_every=k)
        torch.cuda.synchronize()
        reps = 2 if deg else 1
        t0 = time.perf_counter()
        sts = []
        for _ in range(reps):
            x, st = op.apply(b, kind="sqrt", m_max=1500, tol=1e-7, check_every=k, profile=deg > 0)
            sts.append(st)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        e = {"solves_per_s": 1.0 / dt, "iters": sts[-1]["iters"], "mvms": sts[-1]["mvms"],
             "rel_diff_vs_reference": diff(x)}
        if deg:
            nch = sum(s_["n_chain"] for s_ in sts)
            ms = sum(s_["ms_chain"] for s_ in sts)
            by = sts[-1]["chain_bytes"]
            e.update({"chain_launch_us": ms / nch * 1e3, "chain_bytes_per_launch": by,
                      "chain_GBs": by / (ms / nch * 1e-3) / 1e9,
                      "chain_frac": by / (ms / nch * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "launches_timed": nch, "mvms_setup": deg + 1})
        d[f"ritz_degree_{deg}" if deg else "plain"] = e
        log(f"digraph sqrt degree {deg}: {1.0 / dt:.2f} solves/s, m = {e['iters']}, mvms "
            f"{e['mvms']}, diff vs reference {e['rel_diff_vs_reference']:.1e}"
            + (f", CSR chain launch {e['chain_launch_us']:.1f} us, {e['chain_GBs']:.0f} GB/s"
               if deg else ""))
    d["speedup_degree8_over_plain"] = (d["ritz_degree_8"]["solves_per_s"]
                                       / d["plain"]["solves_per_s"])
    out["digraph_sqrt_281903"] = d
    op.release_workspace()
    del op
    for name, (rp, ci, va) in (
            ("powerlaw_digraph_281903", wl.powerlaw_digraph_laplacian_csr(281903, 2594228, seed=5)),
            ("poisson2d_32", wl.stencil_csr((32, 32, 1), wl.laplace_stencil(2)))):
        op = fa.CSR(rp, ci, va, device=dev)
        x = torch.from_numpy(wl.rhs(op.n, seed=1)).to(dev)
        y = torch.empty_like(x)
        for _ in range(3):
            op.op_apply(x, out=y)
        torch.cuda.synchronize()
        reps = 50
        t0 = time.perf_counter()
        for _ in range(reps):
            op.op_apply(x, out=y)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        n, nnz = op.n, len(ci)
        nbytes = 4 * (n + 1) + 12 * nnz + 16 * n
        out[name] = {"n": n, "nnz": nnz, "us_per_call_host": dt * 1e6,
                     "GBs_per_call_host": nbytes / dt / 1e9, "bytes": nbytes}
        log(f"CSR SpMV {name}: {dt * 1e6:.1f} us per call (host), "
            f"{nbytes / dt / 1e9:.0f} GB/s")
    return out


def batched_leg(fa, torch, wl, dev):
    """96^3 convection-diffusion (Pe = 50), 64 right-hand sides N(0, 1) as one
    block Arnoldi (fa_block_apply), Chebyshev degree 16, FP32 stencil chain
    (the 64 columns as one batch of vectors) with FP64 orthogonalization and
    H^{-1/2} (tol 1e-7), and the FP64 block solve (tol 1e-10); compared with the
    same right-hand sides solved one at a time (FP64, tol 1e-10: the
    per-column reference) on the same GPU."""
    import numpy as np
    N, s, K = 96, 64, 16
    dims = (N, N, N)
    op = fa.Stencil7(dims, wl.convdiff_stencil(N, 50.0), device=dev)
    op.poly_setup(K, "cheb")
    B = torch.from_numpy(np.stack([wl.rhs(N ** 3, seed=c) for c in range(s)], 1)).to(dev)
    log("batched: 96^3 x 64 right-hand sides, block Arnoldi, mixed precision")
    _, st0 = op.block_apply(B, m_max=30, tol=1e-7, mixed=True)  # first use: autotuning
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        X, st = op.block_apply(B, m_max=30, tol=1e-7, mixed=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    Xf, stf = op.block_apply(B, m_max=30, tol=1e-10)  # the FP64 block path
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Xf, stf = op.block_apply(B, m_max=30, tol=1e-10)
    torch.cuda.synchronize()
    dtf = time.perf_counter() - t1
    # per-column references: single-vector FP64 solves
    errs = []
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    refs = []
    for c in range(s):
        xc, _ = op.apply(B[:, c].contiguous(), m_max=100, tol=1e-10)
        refs.append(xc.clone())
    torch.cuda.synchronize()
    dts = time.perf_counter() - t2
    for c in range(s):
        errs.append(float(torch.linalg.vector_norm(X[:, c] - refs[c])
                          / torch.linalg.vector_norm(refs[c])))
    # the same 64 right-hand sides one at a time in the same precision mode
    cols = [B[:, c].contiguous() for c in range(s)]
    op.apply(cols[0], m_max=100, tol=1e-7, mixed=True)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for c in range(s):
        op.apply(cols[c], m_max=100, tol=1e-7, mixed=True)
    torch.cuda.synchronize()
    dtm = time.perf_counter() - t3
    # block steps replayed from HIP graphs (captured on the first graph call)
    op.block_apply(B, m_max=30, tol=1e-7, mixed=True, graph=True)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(reps):
        Xg, stg = op.block_apply(B, m_max=30, tol=1e-7, mixed=True, graph=True)
    torch.cuda.synchronize()
    dtg = (time.perf_counter() - t4) / reps
    same = bool(torch.equal(Xg, X))
    # a small block (launch-bound): 32^3, 16 right-hand sides, eager vs graphs
    Ns, ss = 32, 16
    ops_ = fa.Stencil7((Ns, Ns, Ns), wl.convdiff_stencil(Ns, 50.0), device=dev)
    ops_.poly_setup(K, "cheb")
    Bs = torch.from_numpy(np.stack([wl.rhs(Ns ** 3, seed=c) for c in range(ss)], 1)).to(dev)
    small = {}
    for g in (False, True):
        ops_.block_apply(Bs, m_max=30, tol=1e-7, mixed=True, graph=g)
        ops_.block_apply(Bs, m_max=30, tol=1e-7, mixed=True, graph=g)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        for _ in range(10):
            _, sts = ops_.block_apply(Bs, m_max=30, tol=1e-7, mixed=True, graph=g)
        torch.cuda.synchronize()
        small["graph" if g else "eager"] = (time.perf_counter() - t5) / 10 * 1e3
    ops_.release_workspace()
    out = {"workload": "convdiff3d_96^3 Pe=50 invsqrt chebyshev degree 16, 64 rhs",
           "rhs_solves_per_s": s / dt, "ms_per_block_solve": dt * 1e3,
           "block_iters": st["iters"], "tol": 1e-7, "max_col_rel_err_vs_fp64": max(errs),
           "ms_fH": st["ms_fH"], "ns_iters": st["ns_iters"],
           "autotune_ms_first_call": st0["ms_tune"],
           "fp64_block": {"rhs_solves_per_s": s / dtf, "iters": stf["iters"], "tol": 1e-10},
           "single_vector_fp64_tol1e-10": {"rhs_solves_per_s": s / dts},
           "single_vector_mixed_tol1e-7": {"rhs_solves_per_s": s / dtm},
           "speedup_vs_single_vector_same_mode": dtm / dt,
           "hip_graph_steps": {"ms_per_block_solve": dtg * 1e3, "graph_steps": stg["graph_steps"],
                               "same_result_as_eager": same,
                               "small_32^3_x16_ms": {"eager": small["eager"],
                                                     "graph": small["graph"],
                                                     "block_iters": sts["iters"]}}}
    log(f"batched: {s / dt:.1f} rhs-solves/s ({dt * 1e3:.0f} ms per block of 64, m = {st['iters']}), "
        f"max col err {max(errs):.2e}; FP64 block {s / dtf:.1f}/s; one at a time: FP64 "
        f"{s / dts:.1f}/s, mixed {s / dtm:.1f}/s; steps from HIP graphs {dtg * 1e3:.0f} ms "
        f"(same bits: {same}); 32^3 x 16: eager {small['eager']:.2f} ms, graphs "
        f"{small['graph']:.2f} ms")
    op.release_workspace()
    return out


def serving_leg(args, fa, torch, wl, dev):
    """Requests through the library's server (fa_server_*): operators and
    polynomials set up once and kept on the device; each request gets its
    own output vector; latency = completion - submission (server clock)."""
    import threading
    import queue

    import numpy as np

    log("serving: building the operators of the mix")
    ops, bs = {}, {}
    for name, _ in wl.SERVING_TYPES:
        if name == "laplace2d_256":
            op = fa.Stencil7((256, 256, 1), wl.laplace_stencil(2), hermitian=True, device=dev)
            op.poly_setup(8, "cheb")
            m_max = 300
        elif name.startswith("convdiff3d_"):
            n1 = int(name.split("_")[1])
            op = fa.Stencil7((n1, n1, n1), wl.convdiff_stencil(n1, 50.0), device=dev)
            op.poly_setup(16, "cheb")
            m_max = 100
        else:
            op = fa.Wilson(wl.su3_links(16, eps=0.3, seed=1), 0.05, device=dev)
            st = torch.from_numpy(wl.rhs(op.n, seed=11, complex_=True)).to(dev)
            op.poly_setup(16, "ritz", start=st)
            m_max = 150
        cplx = op.dtype == torch.complex128
        ops[name] = (op, m_max)
        bs[name] = [torch.from_numpy(wl.rhs(op.n, seed=s, complex_=cplx)).to(dev)
                    for s in range(4)]
    torch.cuda.synchronize()
    pool = int(args.serve_pool_gb * (1 << 30))
    srv = fa.Server(pool, n_workers=args.serve_workers, device=dev)

    def run(reqs, arrivals):
        out = []
        q = queue.Queue()

        def waiter():
            while True:
                item = q.get()
                if item is None:
                    return
                t, r = item
                x, info = srv.wait(t, raise_errors=False)
                out.append((r, info))
                del x

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for i, r in enumerate(reqs):
            if arrivals is not None:
                delay = t0 + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
            op, m_max = ops[r["type"]]
            t = srv.submit(op, bs[r["type"]][r["seed"] % 4], kind=r["kind"], m_max=m_max,
                           tol=r["tol"])
            q.put((t, r))
        q.put(None)
        th.join()
        sub = min(info["t_submit_ms"] for _, info in out)
        end = max(info["t_done_ms"] for _, info in out)
        lat = np.array([info["t_done_ms"] - info["t_submit_ms"] for _, info in out])
        wait = np.array([info["t_start_ms"] - info["t_submit_ms"] for _, info in out])
        return {"requests": len(out), "solves_per_s": len(out) / ((end - sub) * 1e-3),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_queue_wait_ms": float(wait.mean()),
                "errors": sum(1 for _, i in out if i["status"] < 0),
                "not_converged": sum(1 for _, i in out if i["status"] == 1),
                "mean_iters": float(np.mean([i["stats"]["iters"] for _, i in out]))}

    # each type alone (invsqrt, tol 1e-10) for reference, after one warm-up
    solo = {}
    for name, (op, m_max) in ops.items():
        for rep in range(2):
            t = srv.submit(op, bs[name][0], m_max=m_max, tol=1e-10)
            _, info = srv.wait(t)
        solo[name] = {"ms": info["t_done_ms"] - info["t_start_ms"],
                      "iters": info["stats"]["iters"]}
    log("serving: solo " + ", ".join(f"{k} {v['ms']:.1f} ms (m={v['iters']})"
                                     for k, v in solo.items()))
    mix = wl.serving_mix(args.serve_requests)
    cap = run(mix[: max(1, args.serve_requests // 2)], None)
    log(f"serving: saturated ({cap['requests']} requests submitted at once): "
        f"{cap['solves_per_s']:.1f} solves/s, p50 {cap['p50_ms']:.0f} ms, p99 {cap['p99_ms']:.0f} ms")
    arr = wl.poisson_arrivals(args.qps, args.serve_requests)
    poi = run(mix, arr)
    poi["offered_qps"] = args.qps
    log(f"serving: Poisson {args.qps:.0f} QPS ({poi['requests']} requests): "
        f"{poi['solves_per_s']:.1f} solves/s, p50 {poi['p50_ms']:.1f} ms, p99 {poi['p99_ms']:.1f} ms")
    half = 0.5 * cap["solves_per_s"]
    nh = max(20, min(args.serve_requests // 2, int(half * 3)))
    low = run(wl.serving_mix(nh, seed=13), wl.poisson_arrivals(half, nh, seed=14))
    low["offered_qps"] = half
    log(f"serving: Poisson {half:.0f} QPS (half the saturated rate, {nh} requests): "
        f"{low['solves_per_s']:.1f} solves/s, p50 {low['p50_ms']:.1f} ms, p99 {low['p99_ms']:.1f} ms")
    stt = srv.status()
    srv.close()
    return {"workers": args.serve_workers, "pool_GB": args.serve_pool_gb,
            "mix": {k: w for k, w in wl.SERVING_TYPES}, "solo": solo,
            "saturated": cap, f"poisson_{args.qps:.0f}qps": poi, "poisson_half_saturated": low,
            "peak_inflight": stt["peak_inflight"],
            "peak_pool_GB_in_flight": stt["peak_bytes_inflight"] / (1 << 30)}


def cpu_baseline(coeffs, dims, degree, tol):
    """The oracle leg (NumPy/SciPy FP64 on the host; nothing else runs it):

    * references for the true errors: the oracle's solve of the same b at
      degree 32 and tol 1e-12 (A^{-1/2} b), and A times it (A^{1/2} b);
    * the CPU baseline: the median of 3 whole oracle solves of the headline
      configuration (degree `degree`, tol `tol`), timed; the polynomial setup
      and the host H_j^{-1/2} e_1 evaluations are reported apart;
    * the 2D Poisson 32 x 32 configuration: oracle seconds per solve at
      degrees 0 and 8 (tol 1e-10, Lanczos) and tol-1e-12 references;
    * Table 1's workload (100^3 Laplacian): the DST closed form of A^{-1/2} b."""
    import numpy as np

    import workloads as wl
    from oracle import exact, krylov, operators, polynomials

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    b = wl.rhs(int(np.prod(dims)), seed=0)
    A = lambda v: operators.stencil_apply(coeffs, dims, v)  # noqa: E731
    # time spent in the oracle's dense H^{-1/2} e_1 (wrapped, not changed)
    fH = {"s": 0.0}
    inner = krylov.hessenberg_invsqrt_e1

    def timed_fH(H, beta):
        t = time.perf_counter()
        try:
            return inner(H, beta)
        finally:
            fH["s"] += time.perf_counter() - t

    krylov.hessenberg_invsqrt_e1 = timed_fH
    try:
        a, bb = operators.stencil_interval(coeffs, dims)
        log("oracle: reference solve (degree 32, tol 1e-12)")
        t0 = time.perf_counter()
        ref = krylov.fAb(A, b, polynomials.chebyshev(a, bb, 32), "invsqrt", m_max=100, tol=1e-12)
        t_ref = time.perf_counter() - t0
        log(f"oracle: reference m = {ref.iters}, est {ref.est:.1e}, {t_ref:.1f} s")
        runs = []
        for r in range(3):
            fH["s"] = 0.0
            t0 = time.perf_counter()
            q = polynomials.chebyshev(a, bb, degree)
            t1 = time.perf_counter()
            res = krylov.fAb(A, b, q, "invsqrt", m_max=200, tol=tol)
            t2 = time.perf_counter()
            runs.append({"s_total": t2 - t0, "s_setup": t1 - t0, "s_fH": fH["s"],
                         "iters": res.iters,
                         "rel_err_vs_ref": float(np.linalg.norm(res.x - ref.x)
                                                 / np.linalg.norm(ref.x))})
            log(f"oracle: solve {r + 1}/3 {t2 - t0:.1f} s (m = {res.iters}, host f(H) "
                f"{fH['s']:.2f} s)")
        # 2D Poisson 32 x 32, Lanczos (the small configuration)
        N2 = 32
        c2 = wl.laplace_stencil(2)
        rp, ci, va = wl.stencil_csr((N2, N2, 1), c2)
        A2 = lambda v: operators.csr_apply(rp, ci, va, v)  # noqa: E731
        lo, hi = operators.stencil_interval(c2, (N2, N2, 1))
        b2 = wl.rhs(N2 * N2, seed=0)
        p2, p2ref = {}, {}
        for deg in (0, 8):
            q2 = polynomials.chebyshev(lo, hi, deg)
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                r2 = krylov.fAb(A2, b2, q2, "invsqrt", m_max=200, tol=1e-10, orth="lanczos")
                ts.append(time.perf_counter() - t0)
            p2[f"degree_{deg}"] = {"s_per_solve": float(np.median(ts)), "iters": r2.iters}
            p2ref[deg] = krylov.fAb(A2, b2, q2, "invsqrt", m_max=200, tol=1e-12,
                                    orth="lanczos").x
        # Table 1's workload (Sec. 6, Example 1): the closed form of A^{-1/2} b
        N1 = 100
        b1 = wl.rhs(N1 ** 3, seed=0)
        b1 = b1 / np.linalg.norm(b1)
        t1ref = exact.stencil_fAb_dst(wl.laplace_stencil(3), (N1, N1, N1), b1, "invsqrt")
    finally:
        krylov.hessenberg_invsqrt_e1 = inner
    med = sorted(runs, key=lambda r: r["s_total"])[1]
    x_sqrt = A(ref.x)  # A^{1/2} b = A (A^{-1/2} b)
    log(f"oracle: median solve {med['s_total']:.1f} s, {threads} BLAS threads")
    return {"value": 1.0 / med["s_total"], "unit": "solves/s", "cores": threads,
            "kind": "oracle",
            "sample": f"3 whole oracle solves of the headline configuration (128^3, degree "
                      f"{degree}, tol {tol:g}), median; stencil products are single-threaded "
                      f"NumPy, Gram-Schmidt and the dense H^(-1/2) use BLAS/LAPACK with "
                      f"{threads} threads",
            "s_per_solve_median": med["s_total"], "s_setup": med["s_setup"],
            "s_host_fH": med["s_fH"], "iters": med["iters"],
            "rel_err_vs_ref": med["rel_err_vs_ref"], "runs_s": [r["s_total"] for r in runs],
            "reference_solve": {"degree": 32, "tol": 1e-12, "iters": ref.iters,
                                "s": t_ref},
            "poisson2d_32": p2,
            "x_ref_invsqrt": ref.x, "x_ref_sqrt": x_sqrt, "poisson2d_32_ref": p2ref,
            "table1_ref": t1ref}


if __name__ == "__main__":
    main()
