"""Benchmark: f(A)b solves/s on one MI355X, polynomially preconditioned vs plain.

Workload (the metric's configuration): 3D convection-diffusion, 7-point
first-order upwind stencil on a 128^3 grid (n = 2,097,152), Pe = 50 with
convection direction (1, 0.5, 0.25), real FP64; b ~ N(0, 1) (seed 0);
f = A^{-1/2}; Chebyshev polynomial of degree 16 on the exact spectral interval;
stopping tolerance 1e-8 on the difference-of-iterates estimate.

A step is one fa_apply solve (setup of the operator and polynomial excluded,
inputs resident in HBM).  Printed as one JSON line with a roofline object for
the dominant kernel (the stencil chain launch that evaluates three Clenshaw
terms: HIP events around each run of such launches in every timed solve) and
the CPU oracle timed on a bounded sample.  Extra fields report plain Arnoldi
(degree 0), degrees 4 and 32 and the square root on the same GPU, and the
serving workload: Poisson arrivals of a request mix (2D Laplacian 256^2,
convection-diffusion 64^3 / 96^3 / 128^3, Wilson 16^4; f in {sqrt, invsqrt},
tol in {1e-6, 1e-10}) through the library's request loop, with solves/s and
p50/p99 latency from submission to completion.
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
# st7_multi<..., NT, 8, true, true> at 128^3, keyed by NT: FETCH_SIZE x 2.00 +
# WRITE_SIZE x 1.00, the factors of a 2 GiB copy), from the rocprofv3 counter
# runs in profiles/st7_multi_convdiff128_deg16_hbm_counters.md
MULTI_TRAFFIC_BYTES = {3: (73777 + 32768) * 1024, 4: (83750 + 32768) * 1024}


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
    ap.add_argument("--qps", type=float, default=2000.0, help="serving arrival rate")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-workers", type=int, default=8)
    ap.add_argument("--serve-pool-gb", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
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

    # reference for the true error: degree 32, tight tolerance
    log("reference solve (degree 32, tol 1e-12)")
    op_ref = make(32)
    x_ref, _ = op_ref.apply(b, m_max=100, tol=1e-12)
    x_ref = x_ref.clone()
    op_ref.release_workspace()
    del op_ref

    def rel_err(x):
        return float(torch.linalg.vector_norm(x - x_ref) / torch.linalg.vector_norm(x_ref))

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
    n_chain = sum(s["n_chain"] for s in stats)
    ms_chain = sum(s["ms_chain"] for s in stats)
    bytes_avg = sum(s["chain_bytes"] * s["n_chain"] for s in stats) / max(n_chain, 1)
    avg_ms = ms_chain / max(n_chain, 1)
    terms = sum(s["n_chain_terms"] for s in stats) / max(n_chain, 1)  # per timed launch
    traffic = MULTI_TRAFFIC_BYTES.get(int(round(terms)))  # None: not measured for this kernel
    # algorithmic bytes of one timed launch as designed: x, v, b_(k+2) read
    # once and the two terms the next launch needs written once (5 vectors,
    # bytes_avg from the solve's statistics); per-term accounting (each term
    # at the 4 vectors of a one-term launch) is reported beside it
    per_term = 4 * (N ** 3) * 8
    algo_bytes = terms * per_term
    achieved = bytes_avg / (avg_ms * 1e-3) / 1e9
    achieved_per_term = algo_bytes / (avg_ms * 1e-3) / 1e9
    log(f"degree {K}: {value:.2f} solves/s, m = {st0['iters']}, err = {err:.2e}, "
        f"chain launch {avg_ms * 1e3:.1f} us ({terms:.0f} terms), {achieved:.0f} GB/s of the "
        f"launch's 5 vectors, {achieved_per_term:.0f} GB/s per-term accounting")
    op.release_workspace()
    del op

    extra = {"iters": st0["iters"], "mvms": st0["mvms"], "inner_products": st0["inner_products"],
             "rel_err_vs_ref": err, "est": st0["est_rel_change"],
             "ms_host_fH_per_solve": st0["ms_host_fH"]}

    # ---- the same solve with one launch per recurrence term ---------------
    o = make(K)
    xu, dtu, stu = timed(o, 5, 1, profile=True, fuse=False)
    nu = sum(s_["n_chain"] for s_ in stu)
    avg_u = sum(s_["ms_chain"] for s_ in stu) / max(nu, 1)
    extra["single_term_launches"] = {
        "solves_per_s": 5 / dtu, "rel_err": rel_err(xu), "kernel": "st7_chain<true,true>",
        "avg_launch_us": avg_u * 1e3, "bytes_per_launch": stu[-1]["chain_bytes"],
        "achieved_GBs": stu[-1]["chain_bytes"] / (avg_u * 1e-3) / 1e9}
    log(f"single-term launches: {5 / dtu:.2f} solves/s, chain launch {avg_u * 1e3:.1f} us")
    o.release_workspace()
    del o

    # ---- mixed precision: the chain in FP32 (tolerance 1e-7) ---------------
    o = make(K)
    xm, dtm, stm = timed(o, 5, 1, profile=True, mixed=True, tol_=1e-7, profile_every=5)
    nm = sum(s_["n_chain"] for s_ in stm)
    avg_m = sum(s_["ms_chain"] for s_ in stm) / max(nm, 1)
    terms_m = sum(s_["n_chain_terms"] for s_ in stm) / max(nm, 1)
    extra["mixed_fp32_chain"] = {
        "solves_per_s": 5 / dtm, "iters": stm[-1]["iters"], "rel_err": rel_err(xm),
        "tol": 1e-7, "kernel": f"st7_multi<float, {terms_m:.0f} terms>",
        "avg_launch_us": avg_m * 1e3, "bytes_per_launch": stm[-1]["chain_bytes"],
        "achieved_GBs": stm[-1]["chain_bytes"] / (avg_m * 1e-3) / 1e9}
    log(f"mixed precision: {5 / dtm:.2f} solves/s, m = {stm[-1]['iters']}, "
        f"err {rel_err(xm):.2e}, chain launch {avg_m * 1e3:.1f} us")
    o.release_workspace()
    del o

    # ---- other degrees and the square root --------------------------------
    others = {}
    for deg, kind in ((4, "invsqrt"), (32, "invsqrt"), (K, "sqrt")):
        o = make(deg)
        xo, dto, sto = timed(o, 3, 1, kind=kind)
        if kind == "sqrt":
            # A^{1/2} b = A (A^{-1/2} b)
            ax = o.op_apply(x_ref)
            e = float(torch.linalg.vector_norm(xo - ax) / torch.linalg.vector_norm(ax))
        else:
            e = rel_err(xo)
        others[f"{kind}_deg{deg}"] = {"solves_per_s": 3 / dto, "iters": sto[-1]["iters"],
                                      "rel_err": e}
        log(f"{kind} degree {deg}: {3 / dto:.2f} solves/s, m = {sto[-1]['iters']}, err {e:.2e}")
        o.release_workspace()
        del o
    extra["other_degrees"] = others

    # ---- plain Arnoldi (degree 0) on the same GPU -------------------------
    if not args.no_plain:
        log("plain Arnoldi (degree 0), 1 timed solve")
        op0 = make(0)
        x0, dt0, st_0 = timed(op0, 1, 0, m_max=1000)
        e0 = rel_err(x0)
        extra["plain"] = {"solves_per_s": 1 / dt0, "iters": st_0[-1]["iters"],
                          "rel_err": e0, "ms_host_fH": st_0[-1]["ms_host_fH"],
                          "speedup_poly_over_plain": value * dt0}
        log(f"plain: {1 / dt0:.3f} solves/s, m = {st_0[-1]['iters']}, err {e0:.2e}, "
            f"host f(H) {st_0[-1]['ms_host_fH']:.0f} ms")
        op0.release_workspace()
        del op0

    # ---- Wilson 16^4 (the lattice operator) --------------------------------
    extra["wilson4d_16"] = wilson_leg(fa, torch, wl, dev)

    # ---- CSR SpMV (the operator of the directed-graph example) ------------
    extra["csr_spmv"] = csr_leg(fa, torch, wl, dev)

    # ---- batched: 64 right-hand sides as one block Arnoldi ------------------
    if not args.no_batch:
        extra["batched"] = batched_leg(fa, torch, wl, dev)

    # ---- serving: Poisson arrivals of a request mix ------------------------
    if not args.no_serve:
        extra["serving"] = serving_leg(args, fa, torch, wl, dev)

    # ---- CPU oracle on a bounded sample -----------------------------------
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(coeffs, dims, K, st0["iters"])

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
                     "per_term_accounting": {
                         "bytes_per_launch": algo_bytes, "achieved": achieved_per_term,
                         "frac": achieved_per_term / HBM_PEAK_GBS,
                         "unit": "each term at 4 vectors, as one term per launch moves"},
                     "traffic_frac": (traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None),
                     "avg_launch_us": avg_ms * 1e3, "launches_timed": n_chain},
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


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
    """y = A x with the CSR kernel: a synthetic directed power-law graph
    Laplacian of the shape of the paper's graph example (n = 281,903, about
    2.59M stored entries) and the 2D Poisson 32 x 32 matrix.  GB/s counts
    row pointers, column indices, values, x and y once."""
    out = {}
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
        out[name] = {"n": n, "nnz": nnz, "us_per_spmv": dt * 1e6,
                     "GBs": nbytes / dt / 1e9, "bytes": nbytes}
        log(f"CSR SpMV {name}: {dt * 1e6:.1f} us, {nbytes / dt / 1e9:.0f} GB/s")
    return out


def batched_leg(fa, torch, wl, dev):
    """96^3 convection-diffusion (Pe = 50), 64 right-hand sides N(0, 1) as one
    block Arnoldi (fa_block_apply), Chebyshev degree 16, FP32 stencil chain
    with FP64 orthogonalization and H^{-1/2} (tol 1e-7); compared with the
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
           "ms_fH": st["ms_fH"], "ns_iters": st["ns_iters"], "zc": st["zc"],
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


def cpu_baseline(coeffs, dims, degree, m_gpu):
    """The oracle (NumPy FP64) on the host: a fixed sample of Krylov steps at the
    full size, scaled to one whole solve of m_gpu steps."""
    import numpy as np

    import workloads as wl
    from oracle import krylov, operators, polynomials

    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    b = wl.rhs(int(np.prod(dims)), seed=0)
    a, bb = operators.stencil_interval(coeffs, dims)
    q = polynomials.chebyshev(a, bb, degree)
    A = lambda v: operators.stencil_apply(coeffs, dims, v)  # noqa: E731
    steps = 3
    log(f"cpu oracle: {steps} steps at full size (degree {degree})")
    t0 = time.perf_counter()
    krylov.fAb(A, b, q, "invsqrt", m_max=1, tol=0.0)
    t1 = time.perf_counter()
    krylov.fAb(A, b, q, "invsqrt", m_max=1 + steps, tol=0.0)
    t2 = time.perf_counter()
    per_step = ((t2 - t1) - (t1 - t0)) / steps
    start = (t1 - t0) - per_step
    est_solve = start + per_step * m_gpu
    log(f"cpu oracle: {per_step:.2f} s per Krylov step, est. {est_solve:.1f} s per solve")
    return {"value": 1.0 / est_solve, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle runs of 1 and {1 + steps} Krylov steps at the full 128^3 size, "
                      f"degree {degree}; the per-step time times the GPU's m = {m_gpu} plus the "
                      f"start cost gives one solve ({est_solve:.1f} s); stencil products are "
                      f"single-threaded NumPy, Gram-Schmidt uses BLAS with {threads} threads"}


if __name__ == "__main__":
    main()
