#!/usr/bin/env python3
"""Refined solves/s to backward error 1e-14, recycled vs plain GMRES-IR, n=8192.

One timed step is the whole hot path on one system: gmresir_factor (LU in
u_f = fp16 with the copies of A the solve needs) followed by gmresir_solve
(x0, refinement steps with the fp64 residual and the GCRO-DR(30, 10)
correction solve, x update), on a seeded synthetic randsvd matrix (mode 3:
geometric singular values from 1 to 1/kappa, Haar factors) with
x_true ~ U(-1, 1), b = A x_true, precisions (fp16, fp32, fp64).  The inputs
are generated on the GPU and are resident in HBM before the timed region.
The same steps are then timed with k = 0 (plain GMRES-IR(30)), and the
outcome (status, refinement steps, Arnoldi iterations) of the kappa = 1e6
and 1e10 systems of the same size is reported for both.

Live kernel timing: the library brackets every launch of its kernel classes
with HIP events on the stream they run on (opts.timing); the class with the
largest share of the timed steps gives the roofline object: the
factorisation's classes against the fp16 matrix-core peak (algorithmic flops
of their launches over their summed duration), the solve's against 8 TB/s
(algorithmic bytes).  The object also carries the whole factorisation's
matrix-core fraction (2 n^3 / 3 flops over its wall time), the GEMM-only
update launches, and one whole Arnoldi step against HBM (n^2 (s_A + s_f)
bytes plus one read of the basis, per step).  HBM traffic measured with
rocprofv3 counters is read from profiles/traffic.json when that file was
taken on the current source of the kernel.

Also reported: M2, the factorisation amortised over 16 right-hand sides
solved in sequence with the recycle space kept between them (recycled and
plain), and a comparator, plain fp64 LU-based refinement on the same GPU (the
vendor LU through torch.linalg.lu_factor, fp64 corrections with its factors).

cpu_baseline: the CPU oracle (test infrastructure, numpy) on the benchmark's
own system at full order (factor and one solve, about 30 s on 16 cores), and
a native fp64 LAPACK LU solve of it as context.

Other configurations (precision triple, order, kappa, m, k) are selected by
flags; --prolate16k adds the outcome of the ill-conditioned Toeplitz system of
order 16384 at both of its precision triples.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP16_MFMA_PEAK_TFLOPS = 2500.0
FP64_MFMA_PEAK_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# source files whose text determines each kernel class (traffic validity)
KERNEL_SOURCES = {
    "lu_panel": "kernels_lu.hip", "lu_trsm": "kernels_lu.hip", "lu_gemm": "kernels_lu.hip",
    "trsv_lower": "kernels_solve.hip", "trsv_upper": "kernels_solve.hip",
    "gemv_au": "kernels_solve.hip", "residual": "kernels_solve.hip", "ortho": "kernels_solve.hip",
}


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--kappa", type=float, default=1e2)
    ap.add_argument("--m", type=int, default=30)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--uf", default="fp16", choices=("fp16", "bf16", "fp32"))
    ap.add_argument("--u", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--ur", default="fp64", choices=("fp64", "dd"))
    ap.add_argument("--tau", type=float, default=None,
                    help="GMRES tolerance (default 1e-4 for u = fp32, 1e-8 for u = fp64)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip timing the gradient (forward solve + adjoint solve + rank-1)")
    ap.add_argument("--outcomes", default="1e6,1e10",
                    help="kappa values whose outcome is reported ('' for none)")
    ap.add_argument("--prolate16k", action="store_true",
                    help="also report the outcome of the ill-conditioned Toeplitz system "
                         "(prolate w = 0.48, n = 16384, m = 50, k = 20 and 0) at "
                         "(bf16, fp32, fp64) and (fp32, fp64, double-double); about 2 minutes")
    ap.add_argument("--batched", type=int, default=128,
                    help="also time this many systems of the uneven batch (n ~ U[128, 2048], "
                         "kappa2 log-uniform in [1e1, 1e8], 1-8 right-hand sides; 128 take "
                         "about 45 s, 512 about 3 minutes) through gmresir_solve_batched "
                         "(0 to skip)")
    ap.add_argument("--batched-workers", type=int, default=8)
    ap.add_argument("--m2-rhs", type=int, default=16,
                    help="right-hand sides of the amortised variant (factor once, keep_recycle=1)")
    ap.add_argument("--no-comparator", action="store_true",
                    help="skip the vendor fp64 LU comparator")
    ap.add_argument("--gen", choices=("gpu", "cpu"), default="gpu",
                    help="draw the system on the GPU (torch) or on the CPU (numpy, slower)")
    ap.add_argument("--copy-ref-mib", type=int, default=0,
                    help="first run one plain fp32 copy kernel (out = -in) over this many MiB, "
                         "the reference for scaling HBM traffic counters")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest(name: str) -> str:
    path = os.path.join(ROOT, "paper_2201_09827_amd", "csrc", name)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_for(kernel: str, launches_per_step: float):
    """HBM bytes per launch from the counter summary, or None when missing or
    taken on another version of the kernel's source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get("kernels", {}).get(kernel)
    if not rec or rec.get("source_sha256_16") != source_digest(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(a_np, b_np, kappa: float, seed: int, m: int, k: int):
    """The oracle (as it stands) on the benchmark's own system (factor and one
    solve at the full order), plus a native fp64 LAPACK LU solve on the same
    cores as context."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import refine
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        threads = 1
    n = a_np.shape[0]
    o = refine.Options(uf="fp16", u="fp32", ur="fp64", m=m, k=k, tau=1e-4, imax=10,
                       berr_target=1e-14, nb=64)
    t0 = time.perf_counter()
    f = refine.factor(a_np, o)
    t1 = time.perf_counter()
    x, info = refine.solve(f, b_np)
    t2 = time.perf_counter()
    t3 = time.perf_counter()
    lu = sla.lu_factor(a_np, check_finite=False)
    xs = sla.lu_solve(lu, b_np, check_finite=False)
    t4 = time.perf_counter()
    rs = b_np - a_np @ xs
    eta_s = float(np.max(np.abs(rs)) / (np.max(np.sum(np.abs(a_np), axis=1)) * np.max(np.abs(xs))
                                        + np.max(np.abs(b_np))))
    return {
        "value": 1.0 / (t2 - t0),
        "unit": "solves/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"oracle factor ({t1 - t0:.1f} s) + solve ({t2 - t1:.1f} s, its {info.its}, "
                   f"status {info.status}) of the benchmark's own randsvd system, n={n} "
                   f"kappa={kappa:g} seed={seed}, one run"),
        "context_lapack_fp64_lu_solve_s": t4 - t3,
        "context_lapack_fp64_berr": eta_s,
    }


def batched_bench(g, count: int, workers: int, oracle: bool):
    """The uneven batch through gmresir_solve_batched (m = 30, k = 10, at most
    300 Arnoldi steps per correction), the first 16 systems also one at a
    time, and the oracle on the batch's first systems (about 20 s)."""
    import torch
    from synthetic import batch_specs, batch_system_torch
    specs = batch_specs(count, 1)
    systems = []
    for sp in specs:
        a, _, b = batch_system_torch(sp)
        systems.append((a, b))
    torch.cuda.synchronize()
    log(f"batched: {count} systems generated on the GPU")
    opts = dict(m=30, k=10, maxit=300)
    t = time.perf_counter()
    out = g.solve_batched(systems, workers=workers, **opts)
    dt = time.perf_counter() - t
    nrhs = sum(len(o[1]) for o in out)
    conv = sum(1 for o in out for i in o[1] if i["status"] == 0)
    st = [o[2] for o in out]
    first = systems[:16]
    t = time.perf_counter()
    g.solve_batched(first, workers=1, **opts)
    d1 = time.perf_counter() - t
    t = time.perf_counter()
    g.solve_batched(first, workers=workers, **opts)
    dw = time.perf_counter() - t
    # the HBM model of one Arnoldi step at order n (the one the library's
    # arnoldi_step class counts): A in fp32 and the fp16 factors once each,
    # plus one read of the basis [C_k V_j] at the cycle's mean j
    steps = 0
    step_bytes = 0.0
    for sp, o in zip(specs, out):
        nn = float(sp["n"])
        for i in o[1]:
            s_ = float(sum(i["its"]))
            steps += s_
            step_bytes += s_ * (6.0 * nn * nn + (8.0 * opts["k"] + 4.0 * (opts["m"] / 2 + 1)
                                                 + 16.0) * nn)
    rec = {"systems": count, "rhs": nrhs, "workers": workers, "seconds": dt,
           "arnoldi_steps": int(steps),
           "persistent_cycles": int(sum(i.get("cycles_persistent", 0) for o in out for i in o[1])),
           "persistent_fallbacks": int(sum(i.get("cycles_fallback", 0)
                                           for o in out for i in o[1])),
           "roofline": {"bound": "hbm", "achieved": step_bytes / dt / 1e9, "peak": 8000.0,
                        "unit": "GB/s", "frac": step_bytes / dt / 1e9 / 8000.0,
                        "what": "Arnoldi-step HBM model summed over every step of the batch, "
                                "over the batch's whole wall time (factorisations, residuals "
                                "and host work included)"},
           "systems_per_s": count / dt, "rhs_per_s": nrhs / dt, "converged_rhs": conv,
           "status_counts": {name: st.count(c) for c, name in
                             ((0, "OK"), (1, "ESINGULAR"), (2, "ERANGE"), (3, "ENOCONV"))},
           "first16_one_at_a_time_s": d1, "first16_batched_s": dw,
           "sum_n3_flop": float(sum(2.0 * sp["n"] ** 3 / 3.0 for sp in specs)),
           "sum_a_bytes": float(sum(8.0 * sp["n"] ** 2 for sp in specs))}
    log(f"batched: {count} systems ({nrhs} right-hand sides) in {dt:.1f} s = "
        f"{count / dt:.2f} systems/s, {conv} right-hand sides converged; first 16: "
        f"{d1:.1f} s one at a time, {dw:.1f} s batched")
    del systems
    if oracle:
        from oracle import refine
        from synthetic import randsvd_problem
        import numpy as np
        o = refine.Options(uf="fp16", u="fp32", ur="fp64", m=30, k=10, tau=1e-4, imax=10,
                           maxit=300, berr_target=1e-14, nb=64)
        # factorisations and right-hand sides in batch order until 20 s have
        # passed; compared per right-hand side (a system's factorisation is
        # charged to its first one)
        t = time.perf_counter()
        rhs = 0
        for sp in specs:
            p = randsvd_problem(sp["n"], sp["kappa"], sp["seed"])
            f = refine.factor(p.a, o)
            gen = np.random.default_rng(sp["seed"])
            for _ in range(sp["nrhs"]):
                refine.solve(f, p.a @ gen.uniform(-1, 1, sp["n"]))
                rhs += 1
                if time.perf_counter() - t > 20.0:
                    break
            if time.perf_counter() - t > 20.0:
                break
        el = time.perf_counter() - t
        rec["cpu_oracle"] = {"value": rhs / el, "unit": "rhs/s", "kind": "oracle",
                             "sample": f"the batch's first {rhs} right-hand sides in order "
                                       f"(systems drawn with numpy), {el:.1f} s"}
        log(f"batched oracle: {rhs} right-hand sides in {el:.1f} s")
    return rec


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported "
              "(multi-GPU sharding is described, not built)", file=sys.stderr)
        return 2
    import torch

    import paper_2201_09827_amd as g
    from synthetic import randsvd_problem_torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 2
    g.load_library()
    dev = torch.device("cuda:0")
    if args.copy_ref_mib > 0:
        src = torch.ones(args.copy_ref_mib * 262144, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log(f"copy reference: {args.copy_ref_mib} MiB read, {args.copy_ref_mib} MiB written")
        del src, dst
    t0 = time.time()
    if args.gen == "gpu":
        a, xt_dev, b = randsvd_problem_torch(args.n, args.kappa, args.seed, dev)
    else:
        from synthetic import randsvd_problem
        p = randsvd_problem(args.n, args.kappa, args.seed)
        a, xt_dev, b = (torch.from_numpy(v).to(dev) for v in (p.a, p.x_true, p.b))
        del p
    torch.cuda.synchronize()
    log(f"generated randsvd(n={args.n}, kappa={args.kappa:g}, seed={args.seed}) on the "
        f"{args.gen.upper()} in {time.time() - t0:.1f} s")
    tau = args.tau if args.tau is not None else (1e-4 if args.u == "fp32" else 1e-8)
    opts = dict(uf=args.uf, u=args.u, ur=args.ur, m=args.m, tau=tau, imax=10,
                berr_target=1e-14)

    def one_step(k, a_, b_, stats=None, mask=0):
        h = g.factor(a_, k=k, timing=mask if stats is not None else 0, **opts)
        x, info = h.solve(b_)
        if stats is not None:
            for r in h.kernel_stats():
                acc = stats.setdefault(r["name"], {"launches": 0, "total_ms": 0.0, "work": 0.0,
                                                   "bound": r["bound"]})
                acc["launches"] += r["launches"]
                acc["total_ms"] += r["total_ms"]
                acc["work"] += r["work"]
        h.free()
        return x, info

    def timed(k, steps, warmup, stats=None, mask=0):
        for _ in range(warmup):
            one_step(k, a, b)
        torch.cuda.synchronize()
        t = time.perf_counter()
        infos = []
        for _ in range(steps):
            x, info = one_step(k, a, b, stats, mask)
            infos.append(info)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        return dt, infos, x

    # one untimed-region step with every kernel class timed picks the class
    # with the largest share (the composite Arnoldi-step class aside); the
    # timed steps then bracket only that class
    survey = {}
    one_step(args.k, a, b, survey, g.timing_mask(g.KERNEL_CLASSES[:8]))
    dom = max(survey, key=lambda kk: survey[kk]["total_ms"])

    def rate(r):
        if r["total_ms"] <= 0:
            return 0.0
        return r["work"] / (r["total_ms"] * 1e-3) / (1e12 if r["bound"] else 1e9)

    kernels = {name: {"launches_per_step": r["launches"], "ms_per_step": r["total_ms"],
                      "avg_us": r["total_ms"] / max(r["launches"], 1) * 1e3,
                      ("TFLOPs" if r["bound"] else "GBps"): rate(r)}
               for name, r in survey.items()}
    # whole Arnoldi steps, timed alone (no nested events): one event pair per
    # step with the separate launches, one per cycle with the persistent
    # launch (its work is that of the steps it took)
    steps_stat = {}
    _, steps_info = one_step(args.k, a, b, steps_stat,
                             g.timing_mask(["arnoldi_step", "arnoldi_cycle"]))
    steps_taken = sum(steps_info["its"])
    # every 8th launch of that class is bracketed (the events' own stream
    # time stays out of most of the timed region)
    kstats = {}
    sample_stride = 8
    dt, infos, x = timed(args.k, args.steps, args.warmup, kstats,
                         g.timing_mask([dom], sample_stride))
    info = infos[-1]
    converged = all(i["status"] == 0 for i in infos)
    ferr = float(torch.max(torch.abs(x - xt_dev)) / torch.max(torch.abs(xt_dev)))
    value = args.steps / dt if converged else 0.0
    log(f"recycled k={args.k}: {dt / args.steps * 1e3:.2f} ms/step status={info['status']} "
        f"its={info['its']} berr={info['berr'][-1]:.2e} factor={info['t_factor_s'] * 1e3:.2f} ms "
        f"solve={info['t_solve_s'] * 1e3:.2f} ms; phases (ms) x0 {info['t_x0_s'] * 1e3:.2f} "
        f"residual {info['t_residual_s'] * 1e3:.2f} precond {info['t_precond_s'] * 1e3:.2f} "
        f"recycle {info['t_recycle_s'] * 1e3:.2f} arnoldi {info['t_arnoldi_s'] * 1e3:.2f}")
    plain = None
    if not args.no_plain:
        dtp, infp, _ = timed(0, args.steps, args.warmup)
        ip = infp[-1]
        plain = {"solves_per_s": (args.steps / dtp) if all(i["status"] == 0 for i in infp) else 0.0,
                 "ms_per_step": dtp / args.steps * 1e3, "status": ip["status"], "its": ip["its"],
                 "berr": ip["berr"][-1]}
        log(f"plain k=0: {dtp / args.steps * 1e3:.2f} ms/step its={ip['its']}")

    # the reuse variant: the recycled pair of the previous refinement step is
    # kept instead of recomputing QR(A-tilde U_k) (same matrix)
    reuse = None
    if not args.no_plain and args.k > 0:
        opts_reuse = dict(opts, reuse_recycle=1)

        def reuse_step():
            h = g.factor(a, k=args.k, **opts_reuse)
            x1, i1 = h.solve(b)
            h.free()
            return i1

        reuse_step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            ir = reuse_step()
        torch.cuda.synchronize()
        dtr = (time.perf_counter() - t) / args.steps
        reuse = {"ms_per_step": dtr * 1e3, "status": ir["status_name"], "its": ir["its"],
                 "berr": ir["berr"][-1], "t_solve_ms": ir["t_solve_s"] * 1e3}
        log(f"recycled k={args.k}, recycled pair reused: {dtr * 1e3:.2f} ms/step its={ir['its']} "
            f"solve={ir['t_solve_s'] * 1e3:.2f} ms")

    # roofline of the dominant class, from its launches in the timed steps
    r = kstats[dom]
    achieved = rate(r)
    mfma = bool(r["bound"])
    peak = FP16_MFMA_PEAK_TFLOPS if mfma else HBM_PEAK_GBS
    # the counter summary was taken on the default workload only
    default_workload = (args.uf, args.u, args.ur, args.n) == ("fp16", "fp32", "fp64", 8192)
    traffic = traffic_for(dom, r["launches"] / args.steps) if default_workload else None
    # the whole factorisation against the fp16 matrix cores (2 n^3 / 3 flops
    # over the factor's wall time), its GEMM-only launches, and one Arnoldi
    # step against HBM (n^2 (s_A + s_f) bytes plus one read of the basis)
    t_lu = sum(i["t_factor_s"] for i in infos) / len(infos)
    lu_flops = 2.0 * args.n ** 3 / 3.0
    lu_peak = FP16_MFMA_PEAK_TFLOPS if args.uf in ("fp16", "bf16") else FP64_MFMA_PEAK_TFLOPS
    gemm = survey.get("lu_gemm")
    st = steps_stat.get("arnoldi_step")
    sc = steps_stat.get("arnoldi_cycle")
    arn = None
    if st and st["launches"] and not (sc and sc["launches"]):
        gbps = st["work"] / (st["total_ms"] * 1e-3) / 1e9
        arn = {"launches": st["launches"], "avg_us": st["total_ms"] / st["launches"] * 1e3,
               "bytes_per_step": st["work"] / st["launches"], "GBps": gbps,
               "frac_hbm": gbps / HBM_PEAK_GBS,
               "ideal_us": st["work"] / st["launches"] / (HBM_PEAK_GBS * 1e9) * 1e6,
               "form": "separate launches, one event pair per step"}
    elif sc and sc["launches"] and steps_taken:
        gbps = sc["work"] / (sc["total_ms"] * 1e-3) / 1e9
        arn = {"launches": sc["launches"], "steps": steps_taken,
               "avg_us": sc["total_ms"] / steps_taken * 1e3,
               "bytes_per_step": sc["work"] / steps_taken, "GBps": gbps,
               "frac_hbm": gbps / HBM_PEAK_GBS,
               "ideal_us": sc["work"] / steps_taken / (HBM_PEAK_GBS * 1e9) * 1e6,
               "form": "persistent cycle: one launch per cycle, its duration (launch, "
                       "residency check and staging included) over the steps it took"}
    roofline = {"bound": "mfma" if mfma else "hbm", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s" if mfma else "GB/s", "frac": achieved / peak,
                "traffic": traffic, "kernel": dom,
                "launches": r["launches"], "avg_us": r["total_ms"] / r["launches"] * 1e3,
                "sampled": f"every {sample_stride}th launch of the class in the timed steps",
                ("algorithmic_flops_per_launch" if mfma else "algorithmic_bytes_per_launch"):
                    r["work"] / r["launches"],
                "lu_whole": {"flops": lu_flops, "t_factor_ms": t_lu * 1e3,
                             "TFLOPs": lu_flops / t_lu / 1e12, "peak": lu_peak,
                             "frac": lu_flops / t_lu / 1e12 / lu_peak},
                "lu_gemm_only": None if not gemm else {
                    "launches_per_step": gemm["launches"], "avg_us": gemm["total_ms"] /
                    max(gemm["launches"], 1) * 1e3, "TFLOPs": rate(gemm),
                    "frac": rate(gemm) / lu_peak,
                    "note": "separate update launches only: with fp16 / bf16 factors the "
                            "rank-64 updates run inside the block-column launches "
                            "(lu_panel) but for the last block column's"},
                "arnoldi_step": arn,
                "kernels_one_step": kernels}
    log(f"dominant kernel class {dom}: {r['launches']} launches, avg "
        f"{r['total_ms'] / r['launches'] * 1e3:.1f} us, {achieved:.2f} "
        f"{'TFLOP/s' if mfma else 'GB/s'} ({achieved / peak * 100:.2f} % of peak); whole LU "
        f"{lu_flops / t_lu / 1e12:.2f} TFLOP/s"
        + (f"; Arnoldi step {arn['avg_us']:.1f} us = {arn['GBps']:.0f} GB/s" if arn else ""))

    # M2: the factorisation amortised over several right-hand sides solved in
    # sequence with the recycle space kept between them (keep_recycle = 1)
    m2 = None
    if args.m2_rhs > 0:
        gx = torch.Generator(device=dev)
        gx.manual_seed(args.seed + 11)
        xs = torch.rand((args.m2_rhs, args.n), generator=gx, dtype=torch.float64,
                        device=dev) * 2.0 - 1.0
        bs = torch.matmul(xs, a.t())                 # row j: A x_j
        m2 = {"rhs": args.m2_rhs}
        for kk in (args.k, 0):
            def m2_step():
                h = g.factor(a, k=kk, keep_recycle=1, **opts)
                xm, im = h.solve(bs.t())
                h.free()
                return xm, im
            m2_step()
            torch.cuda.synchronize()
            t = time.perf_counter()
            m2_reps = max(1, min(args.steps, 3))
            for _ in range(m2_reps):
                xm, im = m2_step()
            torch.cuda.synchronize()
            dtm = (time.perf_counter() - t) / m2_reps
            rr = bs.t() - torch.matmul(a, xm)
            den = (torch.max(torch.sum(torch.abs(a), dim=1)) * torch.max(torch.abs(xm), dim=0).values
                   + torch.max(torch.abs(bs.t()), dim=0).values)
            eta = (torch.max(torch.abs(rr), dim=0).values / den).max().item()
            key = "recycled" if kk else "plain"
            m2[key] = {"k": kk, "ms_per_factor_and_rhs_set": dtm * 1e3,
                       "solves_per_s": args.m2_rhs / dtm if eta <= 1e-14 else 0.0,
                       "max_berr_fp64": eta, "last_rhs_its": im["its"],
                       "last_rhs_recycle_dim": im["recycle_dim"]}
            log(f"M2 k={kk}: {args.m2_rhs} right-hand sides in {dtm * 1e3:.1f} ms "
                f"({args.m2_rhs / dtm:.1f} solves/s), max berr {eta:.2e}, last its {im['its']}")
        if m2.get("plain", {}).get("solves_per_s"):
            m2["recycled_over_plain"] = m2["recycled"]["solves_per_s"] / m2["plain"]["solves_per_s"]
        del xs, bs

    # comparator: plain fp64 LU-based refinement on the same GPU (the vendor
    # LU, rocSOLVER getrf through torch, then fp64 residuals and corrections
    # with the fp64 factors until the same backward-error target)
    comparator = None
    if not args.no_comparator:
        def fp64_ir():
            lu, piv = torch.linalg.lu_factor(a)
            xv = torch.linalg.lu_solve(lu, piv, b.unsqueeze(1))[:, 0]
            na = torch.max(torch.sum(torch.abs(a), dim=1))
            steps_c = 0
            while True:
                rv = b - torch.mv(a, xv)
                eta_c = (torch.max(torch.abs(rv)) / (na * torch.max(torch.abs(xv))
                                                      + torch.max(torch.abs(b)))).item()
                if eta_c <= 1e-14 or steps_c >= 10:
                    return eta_c, steps_c
                xv = xv + torch.linalg.lu_solve(lu, piv, rv.unsqueeze(1))[:, 0]
                steps_c += 1
        try:
            fp64_ir()
            torch.cuda.synchronize()
            t = time.perf_counter()
            creps = max(1, min(args.steps, 5))
            for _ in range(creps):
                eta_c, steps_c = fp64_ir()
            torch.cuda.synchronize()
            dtc = (time.perf_counter() - t) / creps
            comparator = {"what": "fp64 LU (torch.linalg.lu_factor, vendor getrf) + fp64 "
                                  "refinement with lu_solve to backward error 1e-14",
                          "ms_per_solve": dtc * 1e3, "refinement_steps": steps_c,
                          "berr": eta_c,
                          "ours_speedup": (dtc / (dt / args.steps)) if value else None}
            log(f"comparator fp64 LU + refinement: {dtc * 1e3:.2f} ms/solve ({steps_c} steps, "
                f"berr {eta_c:.2e}); ours {dt / args.steps * 1e3:.2f} ms")
        except Exception as exc:  # the comparator is context only
            comparator = {"error": repr(exc)}
            log(f"comparator failed: {exc!r}")

    # the differentiated solve: forward solve, the adjoint A^T lambda = x - y
    # with its own recycle space, dL/dA = -lambda x^T (L = 0.5 ||x - y||^2)
    adjoint = None
    if not args.no_adjoint and args.u == "fp32" and args.ur == "fp64":
        gy = torch.Generator(device=dev)
        gy.manual_seed(args.seed + 7)
        yv = torch.randn(args.n, generator=gy, dtype=torch.float64, device=dev)
        da = torch.empty((args.n, args.n), dtype=torch.float64, device=dev)

        def adj_step():
            h = g.factor(a, k=args.k, **opts)
            x1, i1 = h.solve(b)
            lam, i2 = h.solve_transposed(x1 - yv)
            g.rank1(-1.0, lam, x1, out=da)
            h.free()
            return i1, i2

        adj_step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            i1, i2 = adj_step()
        torch.cuda.synchronize()
        dta = (time.perf_counter() - t) / args.steps
        adjoint = {"ms_per_step": dta * 1e3, "forward_status": i1["status_name"],
                   "forward_its": i1["its"], "adjoint_status": i2["status_name"],
                   "adjoint_its": i2["its"], "adjoint_berr": i2["berr"][-1],
                   "adjoint_solve_ms": i2["t_solve_s"] * 1e3}
        log(f"gradient (factor + solve + adjoint solve + rank-1): {dta * 1e3:.2f} ms/step, "
            f"adjoint {i2['status_name']} its={i2['its']} berr={i2['berr'][-1]:.2e}")
        del da

    outcomes = []
    for ks in [s for s in args.outcomes.split(",") if s.strip()]:
        kap = float(ks)
        a2, xt2, b2 = randsvd_problem_torch(args.n, kap, args.seed, dev)
        for kk in (args.k, 0):
            torch.cuda.synchronize()
            t = time.perf_counter()
            x2, i2 = one_step(kk, a2, b2)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            fe = float(torch.max(torch.abs(x2 - xt2)) / torch.max(torch.abs(xt2)))
            outcomes.append({"kappa2": kap, "k": kk, "status": i2["status_name"],
                             "steps": i2["steps"], "its": i2["its"], "berr": i2["berr"][-1],
                             "ferr": fe, "seconds": el})
            log(f"outcome kappa={kap:g} k={kk}: {i2['status_name']} its={i2['its']} "
                f"berr={i2['berr'][-1]:.2e} in {el:.2f} s")
        del a2, xt2, b2

    prolate = []
    if args.prolate16k:
        from synthetic import prolate_problem_torch
        n3 = 16384
        a3, xt3, b3 = prolate_problem_torch(n3, 0.48, args.seed, dev)
        for uf, u, ur, tau in (("bf16", "fp32", "fp64", 1e-4), ("fp32", "fp64", "dd", 1e-8)):
            for kk in (20, 0):
                torch.cuda.synchronize()
                t = time.perf_counter()
                h3 = g.factor(a3, uf=uf, u=u, ur=ur, m=50, k=kk, tau=tau, imax=10,
                              berr_target=1e-14)
                rec = {"n": n3, "w": 0.48, "uf": uf, "u": u, "ur": ur, "m": 50, "k": kk,
                       "tau": tau}
                if h3.status in (0, 3):
                    x3, i3 = h3.solve(b3)
                    torch.cuda.synchronize()
                    fe = float(torch.max(torch.abs(x3 - xt3)) / torch.max(torch.abs(xt3)))
                    rec.update(status=i3["status_name"], steps=i3["steps"], its=i3["its"],
                               berr=i3["berr"][-1], ferr=fe,
                               t_factor_ms=i3["t_factor_s"] * 1e3,
                               t_solve_ms=i3["t_solve_s"] * 1e3)
                else:
                    rec.update(status=f"factor status {h3.status}")
                rec["seconds"] = time.perf_counter() - t
                h3.free()
                prolate.append(rec)
                log(f"prolate n={n3} ({uf},{u},{ur}) k={kk}: {rec['status']} "
                    f"its={rec.get('its')} berr={rec.get('berr', float('nan')):.2e} "
                    f"in {rec['seconds']:.1f} s")
        del a3, xt3, b3

    batched = None
    if args.batched > 0:
        batched = batched_bench(g, args.batched, args.batched_workers, not args.no_cpu_baseline)

    cpu = None
    if not args.no_cpu_baseline:
        t = time.time()
        cpu = cpu_baseline(a.cpu().numpy(), b.cpu().numpy(), args.kappa, args.seed, args.m,
                           args.k)
        log(f"cpu baseline ({time.time() - t:.1f} s): {cpu['value']:.3g} solves/s; "
            f"{cpu['sample']}; LAPACK fp64 LU solve {cpu['context_lapack_fp64_lu_solve_s']:.2f} s")

    out = {
        "metric": "refined solves/s to backward err 1e-14, recycled vs plain GMRES-IR, n=8192",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.uf}-lu/{args.u}-krylov/{args.ur}-residual",
        "data": "synthetic",
        "config": {
            "workload": f"randsvd mode 3, n={args.n}, kappa2={args.kappa:g}, seed={args.seed}; "
                        f"(uf,u,ur)=({args.uf},{args.u},{args.ur}); RGMRES-IR m={args.m} "
                        f"k={args.k} tau={tau:g}",
            "n": args.n,
            "kappa2": args.kappa,
            "status": info["status"],
            "its": info["its"],
            "steps_ir": info["steps"],
            "berr": info["berr"][-1],
            "ferr": ferr,
            "t_factor_ms": info["t_factor_s"] * 1e3,
            "t_solve_ms": info["t_solve_s"] * 1e3,
            "plain": plain,
            "recycled_over_plain": (value / plain["solves_per_s"]) if plain and plain["solves_per_s"] else None,
            "outcomes": outcomes,
            "outcomes_prolate16k": prolate or None,
            "gradient": adjoint,
            "reuse_recycle": reuse,
            "m2_amortised": m2,
            "comparator_fp64_lu": comparator,
            "phases_ms": {kk: info[kk] * 1e3 for kk in ("t_x0_s", "t_residual_s", "t_precond_s",
                                                         "t_recycle_s", "t_arnoldi_s")},
            "berr_cw": info["berr_cw"][-1],
            "batched": batched,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
