#!/usr/bin/env python3
"""Rand-QLP throughput on one MI355X.

Workload: A = G1 G2 + E, 8000 x 8000 (rank-200 Gaussian product plus iid
noise at 1e-3 of the signal's RMS), fp64, k = 200, p = 10, q = 2 (d = 210).
A is resident in HBM before timing starts.  One step = one full
randqlp_factor call (Gaussian sketch, 2q+3 products with A, 2q+3 panel QRs,
L = R^T).  Throughput = the Section 4.2 flop model / measured time.

Prints one JSON line with the roofline of the dominant kernel (the product
kernel that streams A, timed with HIP events on its stream) and the fp64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Rand-QLP GFLOP/s + % roofline at fixed error; BF16+learned-q vs FP64 plain"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources of the product kernel: a traffic measurement is only reported
# while they are unchanged since the counters were taken.
KERNEL_SOURCES = ["paper_2110_01011_amd/csrc/gemm.hip"]


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_traffic(path):
    """HBM bytes per product launch from a counter summary (key: value lines),
    or None when it is missing or taken on other kernel sources."""
    full = os.path.join(ROOT, path)
    if not os.path.exists(full):
        return None
    kv = {}
    with open(full) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(mib):
    """A plain device copy of known size (for scaling the HBM byte counters)."""
    import torch
    nbytes = mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: 3 copies of {nbytes} bytes (read {nbytes}, write {nbytes} each)")
    del src, dst


def cpu_baseline(A, k, p, q, flops, budget_s=15.0, max_reps=40):
    """The fp64 oracle on the host cores, on whole factorisations of A."""
    from threadpoolctl import threadpool_info
    from oracle import randqlp, rel_error
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
    times, e = [], None
    t_start = time.perf_counter()
    while len(times) < max_reps and (time.perf_counter() - t_start) < budget_s:
        t0 = time.perf_counter()
        Q, L, P = randqlp(A, k, p, q, seed=0)
        times.append(time.perf_counter() - t0)
        if e is None:
            e = rel_error(A, Q, L, P)
        log(f"  oracle rep {len(times)}: {times[-1]:.2f} s")
    t = sorted(times)[len(times) // 2]
    return {"value": flops / t / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(times)} whole fp64 factorisations of the same {A.shape[0]}x{A.shape[1]} "
                      f"matrix (median {t:.2f} s each, Omega generation included)"}, e


def gpu_svd_matrix(n, sigma, gen):
    """A = U diag(sigma) V^T (n x n, fp64, column-major) with Haar U, V from
    the QR of seeded Gaussian matrices, generated on the device."""
    import torch
    U, R = torch.linalg.qr(torch.randn(n, n, dtype=torch.float64, device="cuda", generator=gen))
    U *= torch.sign(torch.diagonal(R))[None, :]
    V, R = torch.linalg.qr(torch.randn(n, n, dtype=torch.float64, device="cuda", generator=gen))
    V *= torch.sign(torch.diagonal(R))[None, :]
    A = (U * sigma[None, :]) @ V.T
    del U, V, R
    return A.t().contiguous().t()


def device_rel_error(A, Q, L, P):
    import torch
    A64 = A.double()
    R = A64 - Q.double() @ (L.double() @ P.double().T)
    return float(torch.linalg.norm(R) / torch.linalg.norm(A64))


def headline(rq, A_c2, k, p, steps, precision="bf16"):
    """bf16 precision form + learned q (randqlp_factor_auto) against the plain
    fp64 method with q = 2, on 8000 x 8000 matrices of the predictor's three
    training families; factorisations per second and errors.  precision is
    the bf16 form used: "bf16" or "bf16x3"."""
    import numpy as np
    import torch
    wpath = os.path.join(ROOT, "paper_2110_01011_amd", "qpredictor.npy")
    if not os.path.exists(wpath):
        return None
    th = torch.from_numpy(np.load(wpath).astype(np.float32)).cuda()
    n = A_c2.shape[0]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2021)
    j = torch.arange(1, n + 1, dtype=torch.float64, device="cuda")
    cases = [("rank-200 + noise", A_c2)]
    log("generating the poly / exp evaluation matrices on the device")
    cases.append(("poly sigma_j = j^-1", gpu_svd_matrix(n, j ** -1.0, gen)))
    cases.append(("exp sigma_j = exp(-(j-1)/100)", gpu_svd_matrix(n, torch.exp(-(j - 1) / 100.0), gen)))
    out = []

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps, r

    for name, A in cases:
        A32 = rq.colmajor(A.float().t().contiguous().t())
        t64, (Q, L, P) = timed(lambda: rq.factor(A, k, p, 2, 0))
        e64 = device_rel_error(A, Q, L, P)
        ta, (Q, L, P, info, ai) = timed(lambda: rq.factor_auto(A32, k, p, 0, th, q_fallback=2,
                                                               precision=precision,
                                                               return_info=True))
        ea = device_rel_error(A, Q, L, P)
        out.append({"matrix": name, "fp64_q2_per_s": round(1.0 / t64, 2),
                    "bf16_learned_per_s": round(1.0 / ta, 2), "speedup": round(t64 / ta, 3),
                    "e_fp64_q2": e64, "e_bf16_learned": ea, "error_ratio": ea / e64,
                    "q_predicted": ai["q_predicted"], "q_used": ai["q_used"],
                    "resumed": ai["resumed"], "judge_ratio": ai["judge_ratio"]})
        log(f"  {out[-1]}")
        del A32
    sp = [c["speedup"] for c in out]
    return {"metric": "factorisations/s, bf16 precision form + learned q vs plain fp64 q = 2",
            "precision": precision, "workload": f"{n}x{n}, k={k} p={p}", "cases": out,
            "speedup_geomean": float(np.exp(np.mean(np.log(sp)))),
            "errors_within_1.05": all(c["error_ratio"] <= 1.05 for c in out)}


def workload_c3(args):
    """Precision form: 20000 x 16000, sigma_i = exp(-i/100) (rank 4000, Haar
    factors), k = 500, p = 20, q = 2 (d = 520); fp64, fp32, bf16, fp16 and
    bf16x3 (bf16 with the split bf16 final projection) forms, each with its
    error against the fp64 form's value for the same matrix."""
    import torch

    import paper_2110_01011_amd as rq
    from paper_2110_01011_amd.metrics import PEAK_TFLOPS, randqlp_flops
    m, n, r, k, p, q = 20000, 16000, 4000, 500, 20, 2
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    log("generating the 20000 x 16000 exp-decay matrix on the device")
    U, _ = torch.linalg.qr(torch.randn(m, r, dtype=torch.float64, device="cuda", generator=gen))
    V, _ = torch.linalg.qr(torch.randn(n, r, dtype=torch.float64, device="cuda", generator=gen))
    sig = torch.exp(-torch.arange(1, r + 1, dtype=torch.float64, device="cuda") / 100.0)
    A64 = rq.colmajor(((U * sig) @ V.T).t().contiguous().t())
    del U, V
    A32 = rq.colmajor(A64.float().t().contiguous().t())
    d = rq.sketch_width(m, n, k, p)
    flops = randqlp_flops(m, n, d, q)
    opt = float(torch.sqrt(torch.sum(sig[d:] ** 2)).item() / torch.linalg.norm(sig).item())
    forms = {}
    for prec in ("f64", "f32", "bf16", "f16", "bf16x3"):
        A = A64 if prec == "f64" else A32
        for _ in range(args.warmup):
            rq.factor(A, k, p, q, 0, precision=prec)
        torch.cuda.synchronize()
        rq.profile_read()
        rq.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            Q, L, P = rq.factor(A, k, p, q, 0, precision=prec)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        rq.profile_enable(False)
        kms, nl, kfl, kby = rq.profile_read()
        e = device_rel_error(A64, Q, L, P)
        forms[prec] = {"ms_per_step": round(t * 1e3, 3), "gflops": round(flops / t / 1e9, 1),
                       "products_avg_ms": round(kms / max(nl, 1), 4),
                       "products_tflops": round(kfl / max(kms, 1e-9) / 1e9, 2),
                       "e": e, "e_over_eckart_young_d": e / opt}
        log(f"  {prec}: {forms[prec]}")
        del Q, L, P
    ref = forms["f64"]["e"]
    for prec in forms:
        forms[prec]["e_over_fp64"] = forms[prec]["e"] / ref
    b = forms["bf16x3"]
    print(json.dumps({
        "metric": "Rand-QLP GFLOP/s, precision form (bf16 products, split bf16 projection) vs fp64",
        "value": b["gflops"],
        "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": b["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": f"exp-decay sigma_i = exp(-i/100), rank {r}, {m}x{n}, "
                               f"k={k} p={p} q={q} (d={d}), precision form",
                   "flops_per_step": flops},
        "forms": forms}), flush=True)


def workload_batched(args):
    """Batched form: 512 matrices, m, n uniform in 256..4096, sigma_j = j^-alpha
    with alpha uniform in [0.5, 3] and Haar factors, k uniform in 8..128,
    p = 10, q = 2, fp32; grouped launches replayed from a HIP graph, tuned
    tile widths; against the same matrices factored one call at a time."""
    import numpy as np
    import torch

    import paper_2110_01011_amd as rq
    from paper_2110_01011_amd.metrics import PEAK_HBM_GBS, PEAK_TFLOPS, randqlp_flops
    count, p, q = 512, 10, 2
    r = np.random.default_rng(0)
    specs = [(int(r.integers(256, 4097)), int(r.integers(256, 4097)), int(r.integers(8, 129)),
              float(r.uniform(0.5, 3.0))) for _ in range(count)]
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    log("generating 512 matrices on the device")
    As = []
    for (m, n, k, a) in specs:
        rr = min(m, n)
        U, _ = torch.linalg.qr(torch.randn(m, rr, device="cuda", generator=gen))
        V, _ = torch.linalg.qr(torch.randn(n, rr, device="cuda", generator=gen))
        s = torch.arange(1, rr + 1, device="cuda", dtype=torch.float32) ** (-a)
        As.append(rq.colmajor(((U * s) @ V.T).t().contiguous().t()))
        del U, V
    torch.cuda.synchronize()
    ks = [sp[2] for sp in specs]
    seeds = list(range(count))
    F, roof = 0.0, 0.0
    for (m, n, k, a) in specs:
        d = min(k + p, m, n)
        f = randqlp_flops(m, n, d, q)
        F += f
        roof += max(f / (PEAK_TFLOPS["f32"] * 1e12), (2 * q + 3) * m * n * 4 / (PEAK_HBM_GBS * 1e9))
    b = rq.Batch(As, ks, p, q, seeds, tune=True)
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    info = b.info()
    t0 = time.perf_counter()
    for A, k, sd in zip(As, ks, seeds):
        rq.factor(A, k, p, q, sd)
    torch.cuda.synchronize()
    tseq = time.perf_counter() - t0
    b.close()
    print(json.dumps({
        "metric": "Rand-QLP GFLOP/s, batched form", "value": round(F / t / 1e9, 1),
        "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "512 matrices, m, n ~ U{256..4096}, sigma_j = j^-alpha, "
                               "alpha ~ U[0.5, 3], k ~ U{8..128}, p=10, q=2, fp32",
                   "flops_per_step": F},
        "roofline": {"bound": "sum over matrices of max(flops / fp32 peak, bytes / HBM peak)",
                     "roof_ms": round(roof * 1e3, 3), "frac": round(roof / t, 4)},
        "sequential_ms": round(tseq * 1e3, 2), "speedup_vs_sequential": round(tseq / t, 2),
        "plan": info}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--size", type=int, default=8000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-headline", action="store_true")
    ap.add_argument("--workload", choices=["c2", "c3", "batched"], default="c2",
                    help="c2 (default): 8000 x 8000 rank-200 + noise; c3: the precision form "
                         "at 20000 x 16000; batched: 512 uneven matrices")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run a plain copy of this size first (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the factorisation of one matrix runs on a "
              "single MI355X (multi-GPU sharding is described, not built).", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        return workload_c3(args)
    if args.workload == "batched":
        return workload_batched(args)

    import numpy as np
    import torch

    import paper_2110_01011_amd as rq
    import workloads as W
    from paper_2110_01011_amd.metrics import PEAK_TFLOPS, randqlp_flops

    m = n = args.size
    r, k, p, q = 200, 200, 10, 2
    d = rq.sketch_width(m, n, k, p)
    log(f"generating {m}x{n} rank-{r} + noise matrix")
    A64, s = W.rank_plus_noise(m, n, r, 1e-3, seed=0)
    tdt = torch.float64 if args.precision == "f64" else torch.float32
    Ad = rq.colmajor(torch.from_numpy(np.ascontiguousarray(A64.T)).to(tdt).cuda().t())
    torch.cuda.synchronize()
    flops = randqlp_flops(m, n, d, q)
    if args.copy_calibration_mib > 0:
        copy_calibration(args.copy_calibration_mib)

    log("warmup")
    for i in range(args.warmup):
        rq.factor(Ad, k, p, q, seed=i)
    torch.cuda.synchronize()
    rq.profile_read()
    rq.profile_enable(True)
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = [t0]
    for i in range(args.steps):
        Q, L, P = rq.factor(Ad, k, p, q, seed=0)  # returns after the call's stream is done
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = np.diff(np.array(marks)) * 1e3
    rq.profile_enable(False)
    kms, launches, kflops, kbytes = rq.profile_read()
    ms = (t1 - t0) * 1e3 / args.steps
    value = flops / (ms * 1e-3) / 1e9

    avg_ms = kms / max(launches, 1)
    achieved = (kflops / max(launches, 1)) / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = None
    if args.size == 8000:
        traffic = read_traffic(f"profiles/gemm_kernel_rank200_8000_{args.precision}_traffic.txt")
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "kernel": "gemm_rem_kernel (fp64 products with A)", "avg_ms": round(avg_ms, 4),
                "flops_per_launch": kflops / max(launches, 1),
                "bytes_per_launch": kbytes / max(launches, 1)}

    Qn, Ln, Pn = (t.double().cpu().numpy() for t in (Q, L, P))
    from numpy.linalg import norm
    e_gpu = float(norm(A64 - Qn @ (Ln @ Pn.T)) / norm(A64))
    head = None
    if not args.no_headline and args.precision == "f64" and args.size == 8000:
        log("headline: bf16 + learned q vs fp64 q = 2")
        head = headline(rq, Ad, k, p, max(3, args.steps // 4), precision="bf16x3")
    cpu = None
    e_orc = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, e_orc = cpu_baseline(A64, k, p, q, flops)

    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"rank-{r} Gaussian product + 1e-3 noise, {m}x{n}, "
                               f"k={k} p={p} q={q} (d={d}), {args.precision}",
                   "m": m, "n": n, "k": k, "p": p, "q": q, "d": d,
                   "flops_per_step": flops},
        "roofline": roofline,
        "step_ms": {"median": round(float(np.median(step_ms)), 4),
                    "min": round(float(step_ms.min()), 4), "max": round(float(step_ms.max()), 4)},
        # whole step against the flop model at the published peak: sum of
        # t_roof over the step's work / measured time per step
        "step_roofline": {"roof_ms": round(flops / (peak * 1e12) * 1e3, 4),
                          "frac": round(flops / (peak * 1e12) / (ms * 1e-3), 4)},
        "cpu_baseline": cpu,
        "error": {"e_gpu": e_gpu, "e_oracle": e_orc,
                  "ratio": (e_gpu / e_orc) if e_orc else None},
        "headline": head,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
