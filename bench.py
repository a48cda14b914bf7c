"""Throughput of the natively periodic FMM on one MI355X.

Workload: N = 256 periodic mesh, uniform tree of depth L = 4 (16^3-cell
leaves), p = 8 gridlet points per axis (512 effective masses per node), G_S1
(Eq. 9); density = lognormal field exp(delta) - mean with delta a Gaussian
random field of spectrum P(k) ~ k^-1.5 and sigma_delta = 2 (seed 5),
synthetic.  One step = one pfmm_solve (every stage of the method: P2M, M2M,
the interaction zones of levels 2..4, L2L, L2P and the near zone) with the
density already resident in HBM.

Prints one JSON line: cells/s (N^3 / time per solve), the roofline of the
dominant kernel (the near zone) from HIP events recorded on the plan's stream
around each stage in profiled solves after the timed steps, the
interaction-zone (M2L) share per level,
and the CPU FP64 oracle timed on a bounded sample of the same workload
(which also checks the GPU potential: sampled cells against the reference
FMM, the full mesh against PM with the same G).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, L, P, GREEN = 256, 4, 8, "S1"
ALPHA, SIGMA, SEED = 1.5, 2.0, 5
METRIC = "cells/s at 256^3 p=8 periodic FMM, L2 err<=1e-4 vs PM; M2L MFMA util"

PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6}
# MI355X peaks (TFLOP/s) of the units each contraction runs on
PEAK_UNIT = {"bf16 mfma": 2516.6, "f64 mfma": 78.6, "f32 valu": 157.3, "f64 valu": 78.6}
FP64_LEVELS = (2, 3)  # coarse levels kept in FP64 (the plan's default)

# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (KiB; the mean of the two profiled solves' launches), scaled by a
# plain 1 GiB copy (read x2.0, write x1.0), keyed by kernel, precision and the
# SHA-1 prefix of the sources they were taken on (the kernel's file and
# plan.hip, which sets the offset order and groups); a changed source reports
# null.  Counters: profiles/pfmm_solve_256cube_L4_p8_*.md (the default: FFT near
# zone, spectral interaction zones), profiles/zones_gemm_256cube_L4_p8_bf16x3.md
# and profiles/near_direct_256cube_L4_p8_*.md.
TRAFFIC = {
    # the leaf level's spectral zones: node transforms, stencil and inverse together
    ("spectral-L4", "bf16x3", "9df7fc67c4f5"): (162065 * 2.0 + 303326 * 1.0) * 1024,
    ("spectral-L4", "fp32", "9df7fc67c4f5"): (162066 * 2.0 + 303328 * 1.0) * 1024,
    ("zones-L4", "bf16x3", "b7aef9891b13"): (252926 * 2.0 + 262144 * 1.0) * 1024,
    ("near", "bf16x3", "b7aef9891b13"): (1188392 * 2.0 + 65536 * 1.0) * 1024,
    # the FFT near zone: leaf transforms, stencil and inverse together
    ("near-fft", "bf16x3", "e64dd98b8f1f"): (677175 * 2.0 + 1179669 * 1.0) * 1024,
    ("near-fft", "fp32", "e64dd98b8f1f"): (677120 * 2.0 + 1179648 * 1.0) * 1024,
    ("near", "fp32", "1503ffb456c4"): (11731340 * 2.0 + 68856 * 1.0) * 1024,
}
KERNEL_SRC = {"bf16x3": ("toeplitz_mfma.hip", "plan.hip"), "fp32": ("toeplitz.hip", "plan.hip")}
SPECTRAL_SRC = ("m2l_spectral.hip", "plan.hip")
NEAR_FFT_SRC = ("near_fft.hip", "plan.hip")


def traffic_bytes(kernel, precision):
    import hashlib
    h = hashlib.sha1()
    srcs = (SPECTRAL_SRC if kernel.startswith("spectral") else
            NEAR_FFT_SRC if kernel == "near-fft" else KERNEL_SRC[precision])
    for name in srcs:
        h.update(open(os.path.join(ROOT, "paper_2011_07099_amd", "csrc", name), "rb").read())
    return TRAFFIC.get((kernel, precision, h.hexdigest()[:12]))


def near_fft_bytes(N, L, kernels=1):
    """Algorithmic HBM bytes of the FFT near zone per solve: the forward pass
    reads the density and writes every leaf's half spectrum ((2s)^2 (s + 1)
    complex FP32 values); per kernel (the potential's, and one per
    acceleration component from the expansion) the 27-point stencil reads and
    writes the spectra once and the inverse reads them and writes a mesh."""
    s = N >> L
    spectra = 8.0 ** L * (2 * s) ** 2 * (s + 1) * 8
    return 4.0 * N ** 3 + spectra + kernels * (3 * spectra + 4.0 * N ** 3)


def algorithmic_flops(N, L, p):
    """Flops of the two contraction steps in their block form (one multiply
    and one add per kernel entry and source point)."""
    s = N >> L
    near = 27 * 2.0 * s ** 6 * 8 ** L
    m2l = 37 * 2.0 * p ** 6 * 64 + sum(189 * 2.0 * p ** 6 * 8 ** l for l in range(3, L + 1))
    return near, m2l


def cpu_baseline(rho64, phi_gpu, n_side=25):
    """The CPU FP64 oracle (reference FMM, NumPy) on the n_side^3 lattice of
    cells i_k = k (N // n_side) + N // (2 n_side) + 1 (15625 cells: about
    10 s on 16 threads), timed; the same targets check the GPU result, and PM with
    the same G checks the full mesh."""
    from oracle import conv, fmm as ofmm
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    k = np.arange(n_side) * (N // n_side) + N // (2 * n_side) + 1
    tg = np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3)
    t0 = time.perf_counter()
    ref = ofmm.fmm(rho64, L, P, GREEN, targets=tg)
    dt = time.perf_counter() - t0
    got = phi_gpu[tg[:, 0], tg[:, 1], tg[:, 2]]
    sampled = float(np.max(np.abs(got - ref)) / np.max(np.abs(phi_gpu)))
    t1 = time.perf_counter()
    pm = conv.pm(rho64, GREEN)
    pm_s = time.perf_counter() - t1
    a = phi_gpu - phi_gpu.mean()
    b = pm - pm.mean()
    acc = {
        "sampled_max_err_vs_fp64_fmm": sampled,
        "l2_rel_vs_pm": float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))),
        "lmax_rel_vs_pm": float(np.max(np.abs(a - b)) / np.max(np.abs(b))),
    }
    base = {"value": len(tg) / dt, "unit": "cells/s", "cores": int(cores), "kind": "oracle",
            "sample": "reference FMM (oracle/fmm.py, FP64 NumPy) at %d cells (%d^3 lattice) of "
                      "the same 256^3 field, including its full upward pass and coarse levels; "
                      "%.1f s" % (len(tg), n_side, dt)}
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    context = {"pm_fft_s": pm_s, "pm_cells_per_s": N ** 3 / pm_s,
               "pm_note": "PM with the same G (the FP64 FFT convolution the FMM approximates), "
                          "NumPy FFT on the host, table included",
               "cpu_model": cpu_model, "os_cpu_count": os.cpu_count()}
    return base, acc, context


def copy_reference():
    """Plain streaming kernels over 1 GiB: a device-to-device copy and an
    elementwise kernel that reads one 1 GiB array and writes another."""
    import torch
    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(2):
        b.copy_(a)
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    print("copied 2 x 2 x %d bytes" % (4 * n), flush=True)


def batch_bench(args):
    """Batch of 128 independent fields (N in {32, 64, 128}, p in {4, 6, 8},
    lognormal with alpha = 2, sigma_delta ~ U(0.5, 2), seed 1000 + i, L = 3,
    G_S1) solved by one graph launch; fields/s over K launches.  Plans are in
    the --precision given, with the --near zone route (FFT: per-leaf
    transforms in the graph; direct, split: near zones with 8^3-cell
    sub-blocks on the BF16 matrix cores)."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.pfmm import Batch, Plan

    specs = fields.batch_specs(128, seed=4)
    plans, rhos, phis, host = [], [], [], []
    for sp in specs:
        rho = fields.lognormal(sp["N"], sp["alpha"], sp["sigma_delta"], seed=sp["seed"])
        host.append(rho.astype(np.float32))
        plans.append(Plan(sp["N"], 3, sp["p"], GREEN, precision=args.precision, near=args.near,
                          m2l=args.m2l))
        rhos.append(torch.from_numpy(host[-1]).cuda())
        phis.append(torch.empty_like(rhos[-1]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = Batch(plans, rhos, phis)
    create_s = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.solve()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        batch.solve()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    info = batch.info()
    cells = sum(sp["N"] ** 3 for sp in specs)
    flops = sum(sum(algorithmic_flops(sp["N"], 3, sp["p"])) for sp in specs)
    out = {
        "metric": "fields/s, batch of 128 mixed periodic-FMM fields in one graph launch",
        "value": len(specs) / (ms * 1e-3), "unit": "fields/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        # FFT near zones and spectral zones use no split bf16 products
        "dtype": "f32+f64" if (args.near == "fft" and args.m2l == "spectral") else args.precision,
        "data": "synthetic",
        "config": {"workload": "128 lognormal fields, N in {32,64,128}, p in {4,6,8}, "
                               "sigma_delta~U(0.5,2), alpha=2, L=3, G_S1",
                   "cells": cells, "items": info["items"], "create_s": create_s,
                   "near": args.near, "m2l": args.m2l},
        "tuning": info["groups"],
        "achieved_tflops": flops / (ms * 1e-3) / 1e12,
    }
    if not args.no_cpu_baseline:
        from oracle import conv
        errs = []
        for sp, rho, phi in zip(specs, host, phis):
            pm = conv.pm(rho.astype(np.float64), GREEN)
            a = phi.cpu().numpy().astype(np.float64)
            a, b = a - a.mean(), pm - pm.mean()
            errs.append(float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))))
        out["per_field_l2_vs_pm"] = {"max": max(errs), "median": float(np.median(errs)),
                                     "by_p": {str(p): max(e for e, sp in zip(errs, specs)
                                                          if sp["p"] == p) for p in (4, 6, 8)}}
    batch.close()
    for pl in plans:
        pl.close()
    print(json.dumps(out), flush=True)


def learned_bench(args):
    """Train the table-correction network on 512 seeded 64^3 lognormal fields
    (alpha = 2, sigma_delta = 1, p = 6, L = 3, seeds 10000 + i) on the GPU,
    then evaluate at 128^3, p = 6 on 16 unseen fields (seeds 20000 + i) with
    BF16 inference, against G_S1 without correction; the reference is PM with
    G_S1 from the CPU oracle."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.learned import train
    from paper_2011_07099_amd.pfmm import Plan
    t0 = time.perf_counter()
    w, hist = train(N=64, L=3, p=6, n_fields=512, epochs=args.epochs, batch=16, lr=3e-4,
                    seed0=10000)
    train_s = time.perf_counter() - t0
    out = {"metric": "learned G correction: mean relative L2^2 vs PM(G_S1), 128^3 p=6 unseen",
           "unit": "relative L2^2", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "train 512 x 64^3 lognormal (alpha=2, sigma_delta=1) p=6 L=3; "
                                  "evaluate 16 x 128^3 unseen seeds, bf16 inference",
                      "epochs": args.epochs},
           "train_loss": hist, "train_s": train_s}
    if args.no_cpu_baseline:
        print(json.dumps(out), flush=True)
        return
    from oracle import conv
    errs = {"G_S1": [], "learned": []}
    plans = {"G_S1": Plan(128, 3, 6, "S1"), "learned": Plan(128, 3, 6, "S1")}
    plans["learned"].set_learned(w, bf16=True)
    for i in range(16):
        rho = fields.lognormal(128, 2.0, 1.0, seed=20000 + i).astype(np.float32)
        r = torch.from_numpy(rho).cuda()
        pm = conv.pm(rho.astype(np.float64), GREEN)
        b = pm - pm.mean()
        for k, pl in plans.items():
            phi = torch.empty_like(r)
            pl.solve(r, phi)
            a = phi.cpu().numpy().astype(np.float64)
            a = a - a.mean()
            errs[k].append(float(np.sum((a - b) ** 2) / np.sum(b ** 2)))
    for pl in plans.values():
        pl.close()
    out["eval"] = {k: float(np.mean(v)) for k, v in errs.items()}
    out["value"] = out["eval"]["learned"]
    out["gain"] = out["eval"]["G_S1"] / out["eval"]["learned"]
    out["higher_is_better"] = False
    print(json.dumps(out), flush=True)


def table_bench(args):
    """Grid-valued interaction-zone tables (one free relative correction per
    cube-symmetry orbit of table entries and level) fitted by conjugate
    gradients on the training workload of the learned network (512 seeded
    64^3 lognormal fields, alpha = 2, sigma_delta = 1, p = 6, L = 3, seeds
    10000 + i), then evaluated at 128^3, p = 6 on 16 unseen fields (seeds
    20000 + i) against G_S1; the reference is PM with G_S1 from the CPU
    oracle."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.learned import fit_table
    from paper_2011_07099_amd.pfmm import Plan
    t0 = time.perf_counter()
    d, hist = fit_table(N=64, L=3, p=6, n_fields=512, iters=args.iters, seed0=10000,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    fit_s = time.perf_counter() - t0
    out = {"metric": "grid-valued G tables: mean relative L2^2 vs PM(G_S1), 128^3 p=6 unseen",
           "unit": "relative L2^2", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "fit 512 x 64^3 lognormal (alpha=2, sigma_delta=1) p=6 L=3 by "
                                  "conjugate gradients; evaluate 16 x 128^3 unseen seeds",
                      "iterations": args.iters, "free_values": int(d.size)},
           "train_loss": hist, "fit_s": fit_s, "max_abs_delta": float(np.abs(d).max())}
    if args.no_cpu_baseline:
        print(json.dumps(out), flush=True)
        return
    from oracle import conv
    errs = {"G_S1": [], "grid": []}
    plans = {"G_S1": Plan(128, 3, 6, "S1"), "grid": Plan(128, 3, 6, "S1")}
    plans["grid"].set_table(d)
    for i in range(16):
        rho = fields.lognormal(128, 2.0, 1.0, seed=20000 + i).astype(np.float32)
        r = torch.from_numpy(rho).cuda()
        pm = conv.pm(rho.astype(np.float64), GREEN)
        b = pm - pm.mean()
        for k, pl in plans.items():
            phi = torch.empty_like(r)
            pl.solve(r, phi)
            a = phi.cpu().numpy().astype(np.float64)
            a = a - a.mean()
            errs[k].append(float(np.sum((a - b) ** 2) / np.sum(b ** 2)))
    for pl in plans.values():
        pl.close()
    out["eval"] = {k: float(np.mean(v)) for k, v in errs.items()}
    out["value"] = out["eval"]["grid"]
    out["gain"] = out["eval"]["G_S1"] / out["eval"]["grid"]
    out["higher_is_better"] = False
    print(json.dumps(out), flush=True)


def m2l_bench(args):
    """The interaction zones (Eq. 6) three ways on the headline mesh (256^3,
    L = 4, G_S1, the same density): the block-Toeplitz GEMM of this library
    (FP32 portable kernel, and split BF16 on the matrix cores at p = 8), the
    HPM form the paper runs (Sec. 2: per target node one FFT convolution of
    its zone's effective masses with G, rocFFT), and the spectral stencils
    (per-node transforms, FP64), at p = 4, 6, 8.  Levels
    2-3 are FP64 in every variant (FP64 matrix cores at p = 8, FP64
    transforms for the FFT).  Per-level medians of the profiled stage times
    over `steps` solves; `value` is the FFT-to-GEMM time ratio of all levels
    at p = 8 with the default (split) precision."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.pfmm import Plan
    rho = torch.from_numpy(fields.lognormal(N, ALPHA, SIGMA, seed=SEED).astype(np.float32)).cuda()
    phi = torch.empty_like(rho)
    res = {}
    for p in (4, 6, 8):
        for m2l, prec in (("gemm", "fp32"), ("gemm", "bf16x3"), ("fft", "fp32"),
                          ("spectral", "fp32")):
            if prec == "bf16x3" and p != 8:
                continue  # the split matrix-core kernel serves p = 8
            with Plan(N, L, p, GREEN, precision=prec, m2l=m2l) as pl:
                for _ in range(max(args.warmup, 1)):
                    pl.solve(rho, phi)
                pl.set_profile(True)
                per = []
                for _ in range(max(args.steps, 1)):
                    pl.solve(rho, phi)
                    per.append(pl.level_times("m2l"))
                torch.cuda.synchronize()
            lv = {str(l): float(np.median([x[l] for x in per])) for l in range(2, L + 1)}
            key = "p%d %s %s" % (p, m2l, prec)
            res[key] = {"ms_per_level": lv, "ms_total": float(sum(lv.values()))}
            print("m2l", key, res[key], file=sys.stderr, flush=True)
    ratio = res["p8 fft fp32"]["ms_total"] / res["p8 gemm bf16x3"]["ms_total"]
    out = {"metric": "interaction-zone time, HPM FFT convolution / block-Toeplitz GEMM, p=8",
           "value": ratio, "unit": "ratio", "higher_is_better": True, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
           "config": {"workload": "256^3 L=4 G_S1 lognormal (alpha=1.5, sigma_delta=2, seed 5); "
                                  "M2L of levels 2-4, p = 4, 6, 8"},
           "spectral_vs_gemm_p8": res["p8 spectral fp32"]["ms_total"] / res["p8 gemm bf16x3"]["ms_total"],
           "results": res}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="headline", choices=["headline", "batch", "learned", "m2l", "table"])
    ap.add_argument("--epochs", type=int, default=2, help="training epochs (learned workload)")
    ap.add_argument("--accel", default="none", choices=["none", "fd4", "expansion"],
                    help="also form accelerations (headline workload): by differences of "
                         "the potential or from the expansion")
    ap.add_argument("--near", default="fft", choices=["direct", "fft"],
                    help="leaf near zone by direct summation or by FFT convolution "
                         "(headline and batch workloads)")
    ap.add_argument("--m2l", default="spectral", choices=["gemm", "spectral"],
                    help="interaction zones by block-Toeplitz GEMM or spectral stencils "
                         "(headline and batch workloads)")
    ap.add_argument("--iters", type=int, default=20,
                    help="conjugate-gradient iterations (table workload)")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run a plain 1 GiB device copy (3 times): the reference that "
                         "scales FETCH_SIZE / WRITE_SIZE counters to bytes")
    args = ap.parse_args()
    if args.copy_ref:
        copy_reference()
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); a multi-GPU "
              "sharding by octants is not built here", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "learned":
        learned_bench(args)
        return
    if args.workload == "m2l":
        m2l_bench(args)
        return
    if args.workload == "table":
        table_bench(args)
        return

    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.pfmm import Plan

    rho64 = fields.lognormal(N, ALPHA, SIGMA, seed=SEED)
    rho32 = rho64.astype(np.float32)
    dev = torch.device("cuda:0")
    rho = torch.from_numpy(rho32).to(dev)
    phi = torch.empty_like(rho)
    stream = torch.cuda.current_stream(dev)
    plan = Plan(N, L, P, GREEN, precision=args.precision, stream=stream,
                accel="expansion" if args.accel == "expansion" else "fd4", near=args.near,
                m2l=args.m2l)
    acc = (torch.empty((3, N, N, N), dtype=torch.float32, device=dev)
           if args.accel != "none" else None)
    for _ in range(args.warmup):
        plan.solve(rho, phi, acc)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    for _ in range(args.steps):
        plan.solve(rho, phi, acc)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end) / args.steps
    # stage times from separate profiled solves (events around every stage;
    # the near zone then runs before the tree on the plan stream instead of
    # beside it), after the timed region
    plan.set_profile(True)
    for _ in range(min(args.steps, 10)):
        plan.solve(rho, phi, acc)
    stages = plan.stage_times()
    m2l_levels = plan.level_times("m2l")
    plan.close()

    near_flops, m2l_flops = algorithmic_flops(N, L, P)
    if args.accel == "expansion":
        near_flops *= 4  # the potential's near zone and one per acceleration component
    peak = PEAK_TFLOPS[args.precision]
    near_ms = stages["near"][0]
    m2l_ms = stages["m2l"][0]
    near_tf = near_flops / (near_ms * 1e-3) / 1e12
    m2l_tf = m2l_flops / (m2l_ms * 1e-3) / 1e12
    near_unit, near_products = ("bf16 mfma", 3) if args.precision == "bf16x3" else ("f32 valu", 1)
    per_level = {}
    F = (2 * P) ** 2 * (P + 1)  # frequencies per node of the spectral zones
    for lv, lms in sorted(m2l_levels.items()):
        fl = (37 if lv == 2 else 189) * 2.0 * P ** 6 * 8 ** lv
        if args.m2l == "spectral":
            # one complex FP64 multiply-add per zone offset, target node and frequency
            fl = (37 if lv == 2 else 189) * 8.0 * F * 8 ** lv
            tf = fl / (lms * 1e-3) / 1e12
            per_level[str(lv)] = {"ms": lms, "unit": "f64 valu", "products": 1, "achieved": tf,
                                  "issued": tf, "peak": PEAK_UNIT["f64 valu"],
                                  "frac": tf / PEAK_UNIT["f64 valu"], "flops": fl}
            continue
        if lv in FP64_LEVELS:
            unit, products = "f64 mfma", 1
        elif args.precision == "bf16x3":
            unit, products = "bf16 mfma", 6
        else:
            unit, products = "f32 valu", 1
        tf = fl / (lms * 1e-3) / 1e12
        per_level[str(lv)] = {"ms": lms, "unit": unit, "products": products,
                              "achieved": tf, "issued": tf * products, "peak": PEAK_UNIT[unit],
                              "frac": tf * products / PEAK_UNIT[unit]}
    if args.near == "direct":
        # the direct near zone dominates
        roofline = {"bound": "mfma" if near_unit.endswith("mfma") else "alu",
                    "achieved": near_tf, "peak": peak, "unit": "TFLOP/s",
                    "frac": near_tf / peak, "traffic": traffic_bytes("near", args.precision),
                    "kernel": "near zone (%d launch/step, %.3f ms)" % (
                        4 if args.accel == "expansion" else 1, near_ms),
                    "unit_used": near_unit, "products": near_products,
                    "issued_frac": near_tf * near_products / peak}
    elif args.near == "fft" and near_ms > per_level[str(L)]["ms"]:
        # the FFT near zone (leaf transforms, stencil, inverse) is the longest stage
        nbytes = near_fft_bytes(N, L, 4 if args.accel == "expansion" else 1)
        gbs = nbytes / (near_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                    "frac": gbs / 8000.0,
                    "traffic": traffic_bytes("near-fft", args.precision) if args.accel != "expansion"
                    else None,
                    "kernel": "near zone by FFT (3 launches/step: leaf transforms, stencil, "
                              "inverse; %.3f ms)" % near_ms,
                    "algorithmic_bytes": nbytes}
    elif args.m2l == "spectral":
        # the leaf level's spectral zones (transforms, stencil, inverse) dominate
        lv = per_level[str(L)]
        roofline = {"bound": "alu", "achieved": lv["achieved"], "peak": lv["peak"],
                    "unit": "TFLOP/s", "frac": lv["frac"],
                    "traffic": traffic_bytes("spectral-L%d" % L, args.precision),
                    "kernel": "level-%d interaction zones, spectral stencil (3 launches/step: "
                              "node transforms, stencil, inverse; %.3f ms)" % (L, lv["ms"]),
                    "unit_used": "f64 valu", "products": 1, "issued_frac": lv["frac"]}
    else:
        # with the near zone by FFT the leaf level's interaction zones dominate
        lv = per_level[str(L)]
        roofline = {"bound": "mfma" if lv["unit"].endswith("mfma") else "alu",
                    "achieved": lv["achieved"], "peak": PEAK_UNIT[lv["unit"]], "unit": "TFLOP/s",
                    "frac": lv["achieved"] / PEAK_UNIT[lv["unit"]],
                    "traffic": traffic_bytes("zones-L%d" % L, args.precision),
                    "kernel": "level-%d interaction zones (1 launch/step, %.3f ms)" % (L, lv["ms"]),
                    "unit_used": lv["unit"], "products": lv["products"],
                    "issued_frac": lv["frac"]}
    out = {
        "metric": METRIC,
        "value": N ** 3 / (ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # with the FFT near zone and spectral zones no step uses the split
        # bf16 products: FP32 near zone and mesh transfers, FP64 zones
        "dtype": "f32+f64" if (args.near == "fft" and args.m2l == "spectral") else args.precision,
        "data": "synthetic",
        "config": {"workload": "periodic FMM, 256^3 lognormal density (P(k)~k^-1.5, "
                               "sigma_delta=2, seed 5), L=4 (16^3-cell leaves), p=8, G_S1",
                   "N": N, "L": L, "p": P, "green": GREEN, "precision": args.precision,
                   **({"accel": args.accel} if args.accel != "none" else {}),
                   **({"near": args.near} if args.near != "direct" else {}),
                   **({"m2l": args.m2l} if args.m2l != "gemm" else {})},
        "roofline": roofline,
        "m2l": {"method": args.m2l,
                "achieved": (sum(v["flops"] for v in per_level.values()) / (m2l_ms * 1e-3) / 1e12
                             if args.m2l == "spectral" else m2l_tf),
                "unit": "TFLOP/s", "ms": m2l_ms,
                "launches": stages["m2l"][1], "levels": per_level},
        "stages_ms": {k: v[0] for k, v in stages.items()},
    }
    if args.near == "fft":
        nb = near_fft_bytes(N, L, 4 if args.accel == "expansion" else 1)
        gbs = nb / (near_ms * 1e-3) / 1e9
        out["near"] = {"method": "fft", "bound": "hbm", "achieved": gbs, "peak": 8000.0,
                       "unit": "GB/s", "frac": gbs / 8000.0, "bytes": nb, "ms": near_ms}
    else:
        out["near"] = {"method": "direct", "achieved": near_tf, "unit": "TFLOP/s", "ms": near_ms}
    if not args.no_cpu_baseline:
        base, acc, context = cpu_baseline(rho32.astype(np.float64),
                                          phi.cpu().numpy().astype(np.float64))
        out["cpu_baseline"] = base
        out["accuracy"] = acc
        out["cpu_context"] = context
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
