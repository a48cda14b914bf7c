"""Throughput of the natively periodic FMM on one MI355X.

Workload: N = 256 periodic mesh, uniform tree of depth L = 4 (16^3-cell
leaves), p = 8 gridlet points per axis (512 effective masses per node), G_S1
(Eq. 9); density = lognormal field exp(delta) - mean with delta a Gaussian
random field of spectrum P(k) ~ k^-1.5 and sigma_delta = 2 (seed 5),
synthetic.  One step = one pfmm_solve (every stage of the method: P2M, M2M,
the interaction zones of levels 2..4, L2L, L2P and the near zone) with the
density already resident in HBM.

Prints one JSON line:
  - cells/s (N^3 / time per solve) over the timed steps, run as any solve
    runs (the near zone on a second stream beside the tree);
  - per-kernel durations from HIP events the plan records around each
    kernel on its stream: in those timed steps ("live"), and in a second
    timed run of the same number of steps with every stage alone on the
    device ("serial"); the roofline of the dominant single kernel uses its
    serial duration, with its live one beside it;
  - m2l_mfma: the interaction zones as block-Toeplitz GEMMs on the matrix
    cores, timed in the same run on the same density, per level against the
    peak of the matrix-core instruction it uses;
  - the CPU FP64 oracle timed on a bounded sample of the same workload (which
    also checks the GPU potential: sampled cells against the reference FMM,
    the full mesh against PM with the same G).
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
# MI355X peaks (TFLOP/s) of the units each kernel runs on.  The library
# compiles every kernel with packed FP32 instructions disabled, yet the FP32
# vector peak of 157.3 stays reachable: gfx950 issues the two-operand FP32
# multiply-add (v_fmac_f32 e32, all operands in vector registers) at twice
# the rate of the three-operand form.  The FP32 direct near zone's counters
# show it: 3.70e10 VALU instructions in 9.6e7 cycles on 1024 SIMDs, 1.5 per
# four cycles, which one instruction per four cycles could not give.  FP64
# has no such doubling: 78.6.
PEAK_UNIT = {"bf16 mfma": 2516.6, "f64 mfma": 78.6, "f32 valu": 157.3, "f64 valu": 78.6}
FP64_LEVELS = (2, 3)  # coarse levels kept in FP64 (the plan's default at L = 4)

# HBM bytes per launch of a kernel (rocprofv3 --pmc FETCH_SIZE x 2 + WRITE_SIZE
# x 1, KiB per dispatch scaled to bytes by a plain 1 GiB copy) in the serial
# solve of the bench route at 256^3, L = 4, p = 8, keyed by the kernel's name
# in the bench line and the SHA-1 prefix of the sources it was taken on (its
# file and plan.hip); another route or a changed source reports null until the
# counters are taken again.
TRAFFIC = {
    ("near leaf transforms", "82ec6b7cc7ad"): 637840080,
    ("near stencil", "82ec6b7cc7ad"): 1215762554,
    ("near inverse transforms", "82ec6b7cc7ad"): 655559559,
    ("p2m", "a91f476d7c39"): 75561437,
    ("l2p", "a91f476d7c39"): 143449256,
    ("m2l L4 node transforms", "b9145110233e"): 84136325,
    ("m2l L4 stencil", "b9145110233e"): 163756213,
    ("m2l L4 inverse transforms", "b9145110233e"): 92446448,
    ("m2l L3 stencil", "b9145110233e"): 63194849,
    ("m2l L2 stencil", "b9145110233e"): 9186973,
}
TRAFFIC_ROUTE = {"precision": "bf16x3", "near": "fft", "m2l": "spectral", "accel": "none",
                 "zones": "fp32", "N": 256, "L": 4, "p": 8}
KERNEL_SRC = {"m2l": ("m2l_spectral.hip", "plan.hip"), "near": ("near_fft.hip", "plan.hip"),
              "p2m": ("updown.hip", "plan.hip"), "l2p": ("updown.hip", "plan.hip")}


def source_key():
    """{kernel family: SHA-1 prefix of its sources}."""
    import hashlib
    out = {}
    for fam, names in KERNEL_SRC.items():
        h = hashlib.sha1()
        for name in names:
            h.update(open(os.path.join(ROOT, "paper_2011_07099_amd", "csrc", name), "rb").read())
        out[fam] = h.hexdigest()[:12]
    return out


def traffic_bytes(kernel, route):
    """Counted HBM bytes of one launch of `kernel`, or None when the route or
    the kernel's sources differ from those the counters were taken on."""
    fam = kernel.split()[0]
    if fam not in KERNEL_SRC or route != TRAFFIC_ROUTE:
        return None
    return TRAFFIC.get((kernel, source_key()[fam]))


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
    context = {"_pm": pm, "pm_fft_s": pm_s, "pm_cells_per_s": N ** 3 / pm_s,
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
    """Train the table-correction network on seeded 64^3 lognormal fields
    (alpha = 2, sigma_delta = 1, p = 6, L = 3, seeds 10000 + i; 512 by
    default) on the GPU: the output layer solved exactly on the training
    fields (the loss is quadratic in it), the ridge chosen on 16 further
    fields with the BF16 inference tables; with --epochs > 0 Adam epochs on
    every weight follow.  Then evaluate at 128^3, p = 6 on 16 unseen fields
    (seeds 20000 + i) with BF16 inference, against G_S1 without correction;
    the reference is PM with G_S1 from the CPU oracle."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.learned import fit_output, train
    from paper_2011_07099_amd.pfmm import Plan
    t0 = time.perf_counter()
    w, info = fit_output(N=64, L=3, p=6, n_fields=args.fields, n_valid=16, seed0=10000,
                         log=lambda m: print(m, file=sys.stderr, flush=True))
    hist = []
    if args.epochs > 0:
        w, hist = train(N=64, L=3, p=6, n_fields=args.fields, epochs=args.epochs, batch=16,
                        lr=3e-5, seed0=10000, theta=w)
    train_s = time.perf_counter() - t0
    out = {"metric": "learned G correction: mean relative L2^2 vs PM(G_S1), 128^3 p=6 unseen",
           "unit": "relative L2^2", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "train %d x 64^3 lognormal (alpha=2, sigma_delta=1) p=6 L=3: "
                                  "exact output layer, then %d Adam epochs; evaluate 16 x 128^3 "
                                  "unseen seeds, bf16 inference" % (args.fields, args.epochs)},
           "fit": {k: v for k, v in info.items() if k != "fits"}, "adam_loss": hist,
           "train_s": train_s}
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


def gstar_bench(args):
    """G_* as one grid-valued function everywhere (near zone, every level's
    tables, the PM solution; Eq. 8's setting, the gridlet equal to the leaf's
    cells): fitted by conjugate gradients on 32 seeded 64^3 lognormal fields
    (alpha = 2, sigma_delta = 1, L = 4, p = 4, seeds 10000 + i), then the FMM
    against PM, both with the same G, on 16 unseen fields (seeds 20000 + i),
    for G_S1 and the fitted G_*; PM is the library's exact periodic
    convolution with that G."""
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.learned import fit_gstar
    from paper_2011_07099_amd.pfmm import Plan
    N, L, p = 64, 4, 4
    t0 = time.perf_counter()
    d, hist = fit_gstar(N=N, L=L, p=p, n_fields=32, iters=args.iters, seed0=10000,
                        log=lambda m: print(m, file=sys.stderr, flush=True))
    fit_s = time.perf_counter() - t0
    errs = {"G_S1": [], "G_*": []}
    with Plan(N, L, p, GREEN) as pl:
        for i in range(16):
            rho = fields.lognormal(N, 2.0, 1.0, seed=20000 + i).astype(np.float32)
            r = torch.from_numpy(rho).cuda()
            for k, delta in (("G_S1", None), ("G_*", d)):
                pl.set_gstar(delta)
                errs[k].append(pl.gstar_loss(r))
    out = {"metric": "G_* everywhere (Eq. 8): mean relative L2^2 of FMM vs PM, both with G_*, "
                     "64^3 p=4 L=4 unseen",
           "unit": "relative L2^2", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "fit 32 x 64^3 lognormal (alpha=2, sigma_delta=1) p=4 L=4 by "
                                  "conjugate gradients; evaluate 16 unseen seeds",
                      "iterations": args.iters, "free_values": int(d.size)},
           "train_loss": hist, "fit_s": fit_s, "max_abs_delta": float(np.abs(d).max())}
    out["eval"] = {k: float(np.mean(v)) for k, v in errs.items()}
    out["value"] = out["eval"]["G_*"]
    out["gain"] = out["eval"]["G_S1"] / out["eval"]["G_*"]
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--precision", default="bf16x3", choices=sorted(PEAK_TFLOPS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mfma", action="store_true",
                    help="skip the GEMM-route interaction zones timed for the matrix-core "
                         "utilisation (headline workload)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "batch", "learned", "m2l", "table", "gstar"])
    ap.add_argument("--epochs", type=int, default=0,
                    help="Adam epochs after the exact output-layer fit (learned workload)")
    ap.add_argument("--fields", type=int, default=512,
                    help="training fields (learned workload)")
    ap.add_argument("--accel", default="none", choices=["none", "fd4", "expansion"],
                    help="also form accelerations (headline workload): by differences of "
                         "the potential or from the expansion")
    ap.add_argument("--near", default="fft", choices=["direct", "fft"],
                    help="leaf near zone by direct summation or by FFT convolution "
                         "(headline and batch workloads)")
    ap.add_argument("--zones", default="fp32", choices=["fp32", "fp64"],
                    help="arithmetic of the 16^3 leaf level's spectral zone stencil: FP32 "
                         "columns with FP64 totals (PFMM_OPT_ZONES_FP32) or FP64")
    ap.add_argument("--m2l", default="spectral", choices=["gemm", "spectral"],
                    help="interaction zones by block-Toeplitz GEMM or spectral stencils "
                         "(headline and batch workloads)")
    ap.add_argument("--iters", type=int, default=20,
                    help="conjugate-gradient iterations (table and gstar workloads)")
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
    if args.workload == "gstar":
        gstar_bench(args)
        return

    headline(args)


def kernel_table(plan, L, near_fft, spectral):
    """{name: (ms, level, stage, part)} of the timed kernels of the recent
    profiled solves: each stage as a whole, the spectral zones and the FFT
    near zone kernel by kernel."""
    out = {}
    st = plan.stage_times()
    for stage in ("p2m", "l2p", "fd4"):
        if st[stage][1]:
            out[stage] = (st[stage][0], 0, stage, 0)
    for stage in ("m2m", "l2l"):
        for lv, ms in plan.level_times(stage).items():
            out["%s L%d" % (stage, lv)] = (ms, lv, stage, 0)
    names = ("node transforms", "stencil", "inverse transforms")
    for lv in range(2, L + 1):
        parts = plan.kernel_times("m2l", lv)
        if spectral:
            for k, ms in enumerate(parts):
                out["m2l L%d %s" % (lv, names[k])] = (ms, lv, "m2l", k)
        elif parts:
            out["m2l L%d" % lv] = (parts[0], lv, "m2l", 0)
    parts = plan.kernel_times("near", 0)
    if near_fft:
        nn = ("leaf transforms", "stencil", "inverse transforms")
        for k, ms in enumerate(parts):
            out["near %s" % (nn[0] if k == 0 else nn[1 + (k - 1) % 2])
                + ("" if k < 3 else " %d" % ((k - 1) // 2))] = (ms, 0, "near", k)
    elif parts:
        out["near"] = (parts[0], 0, "near", 0)
    return out


def kernel_work(name, N, L, p, route=None):
    """Algorithmic work of one launch of a kernel: (flops, unit, bytes,
    products).  Default route (spectral zones, FFT near zone): flops count 8
    per complex multiply-add; bytes are the kernel's compulsory HBM traffic
    (operands read once, results written once); spectra are complex FP64 at
    the interaction zones ((2p)^2 (p + 1) frequencies per node), complex FP32
    at the near zone ((2s)^2 (s + 1) per leaf).  GEMM zones and the direct
    near zone: 2 p^6 flops per offset and target node, 2 s^6 per neighbour
    leaf and target leaf, on the unit the precision puts them on; `products`
    is the number of bf16 products the split issues per algorithmic product
    (the matrix cores' peak applies to issued flops)."""
    s = N >> L
    route = route or {"m2l": "spectral", "near": "fft", "precision": "bf16x3"}
    if name.startswith("m2l L") and len(name.split()) == 2 and route["m2l"] == "gemm":
        lv = int(name.split()[1][1:])
        fl = (37 if lv == 2 else 189) * 2.0 * p ** 6 * 8 ** lv
        if lv in FP64_LEVELS:
            return fl, ("f64 mfma" if p == 8 else "f64 valu"), None, 1
        if route["precision"] == "bf16x3" and p == 8:
            return fl, "bf16 mfma", None, 6
        return fl, "f32 valu", None, 1
    if name == "near" and route["near"] == "direct":
        fl = 27 * 2.0 * s ** 6 * 8 ** L
        if route["precision"] == "bf16x3" and s in (8, 16):
            return fl, "bf16 mfma", None, 3
        return fl, "f32 valu", None, 1
    r = _default_work(name, N, L, p, s, route.get("fold", False), route.get("zones_fp32_level"))
    return r + (1,)


def _default_work(name, N, L, p, s, fold=False, zones_fp32_level=None):
    if name.startswith("m2l L"):
        lv = int(name.split()[1][1:])
        F = (2 * p) ** 2 * (p + 1)
        nodes = 8 ** lv
        spec = 16.0 * F * nodes
        gl = (8.0 if lv in FP64_LEVELS else 4.0) * p ** 3 * nodes  # gridlet buffer
        if name.endswith("stencil"):
            offs = 37 if lv == 2 else 189
            unit = "f32 valu" if lv == zones_fp32_level else "f64 valu"
            return offs * 8.0 * F * nodes, unit, 2 * spec + 343 * 16.0 * F
        if name.endswith("inverse transforms"):
            return None, "hbm", spec + 2 * gl
        return None, "hbm", spec + gl
    if name.startswith("near"):
        F = (2 * s) ** 2 * (s + 1)
        leaves = 8 ** L
        spec = 8.0 * F * leaves
        # P2M and L2P folded into the transforms: the leaf gridlets written
        # by the forward one and read by the inverse one (FP32)
        gl = 4.0 * p ** 3 * leaves if fold else 0.0
        if "stencil" in name:
            return 27 * 8.0 * F * leaves, "f32 valu", 2 * spec + 27 * 8.0 * F
        return None, "hbm", spec + 4.0 * N ** 3 + gl
    if name in ("p2m",):
        return None, "hbm", 4.0 * N ** 3 + 4.0 * p ** 3 * 8 ** L
    if name in ("l2p",):
        return None, "hbm", 8.0 * N ** 3 + 4.0 * p ** 3 * 8 ** L
    return None, "hbm", None


def gemm_m2l_mfma(rho, args):
    """The interaction zones as block-Toeplitz GEMMs on the matrix cores, on
    the same density: split BF16 (three bf16 terms per operand, six products)
    at the leaf level, FP64 matrix cores at the FP64 levels 2-3.  Per level:
    HIP-event time of its launches (stages one after another), algorithmic
    flops (2 p^6 per offset and target node), issued flops (times the
    products; equal to the MOPS counters) and the fraction of the peak of the
    matrix-core instruction that level runs on."""
    import torch
    from paper_2011_07099_amd.pfmm import Plan
    phi = torch.empty_like(rho)
    with Plan(N, L, P, GREEN, precision="bf16x3", near="direct", m2l="gemm") as pl:
        for _ in range(2):
            pl.solve(rho, phi)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            pl.solve(rho, phi)
        e1.record()
        torch.cuda.synchronize()
        route_ms = e0.elapsed_time(e1) / 5
        pl.set_profile("serial")
        for _ in range(5):
            pl.solve(rho, phi)
        lv_ms = pl.level_times("m2l")
        torch.cuda.synchronize()
    levels, issued, budget = {}, 0.0, 0.0
    for lv, ms in sorted(lv_ms.items()):
        fl = (37 if lv == 2 else 189) * 2.0 * P ** 6 * 8 ** lv
        unit, products = ("f64 mfma", 1) if lv in FP64_LEVELS else ("bf16 mfma", 6)
        peak = PEAK_UNIT[unit]
        tf = fl / (ms * 1e-3) / 1e12
        levels[str(lv)] = {"ms": ms, "unit": unit, "products": products, "flops": fl,
                           "algorithmic_tflops": tf, "issued_tflops": tf * products, "peak": peak,
                           "algorithmic_frac": tf / peak, "issued_frac": tf * products / peak}
        issued += fl * products
        budget += ms * 1e-3 * peak * 1e12
    return {"route": "block-Toeplitz GEMM zones (split bf16 at level 4, FP64 matrix cores at "
                     "levels 2-3), timed on the same density in this run",
            "util": issued / budget, "util_note": "issued matrix-core flops of all levels over "
            "the time-weighted peak of the instruction each level uses",
            "levels": levels, "m2l_ms": sum(lv_ms.values()),
            "solve_ms_with_direct_near_zone": route_ms,
            "phi": phi}


def headline(args):
    import torch
    from paper_2011_07099_amd import fields
    from paper_2011_07099_amd.pfmm import Plan

    rho64 = fields.lognormal(N, ALPHA, SIGMA, seed=SEED)
    rho32 = rho64.astype(np.float32)
    dev = torch.device("cuda:0")
    rho = torch.from_numpy(rho32).to(dev)
    phi = torch.empty_like(rho)
    stream = torch.cuda.current_stream(dev)
    zones32 = args.zones == "fp32" and args.m2l == "spectral" and L == 4
    plan = Plan(N, L, P, GREEN, precision=args.precision, stream=stream,
                accel="expansion" if args.accel == "expansion" else "fd4", near=args.near,
                m2l=args.m2l, zones_fp32=zones32)
    acc = (torch.empty((3, N, N, N), dtype=torch.float32, device=dev)
           if args.accel != "none" else None)
    for _ in range(args.warmup):
        plan.solve(rho, phi, acc)
    torch.cuda.synchronize()
    # Three timed runs of K steps each.  The first, with no timing inside the
    # solve, gives the throughput (HIP events between the kernels would cost
    # 5% of it: every recorded event is one more packet between two kernels
    # on each stream).  The second, as any solve runs (the near zone beside
    # the tree) with HIP events around every kernel group on the stream it
    # runs on, gives each kernel's live duration; the third runs every stage
    # alone on the device, one after another, which gives each kernel's own
    # duration for its roofline.
    spectral, near_fft = args.m2l == "spectral", args.near == "fft"
    runs = {}
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record(stream)
    for _ in range(args.steps):
        plan.solve(rho, phi, acc)
    t_end.record(stream)
    torch.cuda.synchronize()
    plain_ms = t_start.elapsed_time(t_end) / args.steps
    for mode in ("live", "serial"):
        plan.set_profile(mode)
        t_start = torch.cuda.Event(enable_timing=True)
        t_end = torch.cuda.Event(enable_timing=True)
        t_start.record(stream)
        for _ in range(args.steps):
            plan.solve(rho, phi, acc)
        t_end.record(stream)
        torch.cuda.synchronize()
        runs[mode] = {"ms": t_start.elapsed_time(t_end) / args.steps,
                      "kern": kernel_table(plan, L, near_fft, spectral),
                      "stages": plan.stage_times(), "m2l_levels": plan.level_times("m2l")}
    plan.close()
    ms = plain_ms
    kern = runs["serial"]["kern"]
    stages = runs["serial"]["stages"]
    m2l_levels = runs["serial"]["m2l_levels"]

    # P2M and L2P run inside the near zone's leaf transforms when they have
    # no stage of their own
    route = {"m2l": args.m2l, "near": args.near, "precision": args.precision,
             "fold": near_fft and stages["p2m"][1] == 0, "zones_fp32_level": L if zones32 else None}

    def roof(name, dms):
        # the kernel's roofline is the larger of its two floors, flops at the
        # unit's peak and compulsory bytes at the HBM peak; the other is
        # reported beside it
        fl, unit, kbytes, products = kernel_work(name, N, L, P, route)
        mem = None
        if kbytes:
            gbs = kbytes / (dms * 1e-3) / 1e9
            mem = {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                   "frac": gbs / 8000.0}
        if fl is not None:
            peak = PEAK_UNIT[unit]
            tf = fl * products / (dms * 1e-3) / 1e12
            r = {"bound": "mfma" if "mfma" in unit else "alu", "achieved": tf, "peak": peak,
                 "unit": "TFLOP/s", "frac": tf / peak, "unit_used": unit,
                 "flops_per_launch": fl * products}
            if products > 1:
                r.update({"products": products, "algorithmic_flops_per_launch": fl,
                          "algorithmic_tflops": tf / products})
            if mem is not None and mem["frac"] > r["frac"]:
                mem["compute"] = r  # the HBM floor is the higher one
                return mem, kbytes
            if mem is not None:
                r["memory"] = mem
            return r, kbytes
        return (mem or {"bound": "hbm", "achieved": 0.0, "peak": 8000.0, "unit": "GB/s",
                        "frac": 0.0}), kbytes

    # the dominant single kernel (longest on its own) and its roofline
    dom = max(kern, key=lambda k: kern[k][0])
    dms = kern[dom][0]
    roofline, kbytes = roof(dom, dms)
    roofline.update({
        "kernel": "%s (%.4f ms: average over the last %d solves of the serial timed run, HIP "
                  "events on its stream)" % (dom, dms, min(args.steps, 16)),
        "traffic": traffic_bytes(dom, {"precision": args.precision, "near": args.near,
                                            "m2l": args.m2l, "accel": args.accel,
                                            "zones": args.zones, "N": N, "L": L, "p": P}),
        "kernel_compulsory_bytes": kbytes,
        "solve_compulsory_bytes": 4.0 * N ** 3 * 2 + sum(
            (8.0 if lv in FP64_LEVELS else 4.0) * 2 * P ** 3 * 8 ** lv for lv in range(2, L + 1)),
    })
    live = runs["live"]["kern"]
    if dom in live:
        rl, _ = roof(dom, live[dom][0])
        roofline["live"] = {"ms": live[dom][0], "achieved": rl["achieved"], "frac": rl["frac"],
                            "note": "the same kernel in the live timed run, sharing the device "
                                    "with the other stream's kernels"}
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
        "dtype": "f32+f64" if (near_fft and spectral) else args.precision,
        "data": "synthetic",
        "config": {"workload": "periodic FMM, 256^3 lognormal density (P(k)~k^-1.5, "
                               "sigma_delta=2, seed 5), L=4 (16^3-cell leaves), p=8, G_S1",
                   "N": N, "L": L, "p": P, "green": GREEN,
                   "arithmetic": (("FP32 near zone (FFT on the doubled grid) and mesh transfers, "
                                   + ("leaf-level zone stencil in FP32 columns with FP64 totals, "
                                      "FP64 zone transforms, level 2-3 zones and levels 2-3"
                                      if zones32 else
                                      "FP64 interaction zones (spectral stencils) and levels 2-3"))
                                  if (near_fft and spectral) else args.precision),
                   **({"accel": args.accel} if args.accel != "none" else {}),
                   "near": args.near, "m2l": args.m2l,
                   **({"zones": args.zones} if spectral else {})},
        "roofline": roofline,
        "live_profiled_ms_per_step": runs["live"]["ms"],
        "serial_ms_per_step": runs["serial"]["ms"],
        "kernels_ms": {k: v[0] for k, v in sorted(kern.items(), key=lambda kv: -kv[1][0])},
        "kernels_live_ms": {k: v[0] for k, v in sorted(live.items(), key=lambda kv: -kv[1][0])},
        "stages_ms": {k: v[0] for k, v in stages.items()},
        "m2l_levels_ms": {str(k): v for k, v in m2l_levels.items()},
    }
    mf = gemm_m2l_mfma(rho, args) if not args.no_mfma else None
    if mf is not None:
        gemm_phi = mf.pop("phi")
        out["m2l_mfma"] = mf
    if not args.no_cpu_baseline:
        base, accd, context = cpu_baseline(rho32.astype(np.float64),
                                           phi.cpu().numpy().astype(np.float64))
        out["cpu_baseline"] = base
        out["accuracy"] = accd
        if mf is not None:
            from oracle import conv
            pm = context.pop("_pm")
            a = gemm_phi.cpu().numpy().astype(np.float64)
            a, b = a - a.mean(), pm - pm.mean()
            out["m2l_mfma"]["l2_rel_vs_pm"] = float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2)))
            assert conv is not None
        context.pop("_pm", None)
        out["cpu_context"] = context
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
