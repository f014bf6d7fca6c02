#!/usr/bin/env python3
"""All-mode sparse MTTKRP sweep benchmark on one MI355X.

Workload (default): 3-mode COO tensor 50000 x 40000 x 30000, 20M distinct
nonzeros with Zipf(1.2) coordinates over shuffled indices, lognormal(0,1)
values, rank 32, N(0,1) FP32 factors; one step = MTTKRP along all three
modes, each followed by the dynamic remap into the next mode's layout (the
tensor ends where it started).

Reports one JSON line: whole-sweep algorithmic bytes / sweep time (GB/s),
sweep ms, the per-mode kernel's roofline fraction against 8 TB/s HBM, the
BF16-stored-factor sweep (speedup and errors against the FP64 oracle on
sampled rows), and the FP64 oracle timed on one host core.

  python bench.py [--steps K] [--warmup W] [--config 2] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0

METRIC = "all-mode spMTTKRP sweep ms & HBM GB/s; BF16 vs FP32 speedup at stated error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def b_alg_mode(dims, nnz, R, n, sf):
    """Algorithmic bytes of one mode in the paper's traffic model: record read
    + remap write + gathered input-factor rows + output write."""
    N = len(dims)
    E = 4 * N + 4
    return nnz * E * 2 + nnz * (N - 1) * R * sf + dims[n] * R * 4


def b_alg_mttkrp_kernel(dims, nnz, R, n, sf):
    """Algorithmic bytes of one launch of the per-mode MTTKRP kernel (remap
    done by its own kernel): record read + gathers + output write."""
    N = len(dims)
    return nnz * (4 * N + 4) + nnz * (N - 1) * R * sf + dims[n] * R * 4


def b_alg_remap_kernel(dims, nnz):
    """Record read + remap-target read + record write."""
    E = 4 * len(dims) + 4
    return nnz * (2 * E + 4)


def b_min_mttkrp_kernel(dims, nnz, R, n, sf):
    """Compulsory bytes: every record once, every input factor once, output."""
    N = len(dims)
    return nnz * (4 * N + 4) + sum(dims[w] * R * sf for w in range(N) if w != n) \
        + dims[n] * R * 4


def source_sha():
    import hashlib
    h = hashlib.sha256()
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "paper_2309_09131_amd", "csrc")
    for f in ("common.hpp", "mttkrp_kernels.hpp", "inst.hpp", "launch.hpp"):
        with open(os.path.join(here, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(path, key):
    """Calibrated HBM bytes per launch from a committed rocprofv3 summary, or
    None if missing or taken on other kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha") != source_sha():
        return None
    try:
        return int(float(vals[key]))
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--g", type=int, default=0)
    ap.add_argument("--natural-order", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the fused-remap ablation sweep")
    ap.add_argument("--copy-calib-mb", type=int, default=256,
                    help="size of a plain device copy run for counter calibration")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU "
              "path (the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_09131_amd import _abi
    from paper_2309_09131_amd import synthetic as syn
    from paper_2309_09131_amd.api import Plan

    dev = torch.device("cuda:0")
    w = syn.WORKLOADS[args.config]
    t0 = time.time()
    T = syn.generate(args.config)
    log(f"generated {w.name}: nnz={T.nnz} in {time.time() - t0:.1f}s")
    dims, R, N, nnz = T.dims, T.rank, T.nmodes, T.nnz
    idx = torch.from_numpy(T.idx).to(dev)
    vals = torch.from_numpy(T.vals).to(dev)
    f32 = [torch.from_numpy(f).to(dev) for f in T.factors]
    bf = [f.to(torch.bfloat16) for f in f32]
    flags = _abi.NATURAL_ORDER if args.natural_order else 0
    torch.cuda.synchronize()
    tp = time.time()
    plan = Plan(idx, vals, dims, R, g=args.g, flags=flags)
    torch.cuda.synchronize()
    plan_ms = (time.time() - tp) * 1e3
    del idx, vals
    log(f"plan {plan_ms:.1f} ms; shards per mode "
        f"{[plan.info(_abi.INFO_NSHARDS, n) for n in range(N)]}")
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in dims]

    # a plain copy of known size (counter calibration for FETCH/WRITE_SIZE)
    if args.copy_calib_mb > 0:
        a = torch.empty(args.copy_calib_mb << 18, dtype=torch.float32, device=dev)
        a.fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def timed(factors, steps, warm):
        for _ in range(warm):
            plan.mttkrp_all_modes(factors, outs)
        torch.cuda.synchronize()
        plan.profile(True)
        plan.profile_read(_abi.PROF_MTTKRP)      # reset
        plan.profile_read(_abi.PROF_REMAP)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.mttkrp_all_modes(factors, outs)
        e1.record()
        torch.cuda.synchronize()
        sweep_ms = e0.elapsed_time(e1) / steps
        per_mode = [plan.profile_read(_abi.PROF_MTTKRP, n) for n in range(N)]
        per_remap = [plan.profile_read(_abi.PROF_REMAP, n) for n in range(N)]
        plan.profile(False)
        return sweep_ms, per_mode, per_remap

    sweep_ms, per_mode, per_remap = timed(f32, args.steps, args.warmup)
    log(f"fp32 sweep {sweep_ms:.3f} ms; per-mode MTTKRP kernel ms "
        f"{[round(m / max(c, 1), 4) for m, c in per_mode]}; remap kernel ms "
        f"{[round(m / max(c, 1), 4) for m, c in per_remap]}")
    sweep_bytes = sum(b_alg_mode(dims, nnz, R, n, 4) for n in range(N))
    value = sweep_bytes / (sweep_ms * 1e-3) / 1e9

    def kstats(times, bytes_of):
        ms = sum(m for m, _ in times)
        launches = sum(c for _, c in times)
        nbytes = sum(bytes_of(n) * times[n][1] for n in range(N))
        return ms / max(launches, 1), nbytes / max(launches, 1), \
            nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0

    mk_ms, mk_bytes, mk_gbs = kstats(per_mode, lambda n: b_alg_mttkrp_kernel(dims, nnz, R, n, 4))
    rm_ms, rm_bytes, rm_gbs = kstats(per_remap, lambda n: b_alg_remap_kernel(dims, nnz))
    mk_min = sum(b_min_mttkrp_kernel(dims, nnz, R, n, 4) for n in range(N)) / N
    prof_dir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
    ctr = os.path.join(prof_dir, f"mttkrp_kernel_{w.name}_counters.txt")
    fetch = counter_traffic(ctr, "fetch_bytes_per_launch")
    write = counter_traffic(ctr, "write_bytes_per_launch")
    traffic = (fetch + write) if (fetch is not None and write is not None) else None

    # errors on sampled rows against the FP64 oracle (FP32, then BF16)
    import oracle  # test infrastructure: error report and CPU baseline only
    rng = np.random.default_rng(0)
    samples = []
    for n in range(N):
        counts = np.bincount(T.idx[n], minlength=dims[n])
        heavy = np.argsort(counts)[-4:]
        rnd = rng.choice(dims[n], 28, replace=False)
        samples.append(np.unique(np.concatenate([heavy, rnd])))

    def errors(outs_t):
        rep = []
        for n in range(N):
            ref, rabs = oracle.mttkrp_rows(dims, T.idx, T.vals, T.factors, n, samples[n])
            got = outs_t[n][torch.from_numpy(samples[n]).to(dev)].cpu().numpy().astype(np.float64)
            nw = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            el = float(np.max(np.abs(got - ref) / np.where(rabs > 0, rabs, 1)))
            rep.append({"normwise": nw, "elementwise_vs_abs": el,
                        "max_abs": float(np.abs(got - ref).max())})
        return rep

    plan.mttkrp_all_modes(f32, outs)
    torch.cuda.synchronize()
    err32 = errors(outs)
    result_bf16 = None
    if not args.no_bf16:
        bms, bmode, bremap = timed(bf, args.steps, args.warmup)
        plan.mttkrp_all_modes(bf, outs)
        torch.cuda.synchronize()
        errb = errors(outs)
        bbytes = sum(b_alg_mode(dims, nnz, R, n, 2) for n in range(N))
        result_bf16 = {"sweep_ms": round(bms, 4), "speedup_vs_fp32": round(sweep_ms / bms, 3),
                       "alg_GBs": round(bbytes / (bms * 1e-3) / 1e9, 1),
                       "error_vs_fp64_oracle": errb, "tolerance": 2e-2}
        log(f"bf16 sweep {bms:.3f} ms (x{sweep_ms / bms:.2f})")

    def fused_sweep():
        fplan = Plan(torch.from_numpy(T.idx).to(dev), torch.from_numpy(T.vals).to(dev), dims,
                     R, g=args.g, flags=flags | _abi.FUSED_REMAP)
        for _ in range(args.warmup):
            fplan.mttkrp_all_modes(f32, outs)
        torch.cuda.synchronize()
        fe0 = torch.cuda.Event(enable_timing=True)
        fe1 = torch.cuda.Event(enable_timing=True)
        fe0.record()
        for _ in range(args.steps):
            fplan.mttkrp_all_modes(f32, outs)
        fe1.record()
        torch.cuda.synchronize()
        fused_ms = fe0.elapsed_time(fe1) / args.steps
        del fplan
        return fused_ms

    # ablation: remap inside the MTTKRP kernel (the paper's same-agent form)
    fused_ms = None
    if not args.no_ablation:
        fused_ms = fused_sweep()
    log(f"fused-remap fp32 sweep {fused_ms} ms")

    cpu = None
    if not args.no_cpu_baseline:
        tc = time.time()
        for n in range(N):
            oracle.mttkrp(dims, T.idx, T.vals, T.factors, n)
        cs = time.time() - tc
        cpu = {"value": round(sweep_bytes / cs / 1e9, 4), "unit": "GB/s", "cores": 1,
               "kind": "oracle", "sweep_s": round(cs, 2),
               "sample": f"full workload: FP64 oracle MTTKRP along all {N} modes "
                         f"over all {nnz} nonzeros, single thread"}
        log(f"oracle sweep {cs:.1f} s on one core")

    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sweep_ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(dims), "nnz": nnz, "rank": R,
                   "step": "MTTKRP along every mode, each followed by the dynamic "
                           "remap of the tensor into the next mode's layout",
                   "shard_g": plan.info(_abi.INFO_G), "plan_ms": round(plan_ms, 1)},
        "roofline": {"bound": "hbm", "achieved": round(mk_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(mk_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "mk::mttkrp_kernel (per-mode MTTKRP)",
                     "kernel_ms_per_launch": round(mk_ms, 4),
                     "alg_bytes_per_launch": int(mk_bytes),
                     "compulsory_bytes_per_launch": int(mk_min),
                     "compulsory_frac": round(mk_min / (mk_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "note": "algorithmic bytes count every gathered factor row "
                             "(paper's traffic model); most gathers hit L2/MALL"},
        "remap_kernel": {"ms_per_launch": round(rm_ms, 4),
                         "alg_bytes_per_launch": int(rm_bytes),
                         "achieved_GBs": round(rm_gbs, 1),
                         "frac": round(rm_gbs / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "sweep_ms": round(sweep_ms, 4),
        "per_mode_kernel_ms": [round(m / max(c, 1), 4) for m, c in per_mode],
        "per_mode_remap_ms": [round(m / max(c, 1), 4) for m, c in per_remap],
        "fp32_error_vs_fp64_oracle": err32,
        "bf16": result_bf16,
        "fused_remap_sweep_ms": round(fused_ms, 4) if fused_ms else None,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
