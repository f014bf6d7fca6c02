#!/usr/bin/env python3
"""All-mode sparse MTTKRP benchmark on one MI355X.

Default workload (--config 3): a 4-mode COO tensor 1e6 x 5e5 x 2e4 x 2e3
with 100M distinct nonzeros (Zipf(1.1) coordinates over shuffled indices,
lognormal(0,1) values), rank 32, N(0,1) factors.  One step is MTTKRP along
all four modes, each followed by the dynamic remap of the tensor into the
next mode's layout; the tensor ends where it started.  The same sweep runs
with FP32 factors (the headline) and with BF16-stored factors, and the
outputs of both are compared with the FP64 oracle over every output row of
every mode.

Other workloads (explicit runs):
  --config 1  1000x800x600, 100K nnz, R=16: sweep + one CP-ALS sweep
  --config 2  5e4x4e4x3e4, 20M nnz, Zipf(1.2), R=32: FP32 and BF16 sweeps
  --config 4  2e5^3, 50M nnz planted rank 64: sampled CP loss forward +
              autograd backward, finite differences on a 10K subsample
  --config 5  2e6x1e6x1e5x5e3x500, 200M nnz, R=16: full CP-ALS sweep, FP32
              and BF16

Prints one JSON line.  `value` is the HBM rate on compulsory bytes: every
byte the sweep must move through HBM at least once (each stored record read
and written by every mode's MTTKRP and remap, the remap targets, each factor
read once per mode, each output written once) over the sweep time.  The
paper's traffic model (every gathered factor row counted, most of which the
L2 and Infinity Cache serve) is reported beside it as `model_GBs`.
`roofline` is the per-mode MTTKRP kernel on its compulsory bytes per launch
over its mean launch time (HIP events on the launch stream); `traffic` is
the bytes its L2 fetched and wrote beyond itself (rocprofv3 FETCH_SIZE and
WRITE_SIZE, calibrated on a plain copy), read from the committed counter
summary when that was taken on the current kernel sources.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "all-mode spMTTKRP sweep ms & HBM GB/s; BF16 vs FP32 speedup at stated error"
ROOT = os.path.dirname(os.path.abspath(__file__))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- byte models
def rec_bytes(N):
    """Bytes of one COO element in the paper's traffic model: N int32
    coordinates and the FP32 value.  (The stored records pack the
    coordinates and can be smaller; the kernels' own figures use those.)"""
    return 4 * N + 4


def b_alg_mode(dims, nnz, R, n, sf):
    """Paper traffic model for one mode: record read + remap write +
    gathered input-factor rows + output write."""
    N = len(dims)
    return nnz * rec_bytes(N) * 2 + nnz * (N - 1) * R * sf + dims[n] * R * 4


def b_alg_mttkrp_kernel(dims, nnz, R, n, sf):
    """One launch of the per-mode MTTKRP kernel: records + gathers + output."""
    N = len(dims)
    return nnz * rec_bytes(N) + nnz * (N - 1) * R * sf + dims[n] * R * 4


def b_alg_remap_kernel(dims, nnz, rb=None):
    """Record read + remap-target read + record write, for stored records
    of rb bytes (default: the paper's element size)."""
    rb = rec_bytes(len(dims)) if rb is None else rb
    return nnz * (2 * rb + 4)


def b_min_mttkrp_kernel(dims, nnz, R, n, sf, rb=None):
    """Compulsory bytes of one MTTKRP launch: every stored record once,
    every input factor once, the output once."""
    N = len(dims)
    rb = rec_bytes(N) if rb is None else rb
    return nnz * rb + sum(dims[w] * R * sf for w in range(N) if w != n) + dims[n] * R * 4


def b_min_sweep_mode(dims, nnz, R, n, sf, rb):
    """Compulsory bytes of mode n of a sweep: its MTTKRP launch plus the
    remap (record read, remap target read, record write)."""
    return b_min_mttkrp_kernel(dims, nnz, R, n, sf, rb) + nnz * (2 * rb + 4)


def host_cpu():
    """Host CPU model and logical core count (the oracle itself uses one)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count()}


def source_sha():
    """Hash of the MTTKRP kernel sources and of the host library (which
    picks the kernel forms) with comments and blank lines removed: a
    comment edit does not make the counter summary stale."""
    h = hashlib.sha256()
    here = os.path.join(ROOT, "paper_2309_09131_amd", "csrc")
    for f in ("common.hpp", "mttkrp_kernels.hpp", "inst.hpp", "launch.hpp", "mttkrp_lib.hip"):
        with open(os.path.join(here, f), encoding="utf-8") as fh:
            text = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        for line in text.splitlines():
            code = line.split("//", 1)[0].rstrip()
            if code.strip():
                h.update(code.encode() + b"\n")
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


# ---------------------------------------------------------------- helpers
class Timer:
    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, steps, warm):
        torch = self.torch
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps


def oracle_all_modes(oracle, T, threads):
    """FP64 oracle MTTKRP of every mode over every nonzero, with the |.|-sum
    M^abs used as the elementwise error scale.  One thread per mode (the
    oracle is single-threaded C; ctypes releases the GIL during the call)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.time()
    with ThreadPoolExecutor(max_workers=max(1, min(threads, T.nmodes))) as ex:
        futs = [ex.submit(oracle.mttkrp, T.dims, T.idx, T.vals, T.factors, n, True)
                for n in range(T.nmodes)]
        refs = [f.result() for f in futs]
    return refs, time.time() - t0


def error_report(refs, outs, tol):
    """Per mode, over every output row: normwise error, the largest
    |got - ref| / M^abs, and the largest absolute error against the FP64
    oracle; `ok` says whether both relative figures are within tol (rows
    without nonzeros must be exactly zero)."""
    rep = []
    for (ref, rabs), got in zip(refs, outs):
        got = got.astype(np.float64)
        d = np.abs(got - ref)
        nw = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
        zero = rabs == 0
        el = float(np.max(np.where(zero, 0.0, d / np.where(zero, 1.0, rabs))))
        nonzero_where_zero = int(np.count_nonzero(got[zero]))
        rep.append({"rows": int(ref.shape[0]), "normwise": nw, "elementwise_vs_abs": el,
                    "max_abs": float(d.max()) if d.size else 0.0,
                    "ok": bool(nw <= tol and el <= tol and nonzero_where_zero == 0)})
    return rep


# ---------------------------------------------------------------- MTTKRP sweep
def bench_sweep(args, torch, dev, syn, _abi, Plan, oracle):
    w = syn.WORKLOADS[args.config]
    t0 = time.time()
    T = syn.generate(args.config, cache_dir=args.cache_dir, progress=log)
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
    log(f"plan {plan_ms:.1f} ms; shards per mode "
        f"{[plan.info(_abi.INFO_NSHARDS, n) for n in range(N)]}")
    outs = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in dims]
    timer = Timer(torch)

    # a plain copy of known size (counter calibration for FETCH/WRITE_SIZE)
    copy_gbs = device_copy(torch, dev, args.copy_calib_mb, timer)

    def timed(factors):
        # the sweep time without per-kernel events, then the same steps again
        # with the library's HIP events around every MTTKRP and remap launch
        # (on the launch stream) for the per-kernel means
        ms = timer(lambda: plan.mttkrp_all_modes(factors, outs), args.steps, args.warmup)
        plan.profile(True)
        plan.mttkrp_all_modes(factors, outs)
        torch.cuda.synchronize()
        plan.profile_read(_abi.PROF_MTTKRP)      # drop the warm-up launches
        plan.profile_read(_abi.PROF_REMAP)
        timer(lambda: plan.mttkrp_all_modes(factors, outs), args.steps, 0)
        per_mode = [plan.profile_read(_abi.PROF_MTTKRP, n) for n in range(N)]
        per_remap = [plan.profile_read(_abi.PROF_REMAP, n) for n in range(N)]
        plan.profile(False)
        return ms, per_mode, per_remap

    # the FP64 oracle over every nonzero of every mode, one thread per mode,
    # in the background while the GPU is timed (joined before the errors)
    from concurrent.futures import ThreadPoolExecutor
    opool = ThreadPoolExecutor(max_workers=1)
    ofut = None if args.no_errors else opool.submit(oracle_all_modes, oracle, T,
                                                    args.oracle_threads)

    sweep_ms, per_mode, per_remap = timed(f32)
    log(f"fp32 sweep {sweep_ms:.3f} ms; MTTKRP kernel ms "
        f"{[round(m / max(c, 1), 4) for m, c in per_mode]}; remap kernel ms "
        f"{[round(m / max(c, 1), 4) for m, c in per_remap]}")
    rb = plan.info(_abi.INFO_RECORD_BYTES)       # stored record bytes
    sweep_min = sum(b_min_sweep_mode(dims, nnz, R, n, 4, rb) for n in range(N))
    sweep_model = sum(b_alg_mode(dims, nnz, R, n, 4) for n in range(N))
    value = sweep_min / (sweep_ms * 1e-3) / 1e9
    # per-step distribution, and one sweep after a 512 MiB scratch write
    # (factor rows no longer in L2 or the Infinity Cache)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for a0, a1 in ev:
        a0.record()
        plan.mttkrp_all_modes(f32, outs)
        a1.record()
    torch.cuda.synchronize()
    step_ms = sorted(a0.elapsed_time(a1) for a0, a1 in ev)
    scratch = torch.empty(128 << 20, dtype=torch.float32, device=dev)
    scratch.fill_(0.5)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    plan.mttkrp_all_modes(f32, outs)
    c1.record()
    torch.cuda.synchronize()
    cold_ms = c0.elapsed_time(c1)
    del scratch
    log(f"per-step median {step_ms[len(step_ms) // 2]:.3f} ms, min {step_ms[0]:.3f} ms; "
        f"cold-cache sweep {cold_ms:.3f} ms")

    def kstats(times, bytes_of):
        ms = sum(m for m, _ in times)
        launches = sum(c for _, c in times)
        nbytes = sum(bytes_of(n) * times[n][1] for n in range(N))
        return ms / max(launches, 1), nbytes / max(launches, 1), \
            nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0

    mk_ms, mk_min, mk_gbs = kstats(per_mode, lambda n: b_min_mttkrp_kernel(dims, nnz, R, n, 4, rb))
    _, mk_model, mk_model_gbs = kstats(per_mode,
                                       lambda n: b_alg_mttkrp_kernel(dims, nnz, R, n, 4))
    rm_ms, rm_bytes, rm_gbs = kstats(per_remap, lambda n: b_alg_remap_kernel(dims, nnz, rb))
    ctr = os.path.join(ROOT, "profiles", f"mttkrp_kernel_{w.name}_counters.txt")
    fetch = counter_traffic(ctr, "fetch_bytes_per_launch")
    write = counter_traffic(ctr, "write_bytes_per_launch")
    traffic = (fetch + write) if (fetch is not None and write is not None) else None

    plan.mttkrp_all_modes(f32, outs)
    torch.cuda.synchronize()
    got32 = [o.cpu().numpy() for o in outs]

    result_bf16 = None
    gotb = None
    if not args.no_bf16:
        bms, bmode, bremap = timed(bf)
        plan.mttkrp_all_modes(bf, outs)
        torch.cuda.synchronize()
        gotb = [o.cpu().numpy() for o in outs]
        bmin = sum(b_min_sweep_mode(dims, nnz, R, n, 2, rb) for n in range(N))
        bmodel = sum(b_alg_mode(dims, nnz, R, n, 2) for n in range(N))
        result_bf16 = {"sweep_ms": round(bms, 4), "speedup_vs_fp32": round(sweep_ms / bms, 3),
                       "GBs": round(bmin / (bms * 1e-3) / 1e9, 1),
                       "model_GBs": round(bmodel / (bms * 1e-3) / 1e9, 1),
                       "mttkrp_kernel_ms": [round(m / max(c, 1), 4) for m, c in bmode],
                       "remap_kernel_ms": [round(m / max(c, 1), 4) for m, c in bremap],
                       "tolerance": 2e-2}
        log(f"bf16 sweep {bms:.3f} ms (x{sweep_ms / bms:.2f})")

    # gather ceiling: a kernel that issues the MTTKRP kernel's record loads and
    # factor-row gathers (same lane form, same row reuse) and reduces them
    # trivially; the MTTKRP kernel's time over it says how much of the time
    # the gathers themselves take
    ceiling = None
    if not args.no_ablation:
        gplan = Plan(idx, vals, dims, R, g=args.g, flags=flags | _abi.GATHER_ONLY)
        gouts = [torch.empty((d, R), dtype=torch.float32, device=dev) for d in dims]
        ceiling = {}
        for name, F, kt in (("fp32", f32, per_mode),
                            ("bf16", bf, bmode if result_bf16 else None)):
            if kt is None:
                continue
            for _ in range(args.warmup):
                gplan.mttkrp_all_modes(F, gouts)
            torch.cuda.synchronize()
            gplan.profile(True)
            for _ in range(args.steps):
                gplan.mttkrp_all_modes(F, gouts)
            torch.cuda.synchronize()
            gk = [gplan.profile_read(_abi.PROF_MTTKRP, n) for n in range(N)]
            gplan.profile_read(_abi.PROF_REMAP)
            gplan.profile(False)
            g_ms = sum(m for m, _ in gk) / max(sum(c for _, c in gk), 1)
            k_ms = sum(m for m, _ in kt) / max(sum(c for _, c in kt), 1)
            ceiling[name] = {"gather_ceiling_ms": round(g_ms, 4),
                             "mttkrp_kernel_ms": round(k_ms, 4),
                             "kernel_over_ceiling": round(k_ms / g_ms, 3)}
            log(f"gather ceiling {name}: {g_ms:.4f} ms per launch; MTTKRP kernel "
                f"{k_ms:.4f} ms (x{k_ms / g_ms:.3f})")
        del gplan, gouts

    # the paper's "without remapping" baseline: one tensor copy per mode
    # layout (N x the memory), so each mode's MTTKRP runs with no remap;
    # timed here as the MTTKRP of each mode on its own layout
    ncopy_ms = 0.0
    for n in range(N):
        if plan.cur_mode != n:
            plan.remap(n)
        ncopy_ms += timer(lambda: plan.mttkrp_mode(n, f32, outs[n], fuse_remap=False),
                          args.steps, args.warmup)
    plan.remap(0)
    torch.cuda.synchronize()
    log(f"one layout copy per mode (no remap): {ncopy_ms:.3f} ms per sweep")

    fused_ms = None
    if not args.no_ablation:
        # the paper's same-agent form: remap written from inside the MTTKRP kernel
        fplan = Plan(idx, vals, dims, R, g=args.g, flags=flags | _abi.FUSED_REMAP)
        fused_ms = timer(lambda: fplan.mttkrp_all_modes(f32, outs), args.steps, args.warmup)
        del fplan
        log(f"fused-remap fp32 sweep {fused_ms:.3f} ms")
    unpacked_ms = None
    if not args.no_ablation:
        # one 32-bit word per coordinate in the stored records
        uplan = Plan(idx, vals, dims, R, g=args.g, flags=flags | _abi.UNPACKED_RECORDS)
        unpacked_ms = timer(lambda: uplan.mttkrp_all_modes(f32, outs), args.steps, args.warmup)
        del uplan
        log(f"unpacked-record fp32 sweep {unpacked_ms:.3f} ms")

    resident = None
    if not args.no_ablation:
        # memory for time: keep resident the layout whose incoming remap
        # measured slowest (one more tensor copy), then every layout (the
        # paper's "without remapping" case, N + 2 copies), FP32 sweep
        slow = max(range(N), key=lambda n: per_remap[n][0] / max(per_remap[n][1], 1))
        resident = {}
        for name, modes in (("one", [(slow + 1) % N]), ("all", list(range(N)))):
            mask = sum(_abi.RESIDENT_LAYOUT(n) for n in modes)
            rplan = Plan(idx, vals, dims, R, g=args.g, flags=flags | mask)
            rms = timer(lambda: rplan.mttkrp_all_modes(f32, outs), args.steps, args.warmup)
            resident[name] = {"resident_modes": modes, "sweep_ms": round(rms, 4),
                              "extra_tensor_copies": len(modes),
                              "extra_bytes": len(modes) * nnz * rb}
            log(f"resident layouts {modes}: sweep {rms:.3f} ms")
            del rplan

    locality = None
    if args.locality:
        # plan option: Morton order of the two leading inputs inside each
        # output row (Sec. V-J preprocessing) instead of the lexicographic order
        torch.cuda.synchronize()
        t1 = time.time()
        lplan = Plan(idx, vals, dims, R, g=args.g, flags=flags | _abi.LOCALITY_ORDER)
        torch.cuda.synchronize()
        lp_ms = (time.time() - t1) * 1e3
        locality = {"plan_ms": round(lp_ms, 1)}
        for name, F in (("fp32", f32), ("bf16", bf)):
            lms = timer(lambda: lplan.mttkrp_all_modes(F, outs), args.steps, args.warmup)
            lplan.profile(True)
            timer(lambda: lplan.mttkrp_all_modes(F, outs), args.steps, 0)
            lk = [lplan.profile_read(_abi.PROF_MTTKRP, n) for n in range(N)]
            lr = [lplan.profile_read(_abi.PROF_REMAP, n) for n in range(N)]
            lplan.profile(False)
            locality[name] = {"sweep_ms": round(lms, 4),
                              "mttkrp_kernel_ms": [round(m / max(c, 1), 4) for m, c in lk],
                              "remap_kernel_ms": [round(m / max(c, 1), 4) for m, c in lr]}
            log(f"locality order {name}: sweep {lms:.3f} ms; MTTKRP kernel ms "
                f"{locality[name]['mttkrp_kernel_ms']}; remap {locality[name]['remap_kernel_ms']}")
        del lplan

    als = None
    if args.config in (1, 5):
        als = {}
        for name, F in (("fp32", f32), ("bf16", bf)):
            fac = [f.clone() for f in F]
            lam = torch.empty(R, dtype=torch.float64, device=dev)
            mbuf = torch.empty((max(dims), R), dtype=torch.float32, device=dev)
            steps = max(1, min(args.steps, 5))
            ms = timer(lambda: plan.cp_als_sweep(fac, mbuf, lam), steps, 1)
            fac = [f.clone() for f in F]
            lam, fit = plan.cp_als_sweep(fac, mbuf, lam)
            als[name] = {"sweep_ms": round(ms, 3), "fit_after_one_sweep": float(fit.item())}
            log(f"CP-ALS sweep {name}: {ms:.3f} ms, fit {fit.item():.6f}")
        if nnz <= 2_000_000:
            _, olam, ofit, _, _ = oracle.cp_als_sweep(dims, T.idx, T.vals, T.factors)
            als["oracle_fit"] = ofit
        als["bf16_speedup_vs_fp32"] = round(als["fp32"]["sweep_ms"] / als["bf16"]["sweep_ms"], 3)

    ablations = {}
    if args.rank_sweep:
        # time against rank (Sec. V: time grows with R): same tensor, N(0,1)
        # factors of each rank, FP32
        gen = torch.Generator(device=dev)
        gen.manual_seed(7)
        rows = []
        for Rk in [int(x) for x in args.rank_sweep.split(",")]:
            Fk = [torch.randn((d, Rk), generator=gen, device=dev) for d in dims]
            pk = Plan(idx, vals, dims, Rk, g=args.g)
            ok = [torch.empty((d, Rk), dtype=torch.float32, device=dev) for d in dims]
            mk = timer(lambda: pk.mttkrp_all_modes(Fk, ok), args.steps, args.warmup)
            Fb = [f.to(torch.bfloat16) for f in Fk]
            mb = timer(lambda: pk.mttkrp_all_modes(Fb, ok), args.steps, args.warmup)
            bk = sum(b_alg_mode(dims, nnz, Rk, n, 4) for n in range(N))
            rows.append({"rank": Rk, "sweep_ms": round(mk, 4),
                         "alg_GBs": round(bk / (mk * 1e-3) / 1e9, 1),
                         "ms_per_rank_unit": round(mk / Rk, 5),
                         "bf16_sweep_ms": round(mb, 4),
                         "bf16_speedup": round(mk / mb, 3)})
            log(f"rank {Rk}: sweep {mk:.3f} ms, bf16 {mb:.3f} ms (x{mk / mb:.2f})")
            del pk, ok, Fk, Fb
        ablations["rank_sweep"] = rows
    if args.g_sweep:
        # shard size g (Sec. III-C, V-A): plan time and sweep time
        rows = []
        for gk in [int(x) for x in args.g_sweep.split(",")]:
            torch.cuda.synchronize()
            t1 = time.time()
            pk = Plan(idx, vals, dims, R, g=gk)
            torch.cuda.synchronize()
            pms = (time.time() - t1) * 1e3
            mk = timer(lambda: pk.mttkrp_all_modes(f32, outs), args.steps, args.warmup)
            rows.append({"g": gk, "plan_ms": round(pms, 1), "sweep_ms": round(mk, 4),
                         "shards": [pk.info(_abi.INFO_NSHARDS, n) for n in range(N)]})
            log(f"g {gk}: plan {pms:.1f} ms, sweep {mk:.3f} ms")
            del pk
        ablations["g_sweep"] = rows
    if args.m_sweep:
        # super-shard size m_n (Sec. III-A, V-A), the same for every mode
        # (capped at I_n); 0 = the default rule
        rows = []
        for mk_ in [int(x) for x in args.m_sweep.split(",")]:
            pk = Plan(idx, vals, dims, R, g=args.g, m=[mk_] * N if mk_ > 0 else None)
            mk = timer(lambda: pk.mttkrp_all_modes(f32, outs), args.steps, args.warmup)
            rows.append({"m": mk_ if mk_ > 0 else "default",
                         "m_used": [pk.info(_abi.INFO_M, n) for n in range(N)],
                         "super_shards": [pk.info(_abi.INFO_NSUPER, n) for n in range(N)],
                         "shards": [pk.info(_abi.INFO_NSHARDS, n) for n in range(N)],
                         "sweep_ms": round(mk, 4)})
            log(f"m {mk_}: sweep {mk:.3f} ms")
            del pk
        ablations["m_sweep"] = rows

    del idx, vals
    err32, oracle_s = None, None
    if ofut is not None:
        refs, oracle_s = ofut.result()
        err32 = error_report(refs, got32, 1e-5)
        log(f"fp32 errors over every row: {err32}")
        if gotb is not None:
            result_bf16["error_vs_fp64_oracle"] = error_report(refs, gotb, 2e-2)
            log(f"bf16 errors over every row: {result_bf16['error_vs_fp64_oracle']}")
        del refs
    opool.shutdown()
    del got32, gotb

    cpu = None
    if not args.no_cpu_baseline:
        # the FP64 oracle on one core, on a bounded sample of the same tensor
        S = min(nnz, args.cpu_sample)
        tc = time.time()
        for n in range(N):
            oracle.mttkrp(dims, T.idx[:, :S], T.vals[:S], T.factors, n)
        cs = time.time() - tc
        sb = sum(b_min_sweep_mode(dims, S, R, n, 4, rb) for n in range(N))
        what = "all" if S == nnz else f"the first {S} (in generation order) of {nnz}"
        cpu = {"value": round(sb / cs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sweep_s": round(cs, 2), "host": host_cpu(),
               "sample": f"FP64 oracle MTTKRP along all {N} modes over {what} nonzeros, "
                         f"single thread; value = the compulsory sweep bytes of that "
                         f"sample (as for the GPU value) / time"}
        log(f"oracle sweep {cs:.1f} s on one core ({S} nonzeros)")

    tr_gbs = traffic / (mk_ms * 1e-3) / 1e9 if traffic else None
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
        "value_is": "compulsory HBM bytes of the sweep (stored records read and written "
                    "by every mode's MTTKRP and remap, remap targets, each factor once "
                    "per mode, outputs) / sweep time",
        "model_GBs": round(sweep_model / (sweep_ms * 1e-3) / 1e9, 1),
        "model_GBs_is": "the paper's traffic model (every gathered factor row, 4N+4-byte "
                        "records) / sweep time; most gathers are served by L2 and the "
                        "Infinity Cache, so this exceeds the HBM peak",
        "roofline": {"bound": "hbm", "achieved": round(mk_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(mk_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": "mk::mttkrp_kernel (per-mode MTTKRP)",
                     "kernel_ms_per_launch": round(mk_ms, 4),
                     "compulsory_bytes_per_launch": int(mk_min),
                     "achieved_is": "compulsory bytes per launch (stored records once, "
                                    "each input factor once, the output once) / mean "
                                    "launch time from HIP events on the launch stream",
                     "model_bytes_per_launch": int(mk_model),
                     "model_GBs": round(mk_model_gbs, 1),
                     "traffic_is": "bytes the L2 fetched from and wrote to the fabric per "
                                   "launch (FETCH_SIZE x2 + WRITE_SIZE, calibrated on a plain "
                                   "copy); Infinity-Cache hits included, so an upper bound "
                                   "on DRAM bytes",
                     "beyond_l2_GBs": round(tr_gbs, 1) if tr_gbs else None,
                     "stored_record_bytes": rb},
        "gather_ceiling": ceiling,
        "remap_kernel": {"ms_per_launch": round(rm_ms, 4), "record_bytes": rb,
                         "bytes_per_launch": int(rm_bytes),
                         "achieved_GBs": round(rm_gbs, 1),
                         "frac": round(rm_gbs / HBM_PEAK_GBS, 4)},
        "cpu_baseline": cpu,
        "oracle_error_run_s": round(oracle_s, 1) if oracle_s else None,
        "sweep_ms": round(sweep_ms, 4),
        "per_mode_kernel_ms": [round(m / max(c, 1), 4) for m, c in per_mode],
        "per_mode_remap_ms": [round(m / max(c, 1), 4) for m, c in per_remap],
        "fp32_error_vs_fp64_oracle": err32,
        "fp32_tolerance": 1e-5,
        "bf16": result_bf16,
        "fused_remap_sweep_ms": round(fused_ms, 4) if fused_ms else None,
        "unpacked_records_sweep_ms": round(unpacked_ms, 4) if unpacked_ms else None,
        "locality_order": locality,
        "resident_layouts": resident,
        "layout_copy_per_mode_sweep_ms": round(ncopy_ms, 4),
        "cp_als": als,
        "sweep_ms_median": round(step_ms[len(step_ms) // 2], 4),
        "sweep_ms_min": round(step_ms[0], 4),
        "cold_cache_sweep_ms": round(cold_ms, 4),
        "device_copy_GBs": round(copy_gbs, 1) if copy_gbs else None,
        "remap_share": {
            "of_sweep_time": round(sum(m for m, _ in per_remap) / max(sum(c for _, c in per_remap), 1)
                                   * N / sweep_ms, 4),
            "of_compulsory_bytes": round(N * nnz * (2 * rb + 4) / sweep_min, 4),
            "of_model_bytes": round(sum(nnz * rec_bytes(N) for _ in range(N)) / sweep_model, 4)},
        "ablations": ablations or None,
    }
    return rec


# ---------------------------------------------------------------- CP-ALS run
def device_copy(torch, dev, mb, timer):
    """A plain device copy of `mb` MiB: its bandwidth, and the reference the
    FETCH_SIZE / WRITE_SIZE counter runs are calibrated against."""
    if mb <= 0:
        return None
    a = torch.empty(mb << 18, dtype=torch.float32, device=dev)
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    cms = timer(lambda: b.copy_(a), 10, 2)
    gbs = 2 * a.numel() * 4 / (cms * 1e-3) / 1e9      # read + write
    log(f"device copy of {mb} MiB: {gbs:.0f} GB/s")
    del a, b
    return gbs


def als_recovery(torch, dev, Plan, D, R=16, seed=20230916 + 6, max_sweeps=300, tol=1e-4):
    """CP-ALS to convergence on a fully stored D x D x D tensor of planted
    rank R (N(0,1) factors; entries in FP32), from an independent N(0,1)
    start.  Pinned by the planted truth: fit -> 1 and every planted column
    matched (|cos| of normalised columns)."""
    rng = np.random.default_rng(seed)
    dims = (D, D, D)
    true = [rng.standard_normal((D, R)) for _ in range(3)]
    # X[i, j, k] = sum_r A0[i, r] A1[j, r] A2[k, r], built as A0 (A2 (.) A1)^T
    kr = (true[2][:, None, :] * true[1][None, :, :]).reshape(D * D, R)   # row k*D + j
    vals = (true[0] @ kr.T).reshape(-1).astype(np.float32)                # q = i*D*D + k*D + j
    del kr
    q = np.arange(D * D * D, dtype=np.int64)
    idx = np.stack([q // (D * D), q % D, (q // D) % D]).astype(np.int32)
    del q
    nnz = idx.shape[1]
    t0 = time.time()
    plan = Plan(torch.from_numpy(idx).to(dev), torch.from_numpy(vals).to(dev), dims, R)
    torch.cuda.synchronize()
    plan_ms = (time.time() - t0) * 1e3
    del idx, vals
    init = [rng.standard_normal((D, R)).astype(np.float32) for _ in range(3)]
    facs = [torch.from_numpy(f).to(dev) for f in init]
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    lam, fits = plan.cp_als(facs, max_sweeps=max_sweeps, tol=tol)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    fits = fits.cpu().numpy()
    cong = 1.0
    for n in range(3):
        a = facs[n].cpu().numpy().astype(np.float64)
        a /= np.linalg.norm(a, axis=0)
        b = true[n] / np.linalg.norm(true[n], axis=0)
        cong = min(cong, float(np.abs(a.T @ b).max(axis=0).min()))
    out = {"dims": list(dims), "nnz": int(nnz), "rank": R, "plan_ms": round(plan_ms, 1),
           "sweeps": int(len(fits)), "final_fit": float(fits[-1]),
           "fit_after_sweeps_1_2_5_10": [float(fits[k - 1]) for k in (1, 2, 5, 10)
                                         if k <= len(fits)],
           "total_ms": round(ms, 1), "ms_per_sweep": round(ms / len(fits), 3),
           "min_column_congruence": round(cong, 6), "tol": tol}
    log(f"CP-ALS recovery {out}")
    return out


# ---------------------------------------------------------------- CP loss
def bench_loss(args, torch, dev, syn, _abi, Plan, oracle):
    from paper_2309_09131_amd.api import cp_loss
    w = syn.WORKLOADS[4]
    t0 = time.time()
    T = syn.generate(4, cache_dir=args.cache_dir, progress=log)
    log(f"generated {w.name}: nnz={T.nnz} in {time.time() - t0:.1f}s")
    dims, R, N, nnz = T.dims, T.rank, T.nmodes, T.nnz
    idx = torch.from_numpy(T.idx).to(dev)
    vals = torch.from_numpy(T.vals).to(dev)
    tp = time.time()
    plan = Plan(idx, vals, dims, R, g=args.g)
    torch.cuda.synchronize()
    plan_ms = (time.time() - tp) * 1e3
    timer = Timer(torch)
    copy_gbs = device_copy(torch, dev, args.copy_calib_mb, timer)
    fac = [torch.from_numpy(f).to(dev).requires_grad_(True) for f in T.factors]

    def step():
        for f in fac:
            f.grad = None
        loss = cp_loss(plan, fac)
        loss.backward()
        return loss

    ms = timer(step, args.steps, args.warmup)
    fwd_ms = timer(lambda: plan.cp_loss_grad(fac, loss=True, grads=False), args.steps, 1)
    E = rec_bytes(N)
    rb = plan.info(_abi.INFO_RECORD_BYTES)       # stored record bytes
    fac_b = sum(d * R * 4 for d in dims)
    # paper traffic model: every gathered factor row, 4N+4-byte records
    fwd_b = nnz * (E + N * R * 4)
    bwd_b = sum(nnz * (2 * E + N * R * 4) + dims[k] * R * 4 for k in range(N))
    # compulsory HBM bytes: each of the N gradient passes (the first also
    # yields the loss) reads the records and every factor once and writes
    # its gradient, and its remap reads the records and targets and writes
    # the records
    bwd_min = sum(nnz * rb + fac_b + dims[k] * R * 4 + nnz * (2 * rb + 4) for k in range(N))
    value = bwd_min / (ms * 1e-3) / 1e9
    model_gbs = bwd_b / (ms * 1e-3) / 1e9        # the step is the N gradient passes
    log(f"loss fwd+bwd {ms:.3f} ms (fwd {fwd_ms:.3f} ms)")
    # per-kernel means from the library's HIP events (same steps again)
    plan.profile(True)
    step()
    torch.cuda.synchronize()
    for k in (_abi.PROF_RESID, _abi.PROF_LOSS, _abi.PROF_REMAP):
        plan.profile_read(k)
    timer(step, args.steps, 0)
    resid = [plan.profile_read(_abi.PROF_RESID, n) for n in range(N)]
    remk = plan.profile_read(_abi.PROF_REMAP)
    plan.profile_read(_abi.PROF_LOSS)
    # the step takes the loss from its first residual pass; the loss kernel
    # alone runs when no gradient is asked for
    timer(lambda: plan.cp_loss_grad(fac, loss=True, grads=False), args.steps, 0)
    lossk = plan.profile_read(_abi.PROF_LOSS)
    plan.profile(False)
    r_ms = sum(m for m, _ in resid)
    r_launch = sum(c for _, c in resid)
    r_bytes = sum((nnz * (E + N * R * 4) + dims[n] * R * 4) * resid[n][1] for n in range(N))
    r_gbs = r_bytes / (r_ms * 1e-3) / 1e9
    # compulsory bytes of one residual launch: stored records once, every
    # factor once, the gradient rows once
    r_min = sum((nnz * rb + fac_b + dims[n] * R * 4) * resid[n][1] for n in range(N))
    r_min_gbs = r_min / (r_ms * 1e-3) / 1e9
    ctr = os.path.join(ROOT, "profiles", f"resid_kernel_{w.name}_counters.txt")
    fetch = counter_traffic(ctr, "fetch_bytes_per_launch")
    write = counter_traffic(ctr, "write_bytes_per_launch")
    traffic = (fetch + write) if (fetch is not None and write is not None) else None
    r_kms = r_ms / r_launch
    l_gbs = nnz * (E + N * R * 4) * lossk[1] / (lossk[0] * 1e-3) / 1e9
    l_min_gbs = (nnz * rb + fac_b) * lossk[1] / (lossk[0] * 1e-3) / 1e9
    log(f"residual MTTKRP kernel {r_ms / r_launch:.4f} ms/launch ({r_gbs:.0f} GB/s), "
        f"loss kernel {lossk[0] / lossk[1]:.4f} ms ({l_gbs:.0f} GB/s), remap "
        f"{remk[0] / max(remk[1], 1):.4f} ms")

    # the same step with BF16-stored factors (FP32 arithmetic); errors on the
    # subsample below
    bfac = [f.detach().to(torch.bfloat16).requires_grad_(True) for f in fac]

    def bstep():
        for f in bfac:
            f.grad = None
        loss = cp_loss(plan, bfac)
        loss.backward()
        return loss

    bf_ms = timer(bstep, args.steps, args.warmup)
    plan.profile(True)
    timer(bstep, args.steps, 0)
    bres = [plan.profile_read(_abi.PROF_RESID, n) for n in range(N)]
    plan.profile_read(_abi.PROF_REMAP)
    plan.profile(False)
    del bfac
    log(f"bf16 loss fwd+bwd {bf_ms:.3f} ms (x{ms / bf_ms:.2f}); residual kernel ms "
        f"{[round(m / max(c, 1), 4) for m, c in bres]}")

    locality = None
    if args.locality:
        # the same step on a plan with the Morton locality order
        lplan = Plan(idx, vals, dims, R, g=args.g, flags=_abi.LOCALITY_ORDER)
        torch.cuda.synchronize()

        def lstep():
            for f in fac:
                f.grad = None
            loss = cp_loss(lplan, fac)
            loss.backward()
            return loss

        lms = timer(lstep, args.steps, args.warmup)
        lplan.profile(True)
        timer(lstep, args.steps, 0)
        lres = [lplan.profile_read(_abi.PROF_RESID, n) for n in range(N)]
        lplan.profile(False)
        locality = {"step_ms": round(lms, 4),
                    "residual_kernel_ms": [round(m / max(c, 1), 4) for m, c in lres]}
        log(f"locality order: step {lms:.3f} ms; residual kernel ms "
            f"{locality['residual_kernel_ms']}")
        del lplan

    # checks on a 10K-nonzero subsample (first in generation order)
    S = 10_000
    sub_idx = np.ascontiguousarray(T.idx[:, :S])
    sub_val = np.ascontiguousarray(T.vals[:S])
    sp = Plan(torch.from_numpy(sub_idx).to(dev), torch.from_numpy(sub_val).to(dev), dims, R,
              g=256)
    f64 = [f.astype(np.float64) for f in T.factors]
    L_ref, G_ref = oracle.cp_loss_grad(dims, sub_idx, sub_val, f64)
    sf = [torch.from_numpy(f).to(dev) for f in T.factors]
    l_gpu, g_gpu = sp.cp_loss_grad(sf)
    loss_rel = abs(l_gpu.item() - L_ref) / abs(L_ref)
    grad_rel = max(float(np.linalg.norm(g_gpu[k].cpu().numpy() - G_ref[k])
                         / np.linalg.norm(G_ref[k])) for k in range(N))
    rng = np.random.default_rng(1)
    fd_gpu, fd_orc = [], []
    for _ in range(16):
        k = int(rng.integers(0, N))
        i = int(rng.choice(sub_idx[k]))
        r = int(rng.integers(0, R))
        h = 0.25                       # exact: the loss is quadratic per entry
        fp = [f.clone() for f in sf]
        fm = [f.clone() for f in sf]
        fp[k][i, r] += h
        fm[k][i, r] -= h
        lp = sp.cp_loss_grad(fp, grads=False)[0].item()
        lm = sp.cp_loss_grad(fm, grads=False)[0].item()
        g = g_gpu[k][i, r].item()
        fd_gpu.append(abs((lp - lm) / (2 * h) - g) / max(1.0, abs(g)))
        hp = [f.copy() for f in f64]
        hm = [f.copy() for f in f64]
        hp[k][i, r] += 1e-3
        hm[k][i, r] -= 1e-3
        fdo = (oracle.cp_loss_grad(dims, sub_idx, sub_val, hp, want_grad=False)
               - oracle.cp_loss_grad(dims, sub_idx, sub_val, hm, want_grad=False)) / 2e-3
        fd_orc.append(abs(fdo - G_ref[k][i, r]) / max(1.0, abs(G_ref[k][i, r])))
    # BF16-stored factors on the subsample: against the oracle at the
    # BF16-rounded factors (accumulation error) and at the FP32 factors
    # (storage + accumulation)
    sb = [f.to(torch.bfloat16) for f in sf]
    lb, gb = sp.cp_loss_grad(sb)
    rb64 = [f.float().cpu().numpy().astype(np.float64) for f in sb]
    Lb_ref, Gb_ref = oracle.cp_loss_grad(dims, sub_idx, sub_val, rb64)
    bf16_checks = {
        "loss_rel_err_vs_oracle_bf16_factors": abs(lb.item() - Lb_ref) / abs(Lb_ref),
        "grad_normwise_rel_err_vs_oracle_bf16_factors": max(
            float(np.linalg.norm(gb[k].cpu().numpy() - Gb_ref[k]) / np.linalg.norm(Gb_ref[k]))
            for k in range(N)),
        "loss_rel_err_vs_oracle_fp32_factors": abs(lb.item() - L_ref) / abs(L_ref),
        "grad_normwise_rel_err_vs_oracle_fp32_factors": max(
            float(np.linalg.norm(gb[k].cpu().numpy() - G_ref[k]) / np.linalg.norm(G_ref[k]))
            for k in range(N))}
    log(f"bf16 checks {bf16_checks}")
    # loss at the planted truth: expected nnz * sigma^2
    truth = [torch.from_numpy(T.extra[f"true{n}"]).to(dev) for n in range(N)]
    l_true = plan.cp_loss_grad(truth, grads=False)[0].item()
    sigma = float(T.extra["sigma"])
    checks = {"subsample_nnz": S, "loss_rel_err_vs_oracle": loss_rel,
              "grad_normwise_rel_err_vs_oracle": grad_rel,
              "fd_vs_gpu_grad_max_rel": max(fd_gpu), "fd_vs_oracle_grad_max_rel": max(fd_orc),
              "loss_at_truth": l_true, "expected_nnz_sigma2": nnz * sigma ** 2}
    log(f"checks {checks}")
    cpu = None
    if not args.no_cpu_baseline:
        Sc = min(nnz, args.cpu_sample // 8)
        tc = time.time()
        oracle.cp_loss_grad(dims, T.idx[:, :Sc], T.vals[:Sc], f64)
        cs = time.time() - tc
        sb = Sc * (E + N * R * 4) + N * Sc * (2 * E + N * R * 4)
        cpu = {"value": round(sb / cs / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "host": host_cpu(),
               "sample": f"FP64 oracle loss + gradient over the first {Sc} of {nnz} nonzeros, "
                         f"single thread", "seconds": round(cs, 2)}
    return {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "dims": list(dims), "nnz": nnz, "rank": R,
                   "step": "sampled CP loss forward + autograd backward to all factors "
                           "(N residual passes, the first of which also yields the loss)",
                   "plan_ms": round(plan_ms, 1)},
        "value_is": "compulsory HBM bytes of the step (each of the N gradient passes: "
                    "stored records and every factor once, its gradient rows, and its "
                    "remap's record read, target read and record write) / step time",
        "model_GBs": round(model_gbs, 1),
        "model_GBs_is": "the paper's traffic model (every gathered factor row, 4N+4-byte "
                        "records) / step time; most gathers are served by L2 and the "
                        "Infinity Cache, so this can exceed the HBM peak",
        "roofline": {"bound": "hbm", "achieved": round(r_min_gbs, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r_min_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "beyond_l2_GBs": round(traffic / (r_kms * 1e-3) / 1e9, 1) if traffic
                     else None,
                     "kernel": "mk::mttkrp_kernel residual form (loss gradient, per mode)",
                     "kernel_ms_per_launch": round(r_ms / r_launch, 4),
                     "compulsory_bytes_per_launch": int(r_min / r_launch),
                     "achieved_is": "compulsory bytes per launch (stored records once, every "
                                    "factor once, the gradient rows once) / mean launch time "
                                    "from HIP events on the launch stream",
                     "model_bytes_per_launch": int(r_bytes / r_launch),
                     "model_GBs": round(r_gbs, 1),
                     "traffic_is": "bytes the L2 fetched from and wrote to the fabric per "
                                   "launch (FETCH_SIZE x2 + WRITE_SIZE, calibrated on a plain "
                                   "copy); Infinity-Cache hits included",
                     "stored_record_bytes": rb},
        "loss_kernel": {"ms_per_launch": round(lossk[0] / lossk[1], 4),
                        "compulsory_GBs": round(l_min_gbs, 1),
                        "model_bytes_per_launch": int(nnz * (E + N * R * 4)),
                        "model_GBs": round(l_gbs, 1)},
        "cpu_baseline": cpu, "forward_ms": round(fwd_ms, 4),
        "residual_kernel_ms_per_mode": [round(m / max(c, 1), 4) for m, c in resid],
        "bf16": {"ms_per_step": round(bf_ms, 4), "speedup_vs_fp32": round(ms / bf_ms, 3),
                 "residual_kernel_ms_per_mode": [round(m / max(c, 1), 4) for m, c in bres],
                 "checks": bf16_checks, "tolerance": 2e-2},
        "locality_order": locality,
        "device_copy_GBs": round(copy_gbs, 1) if copy_gbs else None,
        "checks": checks,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--g", type=int, default=0)
    ap.add_argument("--natural-order", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the FP64 oracle run over every output (profiling runs)")
    ap.add_argument("--cache-dir", default=None,
                    help="directory for the generated tensor (.npz), reused when present")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the gather ceiling and the fused-remap and unpacked-record "
                         "sweeps")
    ap.add_argument("--cpu-sample", type=int, default=30_000_000,
                    help="nonzeros the CPU oracle baseline processes at most")
    ap.add_argument("--oracle-threads", type=int, default=8,
                    help="threads (one per mode) of the full FP64 oracle run that "
                         "gives the errors over every output row")
    ap.add_argument("--copy-calib-mb", type=int, default=256,
                    help="size of a plain device copy run for counter calibration")
    ap.add_argument("--rank-sweep", default="",
                    help="comma-separated ranks: sweep time against R on the same tensor")
    ap.add_argument("--locality", action="store_true",
                    help="also time a plan with the Morton locality order inside rows")
    ap.add_argument("--m-sweep", default="",
                    help="comma-separated super-shard sizes m (0 = default rule)")
    ap.add_argument("--g-sweep", default="",
                    help="comma-separated shard sizes g: plan and sweep time against g")
    ap.add_argument("--no-loss-workload", action="store_true",
                    help="with the default workload, skip the sampled-loss workload "
                         "(50M nonzeros, R = 64) whose forward + backward step is "
                         "reported in a block of the same line")
    ap.add_argument("--als-recovery", type=int, default=0, metavar="D",
                    help="after the main run: CP-ALS to convergence on a fully stored "
                         "planted rank-16 D x D x D tensor (D = 368: 49.8M nonzeros)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path "
              "(the super-shards of a mode would be split over GPUs, with the "
              "remap as an all-to-all between modes; not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    import oracle  # test infrastructure: error report and CPU baseline only
    from paper_2309_09131_amd import _abi
    from paper_2309_09131_amd import synthetic as syn
    from paper_2309_09131_amd.api import Plan

    dev = torch.device("cuda:0")
    fn = bench_loss if args.config == 4 else bench_sweep
    # all GPU work on one created stream (default priority): launches on the
    # legacy null stream carry implicit synchronisation with other streams
    # and measured about 5% slower back to back
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        rec = fn(args, torch, dev, syn, _abi, Plan, oracle)
        if args.config == 3 and not args.no_loss_workload:
            # the differentiation form on its own workload, in the same line:
            # loss + gradient step, residual-kernel roofline, oracle checks
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            largs = argparse.Namespace(**vars(args))
            largs.no_cpu_baseline = True
            largs.locality = False
            largs.copy_calib_mb = 0
            lrec = bench_loss(largs, torch, dev, syn, _abi, Plan, oracle)
            rec["loss_workload"] = {
                k: lrec[k] for k in ("config", "ms_per_step", "value", "unit", "value_is",
                                     "forward_ms", "residual_kernel_ms_per_mode",
                                     "loss_kernel", "roofline", "checks", "bf16")}
        if args.als_recovery > 0:
            rec["cp_als_recovery"] = als_recovery(torch, dev, Plan, args.als_recovery)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
