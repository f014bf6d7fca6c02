"""Seeded synthetic inputs for the sparse all-mode MTTKRP workloads.

This module is the only code shared between the FP64 oracle and the GPU
path.  It draws random numbers and shapes tensors; it computes no MTTKRP,
no remap and no CP-ALS arithmetic.  (The planted-model workload evaluates
the CP model once to build its values; that is input construction, checked
independently by the loss-at-truth statistics.)

Recipe (all draws from numpy PCG64, seed = 20230916 + config number):
  1. per-mode random permutation pi_n of range(I_n)   (Zipf workloads only)
  2. coordinate batches of 10M draws; inside a batch, mode 0..N-1 in turn.
     Zipf(s): rank k in 1..I_n with weight k^-s (truncated, float64 CDF),
     coordinate = pi_n[k-1].  Uniform: integers in [0, I_n).
  3. keep the first occurrence of each distinct coordinate tuple, in draw
     order; draw further batches until the target count of distinct tuples
     is reached; keep the target count of earliest first occurrences.
  4. one value per kept tuple, in that order: U(0,1) or lognormal(0,1).
  5. factors, modes 0..N-1, each I_n x R row-major float32: N(0,1).
  6. planted workload: factors A_true ~ U(0,1), x = float32(m + sigma*eps)
     with m the rank-R CP model value and sigma = 0.01 * RMS(m);
     evaluation factors ~ U(0,1) from seed + 1.

The five workloads mirror the paper's evaluation tensors (FROSTT, Table of
tensor characteristics) in shape class only: power-law index popularity
stands in for the real data, which is not used.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SYNTH_SO = os.path.join(_HERE, "libsynth.so")
_lib = None

BASE_SEED = 20230916
BATCH = 10_000_000


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SYNTH_SO):
            raise RuntimeError(
                f"{_SYNTH_SO} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_SYNTH_SO)
        lib.synth_inverse_cdf.argtypes = [ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p]
        lib.synth_inverse_cdf.restype = None
        lib.synth_dedupe_first.argtypes = [ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_int64, ctypes.c_void_p]
        lib.synth_dedupe_first.restype = ctypes.c_int64
        _lib = lib
    return _lib


def inverse_cdf(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    lib = _load()
    cdf = np.ascontiguousarray(cdf, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty(u.shape[0], dtype=np.int32)
    lib.synth_inverse_cdf(cdf.ctypes.data, cdf.shape[0], u.ctypes.data,
                          u.shape[0], out.ctypes.data)
    return out


def dedupe_first(coords: list[np.ndarray]) -> np.ndarray:
    """Indices of the first occurrence of each distinct tuple, ascending."""
    lib = _load()
    cols = [np.ascontiguousarray(c, dtype=np.int32) for c in coords]
    n = cols[0].shape[0]
    ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
    keep = np.empty(n, dtype=np.int64)
    nk = lib.synth_dedupe_first(len(cols), ptrs, n, keep.ctypes.data)
    if nk < 0:
        raise MemoryError("dedupe table allocation failed")
    return keep[:nk]


@dataclass
class Workload:
    name: str
    dims: tuple
    nnz: int
    rank: int
    coords: str            # "uniform" or "zipf"
    zipf_s: float = 0.0
    values: str = "uniform"   # "uniform" | "lognormal" | "planted"
    seed: int = BASE_SEED
    note: str = ""


WORKLOADS = {
    1: Workload("tensor3-1000x800x600-nnz100K-R16", (1000, 800, 600), 100_000,
                16, "uniform", values="uniform", seed=BASE_SEED + 1,
                note="uniform distinct coordinates; CP-ALS correctness case"),
    2: Workload("tensor3-50Kx40Kx30K-nnz20M-zipf1.2-R32", (50000, 40000, 30000),
                20_000_000, 32, "zipf", 1.2, "lognormal", BASE_SEED + 2,
                note="power-law indices, small modes (Nell-2 shape class)"),
    3: Workload("tensor4-1Mx500Kx20Kx2K-nnz100M-zipf1.1-R32",
                (1_000_000, 500_000, 20_000, 2_000), 100_000_000, 32, "zipf",
                1.1, "lognormal", BASE_SEED + 3,
                note="4-mode with one small mode (Delicious shape class)"),
    4: Workload("tensor3-200Kcube-nnz50M-planted-R64", (200_000,) * 3,
                50_000_000, 64, "uniform", values="planted",
                seed=BASE_SEED + 4, note="planted rank-64 CP model + 1% noise"),
    5: Workload("tensor5-2Mx1Mx100Kx5Kx500-nnz200M-zipf1.2-R16",
                (2_000_000, 1_000_000, 100_000, 5_000, 500), 200_000_000, 16,
                "zipf", 1.2, "lognormal", BASE_SEED + 5,
                note="5-mode with tiny trailing modes (Vast shape class)"),
}


@dataclass
class Tensor:
    dims: tuple
    idx: np.ndarray          # (N, nnz) int32, 0-based
    vals: np.ndarray         # (nnz,) float32
    rank: int
    factors: list = field(default_factory=list)   # N arrays (I_n, R) float32
    extra: dict = field(default_factory=dict)

    @property
    def nmodes(self):
        return len(self.dims)

    @property
    def nnz(self):
        return int(self.vals.shape[0])


def _zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    return cdf


def draw_coordinates(rng, dims, target, kind, s=0.0, batch=BATCH, progress=None):
    """Steps 1-3 of the recipe: distinct coordinate tuples, draw order."""
    N = len(dims)
    perms, cdfs = [], []
    if kind == "zipf":
        for n in range(N):
            perms.append(rng.permutation(dims[n]).astype(np.int32))
        for n in range(N):
            cdfs.append(_zipf_cdf(dims[n], s))
    chunks = [[] for _ in range(N)]
    total = 0

    def one_batch():
        for n in range(N):
            if kind == "zipf":
                u = rng.random(batch)
                chunks[n].append(perms[n][inverse_cdf(cdfs[n], u)])
            else:
                chunks[n].append(rng.integers(0, dims[n], batch, dtype=np.int64)
                                 .astype(np.int32))

    while total < target:
        one_batch()
        total += batch
        if progress:
            progress(f"drew {total} coordinate tuples")
    while True:
        cols = [np.concatenate(c) if len(c) > 1 else c[0] for c in chunks]
        chunks = [[c] for c in cols]
        keep = dedupe_first(cols)
        if progress:
            progress(f"{keep.shape[0]} distinct of {total} drawn (target {target})")
        if keep.shape[0] >= target:
            keep = keep[:target]
            return np.stack([c[keep] for c in cols]).astype(np.int32)
        need = target - keep.shape[0]
        ratio = max(keep.shape[0] / total, 1e-3)
        nb = max(1, int(np.ceil(1.5 * need / ratio / batch)))
        for _ in range(nb):
            one_batch()
            total += batch


def _planted_values(idx, factors, chunk=1 << 20):
    """CP model value for each coordinate (input construction, FP64)."""
    nnz = idx.shape[1]
    out = np.empty(nnz, dtype=np.float64)
    for a in range(0, nnz, chunk):
        b = min(nnz, a + chunk)
        p = factors[0][idx[0, a:b]].astype(np.float64)
        for n in range(1, len(factors)):
            p *= factors[n][idx[n, a:b]]
        out[a:b] = p.sum(axis=1)
    return out


def generate(cfg: int, nnz: int | None = None, dims: tuple | None = None,
             rank: int | None = None, batch: int = BATCH,
             cache_dir: str | None = None, progress=None) -> Tensor:
    """Build workload `cfg` (1..5); nnz/dims/rank override for scaled cases."""
    w = WORKLOADS[cfg]
    dims = tuple(int(d) for d in (dims or w.dims))
    nnz = int(nnz or w.nnz)
    R = int(rank or w.rank)
    key = f"c{cfg}_{'x'.join(map(str, dims))}_{nnz}_{R}_{batch}"
    if cache_dir:
        path = os.path.join(cache_dir, key + ".npz")
        if os.path.exists(path):
            z = np.load(path)
            N = len(dims)
            t = Tensor(dims, z["idx"], z["vals"], R,
                       [z[f"f{n}"] for n in range(N)])
            for k in z.files:
                if k.startswith("x_"):
                    t.extra[k[2:]] = z[k]
            return t
    rng = np.random.Generator(np.random.PCG64(w.seed))
    idx = draw_coordinates(rng, dims, nnz, w.coords, w.zipf_s, batch, progress)
    extra = {}
    if w.values == "lognormal":
        vals = rng.lognormal(0.0, 1.0, nnz).astype(np.float32)
    elif w.values == "uniform":
        vals = rng.random(nnz).astype(np.float32)
    else:  # planted
        a_true = [rng.random((d, R)).astype(np.float32) for d in dims]
        m = _planted_values(idx, a_true)
        sigma = 0.01 * float(np.sqrt(np.mean(m * m)))
        vals = (m + sigma * rng.standard_normal(nnz)).astype(np.float32)
        for n, a in enumerate(a_true):
            extra[f"true{n}"] = a
        extra["sigma"] = np.array(sigma)
    if w.values == "planted":
        rng2 = np.random.Generator(np.random.PCG64(w.seed + 1))
        factors = [rng2.random((d, R)).astype(np.float32) for d in dims]
    else:
        factors = [rng.standard_normal((d, R)).astype(np.float32) for d in dims]
    t = Tensor(dims, idx, vals, R, factors, extra)
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        arrs = {"idx": idx, "vals": vals}
        for n, f in enumerate(factors):
            arrs[f"f{n}"] = f
        for k, v in extra.items():
            arrs["x_" + k] = v
        np.savez(os.path.join(cache_dir, key + ".npz"), **arrs)
    return t


def random_tensor(dims, nnz, rank, seed, values="uniform", factors="normal",
                  distinct=True, int_values=False, zipf_s=0.0):
    """Small test tensors.

    int_values: values integer in [1,4] and factor entries integer in
    [-2,2], so every product and partial sum is an exactly representable
    integer (used for bit-exact checks).
    distinct=False keeps duplicate coordinates (drawn with replacement).
    zipf_s > 0 draws coordinates from a truncated Zipf over shuffled ids.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dims = tuple(int(d) for d in dims)
    N = len(dims)
    if distinct:
        space = 1
        for d in dims:
            space *= d
        if nnz > space:
            raise ValueError("more distinct nonzeros than coordinates")
        kind = "zipf" if zipf_s > 0 else "uniform"
        idx = draw_coordinates(rng, dims, nnz, kind, zipf_s,
                               batch=max(64, 2 * nnz)) if nnz > 0 else \
            np.zeros((N, 0), np.int32)
    else:
        idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
    if int_values:
        vals = rng.integers(1, 5, nnz).astype(np.float32)
        fac = [rng.integers(-2, 3, (d, rank)).astype(np.float32) for d in dims]
    else:
        if values == "lognormal":
            vals = rng.lognormal(0.0, 1.0, nnz).astype(np.float32)
        else:
            vals = rng.random(nnz).astype(np.float32)
        if factors == "uniform":
            fac = [rng.random((d, rank)).astype(np.float32) for d in dims]
        else:
            fac = [rng.standard_normal((d, rank)).astype(np.float32)
                   for d in dims]
    return Tensor(dims, idx, vals, rank, fac)
