"""AddressSanitizer / UndefinedBehaviorSanitizer builds of the host code, CPU
only.

* The FP64 oracle, built with gcc's sanitizers, runs every function on
  small tensors (duplicates, empty rows, two to five modes).
* The host side of the GPU library, built with hipcc with the sanitizers on
  the host pass only, runs the host logic: workspace layout for many shapes
  and every argument-error path.  The kernel launchers of the per-mode-count
  translation units are stubbed, since nothing is launched without a GPU;
  the kernels themselves are covered by the determinism (bit-identical
  repeat) tests on the GPU.

Each library runs in a subprocess with its sanitizer runtime preloaded; any
sanitizer report fails the test.
"""
import glob
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_09131_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")

SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_asan():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def _clang_asan():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    for pat in ("llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so",
                "llvm/lib/clang/*/lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"):
        hits = sorted(glob.glob(os.path.join(rocm, pat)))
        if hits:
            return hits[-1]
    return None


def _run(script, preload, tmp_path):
    env = dict(os.environ, LD_PRELOAD=preload, **SAN_ENV)
    f = tmp_path / "run.py"
    f.write_text(script)
    r = subprocess.run([sys.executable, str(f)], env=env, capture_output=True, text=True,
                       timeout=600, cwd=ROOT)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "ERROR: AddressSanitizer" not in report, report[-4000:]
    assert "runtime error" not in report, report[-4000:]
    assert "sanitizer active" in r.stdout, report[-2000:]
    return r.stdout


ACTIVE = f"""
import ctypes, sys
sys.path.insert(0, {ROOT!r})
assert hasattr(ctypes.CDLL(None), "__asan_report_load4")
print("sanitizer active")
"""


def test_oracle_under_asan_ubsan(tmp_path):
    rt = _gcc_asan()
    if rt is None:
        pytest.skip("gcc libasan not found")
    so = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC", "-shared",
                           "-std=c99", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-o", str(so),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
    script = ACTIVE + textwrap.dedent(f"""
        import numpy as np
        import oracle
        oracle._SO = {str(so)!r}
        oracle._lib = None
        rng = np.random.default_rng(5)
        cases = [((7, 5, 6), 120), ((40, 3, 30, 5), 600), ((9, 2, 11, 3, 4), 300),
                 ((30, 20), 200), ((1, 8, 6), 40), ((50, 40, 30), 0)]
        for dims, nnz in cases:
            N = len(dims)
            idx = np.stack([rng.integers(0, d, nnz) for d in dims]).astype(np.int32)
            if nnz:
                idx[:, 1] = idx[:, 0]                     # a duplicate coordinate
            vals = rng.random(nnz)
            facs = [rng.standard_normal((d, 4)) for d in dims]
            for n in range(N):
                m, a = oracle.mttkrp(dims, idx, vals, facs, n, with_abs=True)
                sub, _ = oracle.mttkrp_rows(dims, idx, vals, facs, n, [0, dims[n] - 1])
                assert np.allclose(sub, m[[0, dims[n] - 1]])
            l0 = oracle.canonical_order(idx)
            lay, perm, rps = oracle.remap_replay(dims, idx, l0)
            llay, lperm = oracle.locality_layouts(dims, idx)
            for n in range(N):
                sh = oracle.shards(dims[n], rps[n], max(1, dims[n] // 3), 16)
                oracle.lpt(sh["ss_shards"], 3)
            if nnz:
                oracle.cp_als_sweep(dims, idx, vals, facs)
                oracle.cp_loss_grad(dims, idx, vals, facs)
                oracle.cp_loss_grad(dims, idx, vals, facs, want_grad=False)
        print("oracle ok")
    """)
    out = _run(script, rt, tmp_path)
    assert "oracle ok" in out


# launchers of the per-mode-count translation units: never reached without a
# GPU (the host checks return before any launch)
STUBS = """
#include "launch.hpp"
namespace mk {
#define STUB(N)                                                                          \\
    template <> hipError_t launch_mttkrp<N>(const Args &, int, LaneCfg, int, unsigned,   \\
                                            hipStream_t) { return hipErrorNotSupported; } \\
    template <> hipError_t launch_remap<N>(const uint32_t *, uint32_t *, const int32_t *, \\
                                           int64_t, int, const RemapMap &, hipStream_t)   \\
    { return hipErrorNotSupported; }                                                      \\
    template <> hipError_t launch_pack<N>(const int32_t *, const float *, const int32_t *, \\
                                          int64_t, uint32_t *, int, PackMap, hipStream_t)  \\
    { return hipErrorNotSupported; }
STUB(2) STUB(3) STUB(4) STUB(5) STUB(6) STUB(7) STUB(8)
}
"""


def test_host_library_under_asan_ubsan(tmp_path):
    rt = _clang_asan()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("hipcc or the clang ASan runtime not found")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", INCLUDE, "-I", CSRC]
    stub = tmp_path / "stubs.hip"
    stub.write_text(STUBS)
    objs = []
    for src in (os.path.join(CSRC, "mttkrp_lib.hip"), str(stub)):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.check_call([HIPCC, *flags, "-c", "-o", obj, src],
                              stderr=subprocess.DEVNULL)
        objs.append(obj)
    so = str(tmp_path / "libmttkrp_san.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", "-o", so, *objs])
    script = ACTIVE + textwrap.dedent(f"""
        import ctypes
        lib = ctypes.CDLL({so!r})
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.mttkrp_status_str.restype = ctypes.c_char_p
        lib.mttkrp_last_error.restype = ctypes.c_char_p
        lib.mttkrp_last_error.argtypes = [vp]
        lib.mttkrp_plan_workspace.argtypes = [ctypes.c_int, vp, i64, ctypes.c_int, vp, vp]

        class Opts(ctypes.Structure):
            _fields_ = [("g", ctypes.c_int32), ("m", ctypes.c_int32 * 8),
                        ("workers", ctypes.c_int32), ("flags", ctypes.c_uint32)]

        def ws(dims, nnz, R, opts=None):
            d = (i64 * len(dims))(*dims)
            out = ctypes.c_size_t(0)
            st = lib.mttkrp_plan_workspace(len(dims), d, nnz, R,
                                           ctypes.byref(opts) if opts else None,
                                           ctypes.byref(out))
            return st, out.value

        MAX_NNZ = (1 << 31) - (1 << 20)
        ok = [((10, 20, 30), 1000, 16), ((1, 1), 0, 1), ((2,) * 8, 255, 256),
              ((300000, 200000, 5000), 5000, 32), ((2**31 - 1, 3), 77, 5),
              ((1000000, 500000, 20000, 2000), 100000000, 32),
              ((2000000, 1000000, 100000, 5000, 500), 200000000, 16),
              ((1 << 20,) * 3, MAX_NNZ, 16)]
        for dims, nnz, R in ok:
            st, b = ws(dims, nnz, R)
            assert st == 0 and b > 0, (dims, nnz, R, st)
        for flags in (0, 1, 2, 4, 8, 16, 32, 63):
            o = Opts()
            o.g, o.workers, o.flags = 100, 7, flags
            for k in range(8):
                o.m[k] = 3 + k
            assert ws((50, 40, 30, 20), 9999, 24, o)[0] == 0
        bad = [((10,), 5, 4), ((2,) * 9, 5, 4), ((10, 20), 5, 0), ((10, 20), 5, 257),
               ((10, 0, 3), 5, 4), ((10, 20), -1, 4), ((10, 20), MAX_NNZ + 1, 4),
               ((10, -4), 5, 4)]
        for dims, nnz, R in bad:
            st, _ = ws(dims, nnz, R)
            assert st == 1, (dims, nnz, R, st)
            assert lib.mttkrp_last_error(None)
        o = Opts()
        o.g = -5
        assert ws((10, 20), 5, 4, o)[0] == 1
        out = ctypes.c_size_t(0)
        assert lib.mttkrp_plan_workspace(3, None, 5, 4, None, ctypes.byref(out)) == 1
        # plan: argument errors before any device work
        h = ctypes.c_void_p(None)
        d3 = (i64 * 3)(10, 20, 30)
        assert lib.mttkrp_plan(3, d3, 100, None, None, 4, None, None, 0, None,
                               ctypes.byref(h)) == 1
        # every call on a NULL plan is EINVAL
        assert lib.mttkrp_mode(None, 0, None, 0, None, 0, None) == 1
        assert lib.mttkrp_all_modes(None, None, 0, None, None) == 1
        assert lib.remap(None, 0, None) == 1
        assert lib.cp_loss_grad(None, None, 0, None, None, None, None) == 1
        assert lib.cp_als_sweep(None, None, 0, None, None, None, None) == 1
        assert lib.cp_als_sweep_static(None, None, 0, None, None, None) == 1
        assert lib.cp_als(None, None, 0, None, None, 1, ctypes.c_double(0.0), None, None,
                          None, None) == 1
        assert lib.mttkrp_plan_query(None, 0, 0, None, 0, None) == 1
        v = i64(0)
        assert lib.mttkrp_plan_info(None, 0, 0, ctypes.byref(v)) == 1
        assert lib.mttkrp_profile(None, 1) == 1
        assert lib.mttkrp_plan_destroy(None) == 1
        for st in range(-2, 9):
            assert lib.mttkrp_status_str(st)
        print("host library ok")
    """)
    out = _run(script, rt, tmp_path)
    assert "host library ok" in out
