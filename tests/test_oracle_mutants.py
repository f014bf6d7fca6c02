"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a copy of oracle/oracle.c (a dropped
term, a wrong index or sign, a transposed or reversed operand, a wrong tie
rule or rounding), builds it with gcc into a temporary library, and runs the
pin suite (tests/test_oracle_pins.py) against that library in a child
process.  Every planted mistake must make at least one pin fail.  The
mistakes are chosen so that the mutant still reads and writes only inside
its buffers.  Nothing here touches the GPU library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement); the first occurrence is replaced
MUTANTS = [
    # MTTKRP (Sec. II-B, Eq. of the mode-n MTTKRP)
    ("mttkrp: value dropped", "double v = vals[e];", "double v = 1.0;"),
    ("mttkrp: output mode's own factor multiplied in",
     "if (w == mode) continue;", "if (w == mode && 0) continue;"),
    ("mttkrp: input row taken at the next mode's coordinate",
     "const double *row = factors[w] + (int64_t)idx[(int64_t)w * nnz + e] * R;",
     "const double *row = factors[w] + (int64_t)(idx[(int64_t)((w + 1) % N) * nnz + e]"
     " % dims[w]) * R;"),
    ("mttkrp: rank index reversed", "out[i * R + r] += v * ell[r];",
     "out[i * R + r] += v * ell[R - 1 - r];"),
    ("mttkrp: |.| scale keeps the value's sign",
     "if (out_abs) out_abs[i * R + r] += fabs(v) * ela[r];",
     "if (out_abs) out_abs[i * R + r] += v * ela[r];"),
    ("mttkrp rows: last nonzero kept instead of the sum", "out[k * R + r] += p;",
     "out[k * R + r] = p;"),
    ("mttkrp rows: factors added instead of multiplied", "p *= a; pa *= fabs(a);",
     "p += a; pa *= fabs(a);"),
    ("mttkrp rows: a repeated row listed only at its last listing",
     "if (k0 == k) continue;", "continue;"),
    # layouts (Sec. III-B, Alg. Dynasor remap)
    ("layout L_0: keys in the wrong cyclic direction",
     "int m = (k == 0) ? 0 : g_N - k;", "int m = (k == 0) ? 0 : k;"),
    ("layout L_0: equal keys in reverse input order",
     "return (a < b) ? -1 : (a > b);", "return (a > b) ? -1 : (a < b);"),
    ("row pointers: prefix sum stops one row short",
     "for (int64_t i = 0; i < dims[n]; ++i) rp[i + 1] += rp[i];",
     "for (int64_t i = 0; i + 1 < dims[n]; ++i) rp[i + 1] += rp[i];"),
    ("remap target: the source slot recorded instead of the destination",
     "perm[(int64_t)n * nnz + i] = dst;", "perm[(int64_t)n * nnz + i] = i;"),
    # locality order (Sec. V-J, Z-Morton)
    ("locality: both coordinates on the even Morton bits",
     "z |= (uint64_t)((a >> k) & 1u) << (2 * k + 1);",
     "z |= (uint64_t)((a >> k) & 1u) << (2 * k);"),
    ("locality: leading inputs taken in the wrong cyclic direction",
     "const int m1 = (n + N - 1) % N, m2 = (n + N - 2) % N;",
     "const int m1 = (n + 1) % N, m2 = (n + 2) % N;"),
    ("locality: remap target inverted",
     "for (int64_t i = 0; i < nnz; ++i) perm[(int64_t)n * nnz + i] = slot[cur[i]];",
     "for (int64_t i = 0; i < nnz; ++i) perm[(int64_t)n * nnz + i] = cur[slot[i]];"),
    # shards and schedule (Sec. III-A, IV-A)
    ("shards: count rounded down", "ss_shards[j] = (b - a + g - 1) / g;",
     "ss_shards[j] = (b - a) / g;"),
    ("shards: super-shard id of a shard is its own index", "shard_ss[s] = j;",
     "shard_ss[s] = s;"),
    ("schedule: ties go to the highest bin", "if (load[i] < load[best]) best = i;",
     "if (load[i] <= load[best]) best = i;"),
    ("schedule: lightest super-shard first", "(weight[ord[b]] < weight[x] ||",
     "(weight[ord[b]] > weight[x] ||"),
    # CP-ALS (Alg. cp-als)
    ("cp-als: Hadamard includes the updated mode's Gram", "if (w != n)",
     "if (w != n || 1)"),
    ("cp-als: lambda is the squared column norm", "lambda[r] = sqrt(s);",
     "lambda[r] = s;"),
    ("cp-als: Gram matrix keeps only its diagonal", "G[p * R + q] = s;",
     "G[p * R + q] = (p == q) ? s : 0.0;"),
    ("cp-als: Cholesky column not divided by the pivot", "V[i * R + j] = s / d;",
     "V[i * R + j] = s;"),
    ("cp-als: back substitution with L instead of its transpose",
     "for (int k = i + 1; k < R; ++k) s -= L[k * R + i] * x[k];",
     "for (int k = i + 1; k < R; ++k) s -= L[i * R + k] * x[k];"),
    ("cp-als: ||X||^2 summed as |x|", "for (int64_t e = 0; e < nnz; ++e) xx += vals[e] * vals[e];",
     "for (int64_t e = 0; e < nnz; ++e) xx += fabs(vals[e]);"),
    ("cp-als: ||Xhat||^2 with a repeated lambda index", "nrm += lambda[p] * lambda[q] * h;",
     "nrm += lambda[p] * lambda[p] * h;"),
    ("cp-als: ridge left out", "for (int p = 0; p < R; ++p) Vc[p * R + p] += 1e-12 * tr / R;",
     "for (int p = 0; p < R; ++p) Vc[p * R + p] += 0.0 * tr / R;"),
    ("cp-als: fit drops the factor 2 of the cross term",
     "double res2 = xx - 2.0 * inner + nrm;", "double res2 = xx - inner + nrm;"),
    # sampled loss and gradient (Eq. 1, Sec. II-C)
    ("loss: gradient sign flipped", "grads[k][i * R + r] += -2.0 * rho * p;",
     "grads[k][i * R + r] += 2.0 * rho * p;"),
    ("loss: gradient multiplies in the differentiated factor", "if (n != k)",
     "if (n != k || 1)"),
    ("loss: model sums only the first rank", "m += p;", "m += (r == 0) ? p : 0.0;"),
    ("loss: |rho| summed instead of rho^2", "L += rho * rho;", "L += fabs(rho);"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
oracle._SO = {lib!r}
oracle._lib = None
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider",
                      {pins!r}]))
"""


def _run_mutant(case, tmp):
    name, old, new = case
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site not found: {name}"
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)[:60]
    c_path = os.path.join(tmp, tag + ".c")
    so_path = os.path.join(tmp, tag + ".so")
    with open(c_path, "w") as fh:
        fh.write(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", so_path,
                           c_path, "-lm"])
    code = RUNNER.format(root=ROOT, lib=so_path,
                         pins=os.path.join(ROOT, "tests", "test_oracle_pins.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                       text=True, timeout=300)
    return name, r.returncode, r.stdout[-2000:] + r.stderr[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda c: _run_mutant(c, str(tmp_path)), MUTANTS))
    survived = [(n, out) for n, rc, out in results if rc == 0]
    # a pin failed: pytest's exit status 1 with a failure in its summary
    # (anything else, such as an import error in the runner, is no kill)
    crashed = [(n, rc, out) for n, rc, out in results
               if rc != 0 and not (rc == 1 and " failed" in out)]
    assert not crashed, crashed
    assert not survived, "planted mistakes that no pin catches: " + \
        "; ".join(n for n, _ in survived)


def test_the_unmutated_oracle_passes_the_same_runner(tmp_path):
    """Control: the runner itself passes on the oracle as committed."""
    name, rc, out = _run_mutant(("control", "#include", "#include"), str(tmp_path))
    assert rc == 0, out
