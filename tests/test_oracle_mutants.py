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
    ("mttkrp rows: last nonzero kept instead of the sum", "out[k * R + r] += p;",
     "out[k * R + r] = p;"),
    ("mttkrp rows: factors added instead of multiplied", "p *= a; pa *= fabs(a);",
     "p += a; pa *= fabs(a);"),
    # layouts (Sec. III-B, Alg. Dynasor remap)
    ("layout L_0: keys in the wrong cyclic direction",
     "int m = (k == 0) ? 0 : g_N - k;", "int m = (k == 0) ? 0 : k;"),
    ("layout L_0: equal keys in reverse input order",
     "return (a < b) ? -1 : (a > b);", "return (a > b) ? -1 : (a < b);"),
    ("row pointers: prefix sum stops one row short",
     "for (int64_t i = 0; i < dims[n]; ++i) rp[i + 1] += rp[i];",
     "for (int64_t i = 0; i + 1 < dims[n]; ++i) rp[i + 1] += rp[i];"),
    # shards and schedule (Sec. III-A, IV-A)
    ("shards: count rounded down", "ss_shards[j] = (b - a + g - 1) / g;",
     "ss_shards[j] = (b - a) / g;"),
    ("schedule: ties go to the highest bin", "if (load[i] < load[best]) best = i;",
     "if (load[i] <= load[best]) best = i;"),
    ("schedule: lightest super-shard first", "(weight[ord[b]] < weight[x] ||",
     "(weight[ord[b]] > weight[x] ||"),
    # CP-ALS (Alg. cp-als)
    ("cp-als: Hadamard includes the updated mode's Gram", "if (w != n)",
     "if (w != n || 1)"),
    ("cp-als: lambda is the squared column norm", "lambda[r] = sqrt(s);",
     "lambda[r] = s;"),
    ("cp-als: fit drops the factor 2 of the cross term",
     "double res2 = xx - 2.0 * inner + nrm;", "double res2 = xx - inner + nrm;"),
    # sampled loss and gradient (Eq. 1, Sec. II-C)
    ("loss: gradient sign flipped", "grads[k][i * R + r] += -2.0 * rho * p;",
     "grads[k][i * R + r] += 2.0 * rho * p;"),
    ("loss: gradient multiplies in the differentiated factor", "if (n != k)",
     "if (n != k || 1)"),
    ("loss: model sums only the first rank", "m += p;", "m += (r == 0) ? p : 0.0;"),
]

RUNNER = r"""
import sys
sys.path.insert(0, {root!r})
import oracle
oracle._SO = {lib!r}
oracle._lib = None
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
    return name, r.returncode, r.stdout[-2000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda c: _run_mutant(c, str(tmp_path)), MUTANTS))
    survived = [(n, out) for n, rc, out in results if rc == 0]
    crashed = [(n, rc, out) for n, rc, out in results if rc not in (0, 1)]
    assert not crashed, crashed
    assert not survived, "planted mistakes that no pin catches: " + \
        "; ".join(n for n, _ in survived)


def test_the_unmutated_oracle_passes_the_same_runner(tmp_path):
    """Control: the runner itself passes on the oracle as committed."""
    name, rc, out = _run_mutant(("control", "#include", "#include"), str(tmp_path))
    assert rc == 0, out
