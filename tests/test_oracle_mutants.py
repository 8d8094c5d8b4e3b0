"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check
that at least one pin catches each of them.  This is what makes the pins a
check on the oracle rather than a restatement of it."""
import os
import shutil
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests.oracle_pins import PINS

# (name, exact text in hln_oracle.c, replacement)
MUTANTS = [
    ("cc-numerator-R", "double reach = (double)(R[i] - 1);", "double reach = (double)(R[i]);"),
    ("cc-no-wf-factor", "cc[i] = q1 * q2;", "cc[i] = q1;"),
    ("bfs-step-2", "dist[w] = dist[u] + 1;", "dist[w] = dist[u] + 2;"),
    ("h2-at-distance-1", "if (dist[u] == 2) at2 += 1;", "if (dist[u] == 1) at2 += 1;"),
    ("reach-without-self", "reached += 1;", "if (dist[u] > 0) reached += 1;"),
    ("ecc-off", "if (dist[u] > far) far = dist[u];", "if (dist[u] > far) far = dist[u] + 1;"),
    ("keep-self-loops", "if (u == v) continue;                 /* simple graph: drop self-loops */",
     "if (u == v && 0) continue;"),
    ("keep-duplicates", "continue;                         /* simple graph: drop duplicates */", ";"),
    ("and-r-minus-1", "(copies == r)", "(copies >= r - 1)"),
    ("or-needs-two", "(copies >= 1)", "(copies >= 2)"),
    ("penalty-n-minus-1", "P[i] = S[i] + (int64_t)n * (int64_t)(n - R[i]);",
     "P[i] = S[i] + (int64_t)(n - 1) * (int64_t)(n - R[i]);"),
    ("mean-count-minus-1", "return total / (double)count;", "return total / (double)(count > 1 ? count - 1 : 1);"),
    ("above-strict", "if (x[i] >= mean) ids[c++] = i;", "if (x[i] > mean) ids[c++] = i;"),
    ("topk-tie-desc", "return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);\n}\n\nstatic int rank_asc",
     "return x->id > y->id ? -1 : (x->id < y->id ? 1 : 0);\n}\n\nstatic int rank_asc"),
    ("topk-ascending", "if (x->s != y->s) return x->s > y->s ? -1 : 1;",
     "if (x->s != y->s) return x->s < y->s ? -1 : 1;"),
    ("cc2-min", "if (l == 0 || p > best) best = p;", "if (l == 0 || p < best) best = p;"),
    ("cc2-score-n", "score[u] = est[u] > 0 ? (double)(n - 1) / (double)est[u] : 0.0;",
     "score[u] = est[u] > 0 ? (double)n / (double)est[u] : 0.0;"),
    ("cc2-score-wf", "score[u] = est[u] > 0 ? (double)(n - 1) / (double)est[u] : 0.0;",
     "score[u] = est[u] > 0 ? ((double)(n - 1) / (double)est[u]) * ((double)(n - 1) / (double)n) : 0.0;"),
    ("cc2-unpenalised", "int64_t p = S[l][u] + (int64_t)n * (int64_t)(n - R[l][u]);", "int64_t p = S[l][u];"),
    ("naive-union", "in[u] = in[u] && keep[u];", "in[u] = (l == 0) ? keep[u] : (in[u] || keep[u]);"),
    ("naive-topk-any-layer", "for (int32_t u = 0; u < n; ++u) if (hits[u] == r) ids[c++] = u;",
     "for (int32_t u = 0; u < n; ++u) if (hits[u] >= 1) ids[c++] = u;"),
    ("naive-topk-k-plus-1", "int32_t c = oracle_topk_desc(n, cc[l], k, top);",
     "int32_t c = oracle_topk_desc(n, cc[l], k + 1, top);"),
    ("sample-self-counted", "int32_t q = RQ[v] - self;", "int32_t q = RQ[v];"),
    ("sample-population-n", "double c = (double)(n_pop - 1) / (double)(n - 1);", "double c = 1.0;"),
    ("sample-sums-off-by-one", "SQ[u] += dist[u];", "SQ[u] += dist[u] + 1;"),
    ("cc1-degree-max", "if (l == 0 || d < best) best = d;", "if (l == 0 || d > best) best = d;"),
    ("cc1-eq3-min", "if (l == 0 || avg_l > avg) avg = avg_l;", "if (l == 0 || avg_l < avg) avg = avg_l;"),
    ("cc1-central-not-strict", "return m > 0 && ratio < avg;", "return m > 0 && ratio <= avg;"),
    ("cc1-unreachable-zero", "int64_t P = S[l][u] + (int64_t)n * (int64_t)(n - R[l][u]);", "int64_t P = S[l][u];"),
    ("cc1-overlap-over-largest", "if (smallest < 0 || size < smallest) smallest = size;",
     "if (smallest < 0 || size > smallest) smallest = size;"),
    ("cc1-any-layer-cc", "common[u] = common[u] && keep[u];", "common[u] = common[u] || keep[u];"),
]


@pytest.fixture(scope="module")
def workdir():
    d = tempfile.mkdtemp(prefix="hln_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(workdir, name, old, new):
    with open(O._SRC) as f:
        src = f.read()
    assert src.count(old) == 1, "mutation site for %s not found exactly once" % name
    path_c = os.path.join(workdir, name + ".c")
    with open(path_c, "w") as f:
        f.write(src.replace(old, new))
    path_so = os.path.join(workdir, name + ".so")
    subprocess.check_call(["gcc", *O._CFLAGS, "-w", "-o", path_so, path_c])
    variant = O.Variant(path_so)
    caught = []
    for pin in PINS:               # the first pin that catches it is enough
        try:
            pin(variant)
        except AssertionError:
            caught.append(pin.__name__)
        except Exception as e:  # a crash in a pin also counts as detection
            caught.append("%s(%s)" % (pin.__name__, type(e).__name__))
        if caught:
            break
    assert caught, "planted mistake %s passed every pin" % name
