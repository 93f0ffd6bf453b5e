"""Plant plausible mistakes in copies of the oracle (CPU only) and check that the pins catch
every one of them: a dropped term, a transposed operand, a wrong index or sign, an
off-by-one capacity test, a wrong variance denominator, a wrong rounding rule."""
import os
import tempfile

import pytest

import oracle
from oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, exact text in oracle.c, replacement)
MUTANTS = [
    ("drop_inner_arc", "if (p < i - 1) inner += DIST(tour[p], tour[p + 1]);", ";"),
    ("transpose_inner_arc", "inner += DIST(tour[p], tour[p + 1]);",
     "inner += DIST(tour[p + 1], tour[p]);"),
    ("transpose_first_arc", "int64_t route = DIST(0, tour[p]) + inner + DIST(tour[i - 1], 0);",
     "int64_t route = DIST(tour[p], 0) + inner + DIST(tour[i - 1], 0);"),
    ("transpose_last_arc", "int64_t route = DIST(0, tour[p]) + inner + DIST(tour[i - 1], 0);",
     "int64_t route = DIST(0, tour[p]) + inner + DIST(0, tour[i - 1]);"),
    ("capacity_off_by_one", "if (load > Q) break;", "if (load >= Q) break;"),
    ("wrong_f_index", "int64_t cand = f[p] + route;",
     "int64_t cand = f[p > 0 ? p - 1 : 0] + route;"),
    ("wrong_min_sign", "if (cand < best) best = cand;", "if (cand > best || best == INT64_MAX) best = cand;"),
    ("demand_index", "load += q[p]; /* q_{s_{p+1}} */", "load += q[i - 1];"),
    ("base_case", "f[0] = 0;\n    int64_t w_extra", "f[0] = DIST(0, tour[0]);\n    int64_t w_extra"),
    ("population_variance", "*var = ((double)num / (double)S) / (double)(S - 1);",
     "*var = ((double)num / (double)S) / (double)S;"),
    ("round_down", "return (m > k * k + k) ? k + 1 : k;", "return k;"),
    ("round_half_rule", "return (m > k * k + k) ? k + 1 : k;", "return (m >= k * k + k) ? k + 1 : k;"),
    ("mask_strict", "if (load <= Q) {\n                m = p;", "if (load < Q) {\n                m = p;"),
    ("eq3_drop_return_arc", "route += DIST(tour[i - 1], 0);", ";"),
    ("sumsq_truncated", "sumsq += (unsigned __int128)(c * c);", "sumsq += (uint64_t)(c * c) & 0xffffffffffffull;"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_to(str(path), str(tmp_path / f"lib{name}.so"))
    caught = []
    for pin in ALL_PINS:
        try:
            pin(lib=lib)
        except (AssertionError, oracle.OracleError):
            caught.append(pin.__name__)
    assert caught, f"no pin caught mutant {name}"
