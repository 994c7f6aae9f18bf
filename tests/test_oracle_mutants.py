"""The oracle's pins catch plausible mistakes: each mutant below is a
one-line change to fc_oracle.c (a dropped term, a flipped sign, a wrong log
base, a transposed index, an off-by-one, a missing symmetry), compiled on the
CPU and run against the pin battery of test_oracle.py; every mutant must fail
at least one pin.  Mistakes are planted only in copies of the oracle."""
import ctypes
import os
import subprocess

import pytest

from oracle import oracle as orc
from tests import test_oracle as pins

SRC = os.path.join(os.path.dirname(orc.__file__), "fc_oracle.c")

MUTANTS = [
    ("count: wrong digit order", "idx = idx * arity[v] + s;\n        }\n        table[idx] += 1;",
     "idx = idx + s * arity[v];\n        }\n        if (idx >= cells) idx = cells - 1;\n        table[idx] += 1;"),
    ("count: last instance dropped",
     "sizeof(int64_t));\n    for (int64_t p = 0; p < m; ++p) {",
     "sizeof(int64_t));\n    for (int64_t p = 0; p + 1 < m; ++p) {"),
    ("assignment: inverted match", "match = cols[(int64_t)vars[t] * m + p] == states[t];",
     "match = cols[(int64_t)vars[t] * m + p] != states[t];"),
    ("ll: inverted ratio", "log2((double)nijk / (double)nij)", "log2((double)nij / (double)nijk)"),
    ("ll: natural log", "acc_add(&a, (double)nijk * log2((double)nijk / (double)nij));",
     "acc_add(&a, (double)nijk * log((double)nijk / (double)nij));"),
    ("mdl: r instead of r-1", "(double)q * (double)(r - 1);", "(double)q * (double)r;"),
    ("mdl: penalty without 1/2", "double penalty = 0.5 * log2", "double penalty = 1.0 * log2"),
    ("bdeu: a_jk = ess/q", "double ajk = ess / ((double)r * (double)q);", "double ajk = ess / (double)q;"),
    ("bdeu: dropped lnG(a_j)", "        acc_add(&a, lg_aj);\n", "\n"),
    ("bdeu: sign of lnG(a_j + N_ij)", "acc_add(&a, -lgamma(aj + (double)nij));",
     "acc_add(&a, lgamma(aj + (double)nij));"),
    ("mi: weight N/N_ij", "acc_add(&a, ((double)nijk / (double)m) * log1p(x));",
     "acc_add(&a, ((double)nijk / (double)nij) * log1p(x));"),
    ("mi: ratio without m", "int64_t num = m * nijk - den;",
     "int64_t num = nijk - den;"),
    ("gram: no symmetric copy", "gram[(int64_t)b * n + a] = gram[(int64_t)a * n + b];", ";"),
    ("gram: diagonal dropped", "for (int32_t y = x; y < len[i]; ++y)",
     "for (int32_t y = x + 1; y < len[i]; ++y)"),
    ("sparse: counts restart", "counts_out[nd - 1] += 1;", "counts_out[nd - 1] = 1;"),
]


def battery():
    """The pins, as plain calls; returns the number that fail."""
    checks = [pins.test_fig1_count_example, pins.test_fig1_query_table_and_seven_configurations,
              pins.test_fig1_reducer_closed_forms, pins.test_mi_special_cases,
              pins.test_arm_hand_example]
    checks += [lambda s=s: pins.test_count_matches_brute_force(s) for s in range(6)]
    checks += [lambda s=s: pins.test_count_invariants(s) for s in range(4)]
    checks += [lambda s=s: pins.test_single_variable_is_bincount(s) for s in range(2)]
    checks += [lambda s=s: pins.test_count_assignment_is_table_cell(s) for s in range(2)]
    checks += [lambda s=s: pins.test_ll_is_conditional_entropy(s) for s in range(3)]
    checks += [lambda s=s: pins.test_mdl_deterministic_child(s) for s in range(2)]
    checks += [lambda s=s: pins.test_bdeu_is_polya_urn_likelihood(s, 1.0) for s in range(3)]
    checks += [lambda s=s: pins.test_mi_is_entropy_identity(s) for s in range(3)]
    checks += [lambda s=s: pins.test_gram_is_matmul(s) for s in range(2)]
    checks += [lambda s=s: pins.test_sparse_table_is_dense_nonzeros(s) for s in range(3)]
    failed = 0
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError):
            failed += 1
    return failed


def test_unmutated_oracle_passes_the_battery():
    assert battery() == 0


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found: " + name
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-o", str(so), str(mut),
                           "-lm"])
    saved = orc._load()
    orc._lib = orc._bind(ctypes.CDLL(str(so)))
    try:
        assert battery() > 0, "mutant survived: " + name
    finally:
        orc._lib = saved
