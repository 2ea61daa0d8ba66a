"""Planted mistakes in copies of the oracle must each fail at least one pin.

Every mutant is built from a textual edit of oracle/peval_oracle.c into a
temporary shared library; the committed oracle is never modified.
"""
import os
import tempfile

import pytest

import oracle
import oracle_pins as P

SRC = os.path.join(os.path.dirname(oracle.__file__), "peval_oracle.c")

MUTANTS = {
    "drop_first_tail_variable": (
        "for (uint32_t k = 2; k < n; ++k)                  /* * x_k^{g_ik} */",
        "for (uint32_t k = 3; k < n; ++k)                  /* * x_k^{g_ik} */"),
    "wrong_beta_index": (
        "v = mulmod(v, powmod(x[k - 2], r[k], p), p);",
        "v = mulmod(v, powmod(x[(k - 1) % (n - 2)], r[k], p), p);"),
    "t_starts_at_zero": (
        "bt[k] = powmod(beta[k] % p, t, p);",
        "bt[k] = powmod(beta[k] % p, t - 1, p);"),
    "transposed_group_key": (
        "return ((uint64_t)row[0] << 32) | (uint64_t)row[1];",
        "return ((uint64_t)row[1] << 32) | (uint64_t)row[0];"),
    "dropped_last_term": (
        "    for (uint64_t i = 0; i < s; ++i) {\n        const uint32_t *r = exps + i * n;\n        uint64_t v = coeffs[i] % p;                       /* a_i */",
        "    for (uint64_t i = 0; i + 1 < s; ++i) {\n        const uint32_t *r = exps + i * n;\n        uint64_t v = coeffs[i] % p;                       /* a_i */"),
    "ascending_order": (
        "return (a > b) ? -1 : (a < b) ? 1 : 0;",
        "return (a < b) ? -1 : (a > b) ? 1 : 0;"),
    "addmod_without_reduction": (
        "return (uint64_t)(((u128)a + (u128)b) % p);",
        "return a + b;"),
    "mulmod_64bit_product": (
        "return (uint64_t)(((u128)a * (u128)b) % p);",
        "return (a * b) % p;"),
    "exponent_off_by_one": (
        "v = mulmod(v, powmod(x[k - 2], r[k], p), p);",
        "v = mulmod(v, powmod(x[k - 2], r[k] + 1, p), p);"),
    "coefficient_dropped": (
        "uint64_t v = coeffs[i] % p;                       /* a_i */",
        "uint64_t v = 1;                       /* a_i */"),
    "points_wrong_variable": (
        "bt[k] = j->points[(t - j->t0) * m + k] % j->p;",
        "bt[k] = j->points[(t - j->t0) * m + (k + 1) % m] % j->p;"),
    "points_first_row_only": (
        "bt[k] = j->points[(t - j->t0) * m + k] % j->p;",
        "bt[k] = j->points[k] % j->p;"),
    "points_ignored": (
        "        if (j->points) {",
        "        if (0) {"),
    "interp_rows_from_t0": (
        "for (uint64_t j = 0; j < m; ++j) V[(t - 1) * m + j] = powmod(mono[members[j]], t, p);",
        "for (uint64_t j = 0; j < m; ++j) V[(t - 1) * m + j] = powmod(mono[members[j]], t - 1, p);"),
    "interp_wrong_column": (
        "c[t - 1] = images[(t - 1) * G + g] % p;",
        "c[t - 1] = images[(t - 1) * G + (g + 1) % G] % p;"),
    "interp_no_back_substitution": (
        "if (r == col || V[r * m + col] == 0) continue;",
        "if (r <= col || V[r * m + col] == 0) continue;"),
    "powmod_zero_exponent": (
        "uint64_t r = 1 % p;",
        "uint64_t r = base % p;"),
}


# cheaper settings of the pins for the mutant sweep; run in a child process
# because a mutant may also corrupt memory and abort (which counts as caught)
CHILD = r"""
import sys
sys.path[:0] = [{root!r}, {tests!r}]
import oracle, oracle_pins as P
orc = oracle.Oracle({lib!r})
pins = [lambda o: P.pin_full_point_bigint(o, cases=14),
        lambda o: P.pin_small_prime_exhaustive(o, primes=[3, 5]),
        P.pin_closed_forms, P.pin_linearity, P.pin_power_consistency,
        P.pin_group_order, P.pin_gcd_example,
        lambda o: P.pin_points_full_point_bigint(o, cases=10), P.pin_points_character_sums,
        P.pin_points_match_powers, P.pin_points_zero_and_linearity,
        P.pin_interp_round_trip, P.pin_interp_exhaustive, P.pin_interp_closed_forms]
caught = 0
for pin in pins:
    try:
        pin(orc)
    except Exception:
        caught += 1
sys.exit(3 if caught else 0)
"""


def _run_child(src_text, name):
    import subprocess
    import sys
    tests = os.path.dirname(os.path.abspath(__file__))
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, f"mut_{name}.c")
        with open(path, "w") as fh:
            fh.write(src_text)
        lib = os.path.join(tmp, f"libmut_{name}.so")
        oracle.build(lib, path)
        code = CHILD.format(root=os.path.dirname(tests), tests=tests, lib=lib)
        return subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=600)


def test_unmutated_copy_passes_in_child():
    """Control: the harness itself must report success for the real oracle."""
    res = _run_child(open(SRC).read(), "control")
    assert res.returncode == 0, res.stderr.decode()[-2000:]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation {name} does not match exactly once"
    res = _run_child(src.replace(old, new), name)
    assert res.returncode != 0, f"no pin catches mutant {name}"
