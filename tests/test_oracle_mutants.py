"""Planted mistakes in the oracle, on the CPU only.

Each mutant below is the oracle's C source with one plausible slip (a
dropped term, a wrong sign, bit, index or modulus, two steps swapped),
compiled on its own and loaded as a separate copy of the oracle module.
The pins (``test_oracle_pins.py``, ``test_pattern_oracle.py``) that check
the affected step against something other than the oracle itself must
reject it: at least one of the listed pins fails on every mutant, and all
of them pass on the unmodified source built the same way.  Nothing here
touches the GPU library.
"""

import importlib.util
import inspect
import json
import os
import subprocess

import pytest

from tests import test_oracle_pins, test_pattern_oracle

PIN_MODULES = (test_oracle_pins, test_pattern_oracle)

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_DIR = os.path.join(ROOT, "oracle")
SRC = os.path.join(ORACLE_DIR, "phoracle.c")
INIT = os.path.join(ORACLE_DIR, "__init__.py")

# The draw loop of algorithm (9) as the oracle writes it, used to anchor
# mutations to that function (the forward jump repeats its first two lines).
GEN_LOOP = ("    ss = pho_mulmod(a, ss, p);\n"
            "    mm = (uint64_t)(((u128)mm + ss) % n);\n"
            "    uint64_t c = pho_powmod(mm, e, n);\n")

# name, text to replace (must occur exactly once), replacement, pins that
# see the affected step
MUTANTS = [
    ("powmod_tests_wrong_exponent_bit",
     "    if (e & 1) result = pho_mulmod(result, b, n);",
     "    if (e & 2) result = pho_mulmod(result, b, n);",
     ["test_encrypt_matches_python_pow", "test_decryption_recovers_message"]),
    ("draw_adds_skip_before_advancing_it",
     GEN_LOOP,
     "    mm = (uint64_t)(((u128)mm + ss) % n);\n"
     "    ss = pho_mulmod(a, ss, p);\n"
     "    uint64_t c = pho_powmod(mm, e, n);\n",
     ["test_step_relation_of_consecutive_ciphertexts"]),
    ("draw_reduces_skip_mod_n",
     GEN_LOOP,
     GEN_LOOP.replace("pho_mulmod(a, ss, p)", "pho_mulmod(a, ss, n)"),
     ["test_step_relation_of_consecutive_ciphertexts"]),
    ("draw_subtracts_skip",
     GEN_LOOP,
     GEN_LOOP.replace("((u128)mm + ss) % n", "((u128)mm + n - ss) % n"),
     ["test_step_relation_of_consecutive_ciphertexts"]),
    ("draw_encrypts_previous_message",
     GEN_LOOP,
     "    uint64_t prev = mm;\n" + GEN_LOOP.replace("pho_powmod(mm, e, n)", "pho_powmod(prev, e, n)"),
     ["test_step_relation_of_consecutive_ciphertexts"]),
    ("uniform_drops_the_plus_one_of_c",
     "    if (r_out) r_out[t] = (double)(c + 1) / denom;\n  }\n  *m = mm;\n  *s = ss;",
     "    if (r_out) r_out[t] = (double)c / denom;\n  }\n  *m = mm;\n  *s = ss;",
     ["test_uniform_is_correctly_rounded_quotient"]),
    ("uniform_divides_by_n",
     "  double denom = (double)(n + 1);\n  for (uint64_t t = 0; t < count; t++) {\n    ss = pho_mulmod",
     "  double denom = (double)n;\n  for (uint64_t t = 0; t < count; t++) {\n    ss = pho_mulmod",
     ["test_uniform_is_correctly_rounded_quotient"]),
    ("position_period_sum_wrong_sign",
     "((u128)p * (u128)(p - 1)) / 2;",
     "((u128)p * (u128)(p + 1)) / 2;",
     ["test_position_period_structure_32"]),
    ("position_period_taken_as_p",
     "  uint64_t q = k / (p - 1), r = k % (p - 1);",
     "  uint64_t q = k / p, r = k % p;",
     ["test_position_period_structure_32"]),
    ("position_skip_index_off_by_one",
     "  *s_out = pho_mulmod(s0, pho_powmod(a, r, p), p);",
     "  *s_out = pho_mulmod(s0, pho_powmod(a, r + 1, p), p);",
     ["test_position_general_s0_equals_stepping"]),
    ("position_sum_drops_last_term",
     "    for (uint64_t j = 1; j <= r; j++) {",
     "    for (uint64_t j = 1; j < r; j++) {",
     ["test_position_general_s0_equals_stepping"]),
    ("skip_table_prefix_one_term_too_many",
     "  for (uint64_t j = i * tab->stride; j < r; j++) {",
     "  for (uint64_t j = i * tab->stride; j <= r; j++) {",
     ["test_full_period_skip_sum", "test_position_equals_stepping_32"]),
    ("pattern_decrypts_with_e",
     "    uint64_t m = pho_powmod(c, d, n);",
     "    uint64_t m = pho_powmod(c, e, n);",
     ["test_enumeration_equals_full_period_windows"]),
    ("pattern_advances_skip_before_first_point",
     "        if (j > 1) {",
     "        if (j >= 1) {",
     ["test_enumeration_equals_full_period_windows"]),
    ("pattern_bins_over_n_plus_one",
     "((u128)cj * bins) / n)",
     "((u128)cj * bins) / (n + 1))",
     ["test_enumeration_equals_full_period_windows"]),
    ("decryption_inverts_e_mod_n",
     "uint64_t pho_decrypt(uint64_t c, uint64_t e, uint64_t n) {\n  uint64_t d = pho_inverse(e, n - 1);",
     "uint64_t pho_decrypt(uint64_t c, uint64_t e, uint64_t n) {\n  uint64_t d = pho_inverse(e, n);",
     ["test_decryption_recovers_message"]),
]


def _build(tmp_path, text, tag):
    c_path = tmp_path / ("phoracle_%s.c" % tag)
    so_path = tmp_path / ("libphoracle_%s.so" % tag)
    c_path.write_text(text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-pthread",
                    "-o", str(so_path), str(c_path)], check=True)
    spec = importlib.util.spec_from_file_location("oracle_variant_%s" % tag, INIT)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod._LIB_PATH = str(so_path)  # this copy loads the variant, never the shared build
    mod._lib = None
    mod.lib()
    return mod


def _cases(fn):
    """The argument sets of a pin's parametrize marks (their product)."""
    cases = [{}]
    for mark in getattr(fn, "pytestmark", []):
        if mark.name != "parametrize":
            continue
        keys = [k.strip() for k in mark.args[0].split(",")]
        rows = [dict(zip(keys, v if isinstance(v, (tuple, list)) else (v,))) for v in mark.args[1]]
        cases = [dict(c, **r) for c in cases for r in rows]
    return cases


def _run_pin(name, mod, paper):
    """Runs one pin (every parametrized case) against an oracle variant;
    returns None if it passes, else a short description of the first failure."""
    fn = next(getattr(m, name) for m in PIN_MODULES if hasattr(m, name))
    for case in _cases(fn):
        args = dict(case)
        for a in inspect.signature(fn).parameters:
            if a in args:
                continue
            if a == "orc":
                args[a] = mod
            elif a == "paper":
                args[a] = paper
            elif a == "tab32":
                p, g = mod.lcg_params(32)
                args[a] = mod.SkipTab(p, g, 1 << 16, p - 1)
            else:
                raise AssertionError("pin %s needs fixture %s" % (name, a))
        try:
            fn(**args)
        except Exception as exc:  # an assertion or an error both reject the variant
            return "%s %s" % (type(exc).__name__, case)
    return None


@pytest.fixture(scope="module")
def paper():
    with open(os.path.join(HERE, "golden", "paper_values.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmodified_source_passes_every_listed_pin(tmp_path, paper, source):
    mod = _build(tmp_path, source, "control")
    names = sorted({n for m in MUTANTS for n in m[3]})
    failed = {n: r for n in names if (r := _run_pin(n, mod, paper)) is not None}
    assert not failed, failed


@pytest.mark.parametrize("name,old,new,pin_names", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(tmp_path, paper, source, name, old, new, pin_names):
    assert source.count(old) == 1, "mutation site of %s not unique" % name
    mod = _build(tmp_path, source.replace(old, new), name)
    results = {n: _run_pin(n, mod, paper) for n in pin_names}
    assert any(r is not None for r in results.values()), "mutant %s passed %s" % (name, pin_names)
