"""Planted mistakes in the battery oracle, on the CPU only.

Each mutant is ``oracle/battery.py`` with one plausible slip in a bin, a
category law, a test statistic or an ordering convention, loaded as a
separate module and put in place of the oracle for the pins of
``test_battery_oracle.py`` that check that step against enumeration, a
closed form or a hand-built sequence.  At least one listed pin rejects every
mutant; all of them pass on the unmodified source loaded the same way.
"""

import importlib.util
import os

import pytest

from tests import test_battery_oracle as pins

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "battery.py")

# name, text to replace (must occur exactly once), replacement, pins that
# see the affected step
MUTANTS = [
    ("bins_not_clamped",
     "    return np.minimum(np.floor(r * bins), bins - 1).astype(np.int64)",
     "    return np.floor(r * bins).astype(np.int64)",
     ["test_bins_and_clamp"]),
    ("serial_last_element_most_significant",
     "        cell = cell * b + bin_of(tup[:, i], b)",
     "        cell = cell * b + bin_of(tup[:, d - 1 - i], b)",
     ["test_serial_cell_index_convention"]),
    ("serial_tuples_cross_blocks",
     "    tup = blocks[:, : t * d].reshape(-1, d)",
     "    tup = blocks.ravel()[: blocks.size // d * d].reshape(-1, d)",
     ["test_serial_block_tail_is_unused"]),
    ("poker_two_pairs_counted_twice",
     "            c(5, 2) * c(3, 2) // 2 * 10 * 9 * 8,",
     "            c(5, 2) * c(3, 2) * 10 * 9 * 8,",
     ["test_poker_law_by_enumerating_all_hands"]),
    ("poker_full_house_as_three_of_a_kind",
     "    cat[(distinct == 2) & (top == 3)] = 4       # full house",
     "    cat[(distinct == 2) & (top == 3)] = 3       # full house",
     ["test_poker_classifier_examples", "test_poker_law_by_enumerating_all_hands"]),
    ("collisions_off_by_one",
     "        out[i] = COLL_BALLS - np.unique(bin_of(t, COLL_URNS)).size",
     "        out[i] = COLL_BALLS - 1 - np.unique(bin_of(t, COLL_URNS)).size",
     ["test_collisions_per_trial_small_cases"]),
    ("collision_law_counts_the_new_ball",
     "        hit = np.where(occupied > 0, occupied / urns, 0.0)",
     "        hit = np.where(occupied > 0, (occupied + 1) / urns, 0.0)",
     ["test_collision_law_brute_force", "test_collision_law_moments_closed_form"]),
    ("runs_include_the_block_ends",
     "    return np.diff(change)",
     "    return np.diff(np.concatenate([[0], change, [bits.size]]))",
     ["test_runs_interior_only", "test_runs_exact_counts_by_enumeration"]),
    ("runs_law_wrong_power",
     "    w = np.array([max(m - 1 - L, 0) * 2.0 ** -(L + 1) for L in range(1, RUNS_MAX + 1)])",
     "    w = np.array([max(m - 1 - L, 0) * 2.0 ** -L for L in range(1, RUNS_MAX + 1)])",
     ["test_runs_exact_counts_by_enumeration"]),
    ("fourier_negative_exponent",
     "    return np.fft.ifft(x) * (m / math.sqrt(m))",
     "    return np.fft.fft(x) / math.sqrt(m)",
     ["test_fourier_matches_paper_sum"]),
    ("fourier_variance_one_over_12",
     "FOURIER_SCALE = 8.0 * math.sqrt(24.0)",
     "FOURIER_SCALE = 8.0 * math.sqrt(12.0)",
     ["test_fourier_categories_and_law", "test_uniform_variance_is_one_over_24"]),
    ("p_value_upper_tail_only",
     "    return min(q, p)",
     "    return q",
     ["test_p_value_closed_forms"]),
    ("interleave_keeps_stream_order",
     "    return np.ascontiguousarray(np.asarray(streams).T).ravel()",
     "    return np.ascontiguousarray(np.asarray(streams)).ravel()",
     ["test_interleave_order"]),
]


def _load(tmp_path, text, tag):
    path = tmp_path / ("battery_%s.py" % tag)
    path.write_text(text)
    spec = importlib.util.spec_from_file_location("battery_variant_%s" % tag, str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _failures(monkeypatch, mod, names):
    """{pin: failure} for the pins that reject the variant."""
    out = {}
    with monkeypatch.context() as mp:
        mp.setattr(pins, "B", mod)
        for name in names:
            fn = getattr(pins, name)
            marks = getattr(fn, "pytestmark", [])
            param = [m for m in marks if m.name == "parametrize"]
            cases = [dict(zip([a.strip() for a in p.args[0].split(",")], v if isinstance(v, tuple) else (v,)))
                     for p in param for v in p.args[1]] or [{}]
            for kw in cases:
                try:
                    fn(**kw)
                except Exception as exc:  # an assertion or an error both reject the variant
                    out[name] = "%s %s" % (type(exc).__name__, kw)
                    break
    return out


@pytest.fixture(scope="module")
def source():
    with open(SRC) as f:
        return f.read()


def test_unmodified_source_passes_every_listed_pin(tmp_path, monkeypatch, source):
    mod = _load(tmp_path, source, "control")
    names = sorted({n for m in MUTANTS for n in m[3]})
    assert _failures(monkeypatch, mod, names) == {}


@pytest.mark.parametrize("name,old,new,pin_names", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_planted_mistake(tmp_path, monkeypatch, source, name, old, new, pin_names):
    assert source.count(old) == 1, "mutation site of %s not unique" % name
    mod = _load(tmp_path, source.replace(old, new), name)
    assert _failures(monkeypatch, mod, pin_names), "mutant %s passed %s" % (name, pin_names)
