"""Host-side parts of the battery (no GPU needed): the category laws and the
chi-square P-values of the library against the oracle."""

import numpy as np
import pytest

from oracle import battery as B


@pytest.fixture(scope="module")
def ph():
    import paper_1411_2484_amd as ph
    ph.lib()
    return ph


def test_test_names_agree(ph):
    assert tuple(ph.BATTERY_TESTS) == tuple(B.TESTS)


def test_category_laws_match_oracle(ph):
    oracle_laws = {
        "frequency": np.full(B.FREQ_BINS, 1.0 / B.FREQ_BINS),
        "serial2": np.full(1 << 20, 1.0 / (1 << 20)),
        "serial3": np.full(10 ** 6, 1.0 / 10 ** 6),
        "serial4": np.full(1 << 20, 1.0 / (1 << 20)),
        "serial5": np.full(1 << 20, 1.0 / (1 << 20)),
        "poker": B.poker_probabilities(),
        "collision": B.collision_probabilities(),
        "runs": B.runs_probabilities(),
        "fourier": B.fourier_probabilities(),
    }
    for i, name in enumerate(ph.BATTERY_TESTS):
        got = ph.battery_probabilities(i)
        want = oracle_laws[name]
        assert got.size == want.size, name
        assert np.allclose(got, want, rtol=1e-12, atol=0), (name, np.max(np.abs(got / want - 1)))


@pytest.mark.parametrize("dof", [1, 2, 4, 6, 20, 55, 65, 999999, (1 << 20) - 1])
def test_pvalues_match_oracle(ph, dof):
    sd = np.sqrt(2.0 * dof)
    for z in (-7.0, -5.0, -3.0, -1.0, -0.1, 0.0, 0.3, 1.0, 2.5, 4.0, 6.0, 9.0):
        chi2 = dof + z * sd
        if chi2 <= 0:
            continue
        want = B.p_value(chi2, dof)
        got = ph.chi2_pvalue(chi2, dof)
        assert got == pytest.approx(want, rel=1e-7, abs=1e-300), (dof, chi2, got, want)


def test_pvalue_rejects_bad_arguments(ph):
    with pytest.raises(ph.PhprngError):
        ph.chi2_pvalue(-1.0, 3)
    with pytest.raises(ph.PhprngError):
        ph.chi2_pvalue(1.0, 0)


@pytest.mark.parametrize("dof,chi2", [(20, 1.0263340389897238), (999999, 992927.9357236694), (999999, 1004300.0),
                                      ((1 << 20) - 1, 1052000.0), (65, 40.0), (6, 25.0)])
def test_pvalues_against_40_digit_values(ph, dof, chi2):
    """The library's P against the incomplete gamma function evaluated in
    40-digit arithmetic (mpmath), near tail only."""
    mpmath = pytest.importorskip("mpmath")
    with mpmath.workdps(40):
        a, x = mpmath.mpf(dof) / 2, mpmath.mpf(chi2) / 2
        t = mpmath.gammainc(a, 0, x, regularized=True) if x < a else \
            mpmath.gammainc(a, x, mpmath.inf, regularized=True)
        want = float(min(t, 1 - t))
    assert ph.chi2_pvalue(chi2, dof) == pytest.approx(want, rel=1e-11)
