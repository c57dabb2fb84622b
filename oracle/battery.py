"""CPU oracle of the small statistical battery applied to the generator's
uniforms (the chi-square tests listed in the paper's Tests section).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Plain numpy in binary64, written
from the definitions; library routines serve as single steps (``bincount``,
an FFT, the normal distribution and incomplete gamma functions of scipy).

Readings of the paper that fix what is computed (the paper names the tests
and their bin counts but not every convention):

* The tested sequence is consumed in blocks of M = 2^20 uniforms (the Fourier
  length of the Tests section).  Every test works inside a block; a block's
  results do not depend on its neighbours.
* A uniform R is put in bin ``min(floor(R * B), B - 1)`` of B equal bins; the
  clamp only acts on R = 1.0, which 64-bit moduli can produce.
* Serial tests use non-overlapping D-tuples inside a block, the first element
  being the most significant digit of the cell index; the last ``M mod D``
  uniforms of a block are unused.  Cells per axis: 1024 (D=2, 2^20 cells),
  100 (D=3, 10^6 cells), 32 (D=4), 16 (D=5).
* Poker: non-overlapping hands of five digits ``min(floor(10 R), 9)`` inside a
  block, classified as all different, one pair, two pairs, three of a kind,
  full house, four of a kind, five of a kind.
* Collision: 64 trials per block, each throws 2^14 consecutive uniforms into
  2^20 urns; collisions = 2^14 - occupied urns; categories "<= 100", 101 .. 154
  one each, ">= 155".
* Runs: bits ``R > 0.5``; only maximal runs bounded on both sides inside the
  block are counted; lengths 1 .. 20 one category each, ">= 21" merged; the
  expected counts are the observed total times the exact length law.
* Fourier: x_j = R_j - 1/2, coefficients with the paper's positive exponent and
  1/sqrt(M) normalisation for k = 0 .. M/2 - 1; real and imaginary parts go to
  64 bins of width sigma/8 over [-4 sigma, 4 sigma) plus two tails, with
  sigma^2 = 1/24; the bin of a value v is ``floor(v * RN(8 sqrt(24)))``.
* chi^2 = sum (O - E)^2 / E; degrees of freedom = categories - 1; the
  P-value is one-sided about the median: min(Q, 1 - Q) with Q the upper tail.
  A test without samples reports chi^2 = 0 and P = 0.
"""

from __future__ import annotations

import math

import numpy as np
from scipy import special

M = 1 << 20                       # block length and Fourier length
FREQ_BINS = 1 << 20
SERIAL_AXIS = {2: 1024, 3: 100, 4: 32, 5: 16}
POKER_CATS = 7
COLL_BALLS = 1 << 14
COLL_URNS = 1 << 20
COLL_LO, COLL_HI = 100, 155       # categories: <= LO, LO+1 .. HI-1, >= HI
COLL_CATS = COLL_HI - COLL_LO + 1
RUNS_MAX = 20                     # lengths 1..20, then >= 21
RUNS_CATS = RUNS_MAX + 1
FOURIER_HALF = 32                 # bins per side of zero, width sigma / 8
FOURIER_CATS = 2 * FOURIER_HALF + 2
FOURIER_SCALE = 8.0 * math.sqrt(24.0)

TESTS = ("frequency", "serial2", "serial3", "serial4", "serial5", "poker", "collision", "runs", "fourier")


def _blocks(r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    assert r.size % M == 0, "the battery consumes whole blocks of 2^20 uniforms"
    return r.reshape(-1, M)


def bin_of(r, bins):
    """Equal-bin index of uniforms, clamped to the last bin."""
    return np.minimum(np.floor(r * bins), bins - 1).astype(np.int64)


# --- histograms ---------------------------------------------------------------

def frequency_counts(r):
    """One-dimensional frequency test: 2^20 equal bins."""
    return np.bincount(bin_of(_blocks(r).ravel(), FREQ_BINS), minlength=FREQ_BINS)


def serial_counts(r, d):
    """D-dimensional serial test: non-overlapping D-tuples inside each block."""
    b = SERIAL_AXIS[d]
    blocks = _blocks(r)
    t = M // d
    tup = blocks[:, : t * d].reshape(-1, d)
    cell = np.zeros(tup.shape[0], dtype=np.int64)
    for i in range(d):
        cell = cell * b + bin_of(tup[:, i], b)
    return np.bincount(cell, minlength=b ** d)


def poker_category(digits):
    """Category of each hand (rows of five digits 0..9)."""
    counts = np.zeros((digits.shape[0], 10), dtype=np.int64)
    for v in range(10):
        counts[:, v] = (digits == v).sum(axis=1)
    distinct = (counts > 0).sum(axis=1)
    top = counts.max(axis=1)
    cat = np.full(digits.shape[0], -1, dtype=np.int64)
    cat[distinct == 5] = 0                      # all different
    cat[distinct == 4] = 1                      # one pair
    cat[(distinct == 3) & (top == 2)] = 2       # two pairs
    cat[(distinct == 3) & (top == 3)] = 3       # three of a kind
    cat[(distinct == 2) & (top == 3)] = 4       # full house
    cat[(distinct == 2) & (top == 4)] = 5       # four of a kind
    cat[distinct == 1] = 6                      # five of a kind
    assert (cat >= 0).all()
    return cat


def poker_counts(r):
    blocks = _blocks(r)
    h = M // 5
    digits = bin_of(blocks[:, : 5 * h].reshape(-1, 5), 10)
    return np.bincount(poker_category(digits), minlength=POKER_CATS)


def collision_category(c):
    return np.clip(c, COLL_LO, COLL_HI) - COLL_LO


def collisions_per_trial(r):
    """Collisions of every trial: 2^14 balls into 2^20 urns."""
    trials = _blocks(r).reshape(-1, COLL_BALLS)
    out = np.empty(trials.shape[0], dtype=np.int64)
    for i, t in enumerate(trials):
        out[i] = COLL_BALLS - np.unique(bin_of(t, COLL_URNS)).size
    return out


def collision_counts(r):
    return np.bincount(collision_category(collisions_per_trial(r)), minlength=COLL_CATS)


def interior_run_lengths(bits):
    """Lengths of the maximal runs of equal bits that have a differing bit on
    both sides (so neither the first nor the last run of the block)."""
    change = np.flatnonzero(bits[1:] != bits[:-1]) + 1   # starts of runs 2, 3, ...
    return np.diff(change)


def runs_counts(r):
    out = np.zeros(RUNS_CATS, dtype=np.int64)
    for blk in _blocks(r):
        lengths = interior_run_lengths(blk > 0.5)
        out += np.bincount(np.minimum(lengths, RUNS_CATS) - 1, minlength=RUNS_CATS)
    return out


def fourier_coefficients(x):
    """x_hat_k = M^(-1/2) sum_j x_j exp(+2 pi i j k / M), k = 0 .. M-1 (Tests
    section, Fourier test); numpy's inverse FFT carries the positive sign and
    a 1/M factor."""
    m = x.size
    return np.fft.ifft(x) * (m / math.sqrt(m))


def fourier_category(v):
    u = np.floor(v * FOURIER_SCALE)
    return (np.clip(u, -FOURIER_HALF - 1, FOURIER_HALF) + FOURIER_HALF + 1).astype(np.int64)


def fourier_values(r):
    """Real and imaginary parts of the first M/2 coefficients of every block."""
    out = []
    for blk in _blocks(r):
        xh = fourier_coefficients(blk - 0.5)[: M // 2]
        out.append(np.stack([xh.real, xh.imag], axis=1).ravel())
    return np.concatenate(out) if out else np.zeros(0)


def fourier_counts(r):
    return np.bincount(fourier_category(fourier_values(r)), minlength=FOURIER_CATS)


# --- exact category laws --------------------------------------------------------

def poker_probabilities():
    """Exact law of the seven hands with five cards and ten values."""
    c = math.comb
    ways = [10 * 9 * 8 * 7 * 6,
            c(5, 2) * 10 * 9 * 8 * 7,
            c(5, 2) * c(3, 2) // 2 * 10 * 9 * 8,
            c(5, 3) * 10 * 9 * 8,
            c(5, 3) * 10 * 9,
            c(5, 4) * 10 * 9,
            10]
    return np.array(ways, dtype=np.float64) / 10.0 ** 5


def collision_law(balls, urns, cmax):
    """Probability of c collisions, c = 0 .. cmax, when `balls` balls fall
    uniformly into `urns` urns: after i balls with c collisions the next ball
    lands in one of the i - c occupied urns with probability (i - c) / urns."""
    q = np.zeros(cmax + 2)
    q[0] = 1.0
    c = np.arange(cmax + 2, dtype=np.float64)
    for i in range(balls):
        occupied = i - c
        hit = np.where(occupied > 0, occupied / urns, 0.0)
        nq = q * (1.0 - hit)
        nq[1:] += q[:-1] * hit[:-1]
        q = nq
    return q[: cmax + 1]


def collision_probabilities():
    law = collision_law(COLL_BALLS, COLL_URNS, 600)
    p = np.empty(COLL_CATS)
    p[0] = law[: COLL_LO + 1].sum()
    p[1:-1] = law[COLL_LO + 1: COLL_HI]
    p[-1] = 1.0 - law[: COLL_HI].sum()
    return p


def runs_weights(m=M):
    """Expected interior runs of length L per block of m fair bits, for
    L = 1 .. 20 and the merged tail: (m - 1 - L) 2^-(L+1) each."""
    w = np.array([max(m - 1 - L, 0) * 2.0 ** -(L + 1) for L in range(1, RUNS_MAX + 1)])
    tail_l = np.arange(RUNS_MAX + 1, max(m - 1, RUNS_MAX + 1), dtype=np.float64)
    tail = float(np.sum((m - 1 - tail_l) * 2.0 ** -(tail_l + 1)))
    return np.append(w, tail)


def runs_probabilities():
    w = runs_weights()
    return w / w.sum()


def fourier_probabilities():
    """Standard normal mass of the 66 categories (bin u covers [u/8, (u+1)/8)
    standard deviations)."""
    u = np.arange(-FOURIER_HALF, FOURIER_HALF, dtype=np.float64)
    # lower-tail differences on the negative side, upper-tail ones on the positive
    # side, so that no mass is a difference of two numbers close to 1
    neg = special.ndtr((u + 1) / 8.0) - special.ndtr(u / 8.0)
    pos = special.ndtr(-u / 8.0) - special.ndtr(-(u + 1) / 8.0)
    mass = np.where(u < 0, neg, pos)
    tail = special.ndtr(-FOURIER_HALF / 8.0)
    return np.concatenate([[tail], mass, [tail]])


# --- chi-square ------------------------------------------------------------------

def chi_square(observed, expected):
    observed = np.asarray(observed, dtype=np.float64)
    return float(np.sum((observed - expected) ** 2 / expected))


def p_value(chi2, dof):
    """One-sided probability about the median: min(Q, 1 - Q), Q = P(X >= chi2).
    Both tails come straight from scipy's regularised incomplete gamma
    functions (no complement is formed, so neither tail loses digits to
    cancellation); their relative accuracy is about 1e-8 at 10^6 degrees of
    freedom and better below."""
    q = float(special.gammaincc(dof / 2.0, chi2 / 2.0))
    p = float(special.gammainc(dof / 2.0, chi2 / 2.0))
    return min(q, p)


def run_battery(r):
    """All nine tests on a sequence of whole blocks: {name: (counts, expected,
    chi2, dof, p)}."""
    res = {}

    def add(name, counts, probs):
        counts = np.asarray(counts, dtype=np.int64)
        expected = counts.sum() * np.asarray(probs, dtype=np.float64)
        dof = counts.size - 1
        if counts.sum() == 0:       # nothing to test (e.g. no interior run): chi2 = 0, P = 0
            res[name] = (counts, expected, 0.0, dof, 0.0)
            return
        chi2 = chi_square(counts, expected)
        res[name] = (counts, expected, chi2, dof, p_value(chi2, dof))

    add("frequency", frequency_counts(r), np.full(FREQ_BINS, 1.0 / FREQ_BINS))
    for d in (2, 3, 4, 5):
        n = SERIAL_AXIS[d] ** d
        add("serial%d" % d, serial_counts(r, d), np.full(n, 1.0 / n))
    add("poker", poker_counts(r), poker_probabilities())
    add("collision", collision_counts(r), collision_probabilities())
    add("runs", runs_counts(r), runs_probabilities())
    add("fourier", fourier_counts(r), fourier_probabilities())
    return res


def interleave(streams):
    """Interstream order of the Tests section: R_1 of every stream, then R_2 of
    every stream, ...  `streams` is (number of streams, length)."""
    return np.ascontiguousarray(np.asarray(streams).T).ravel()
