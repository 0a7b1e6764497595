"""Pins of the TTS statistics (Supp. TTS methodology) against closed forms."""
import math

import numpy as np

from paper_2509_23043_amd import tts


def test_repetitions_closed_form():
    # ceil(log(0.01) / log(0.5)) = ceil(6.64) = 7
    assert tts.repetitions(0.5) == 7
    assert tts.repetitions(0.99) == 1
    assert tts.repetitions(1.0) == 1
    assert tts.repetitions(0.0) == math.inf
    # 1 - (1 - s)^R >= 0.99 holds at R and fails at R - 1
    for s in (0.01, 0.1, 0.37, 0.8):
        R = tts.repetitions(s)
        assert 1 - (1 - s) ** R >= 0.99 > 1 - (1 - s) ** (R - 1)


def test_success_probability_counts_hits_up_to_t():
    hits = np.array([-1, 0, 5, 10, 10, 11, -1, 3])
    assert tts.success_probability(hits, 10) == 5 / 8
    assert tts.success_probability(hits, 0) == 1 / 8
    assert tts.success_probability(hits, 1000) == 6 / 8


def test_tts_star_minimises_over_run_length():
    # first hits spread so that s(t) = t / 100 for t = 1..100 (100 runs)
    hits = np.arange(1, 101)
    grid = [1, 10, 25, 50, 69, 100]
    best, arg = tts.tts_star(hits, grid)
    want = min(t * tts.repetitions(t / 100) for t in grid)
    assert best == want and arg in grid and tts.tts_mcs(arg, arg / 100) == want
    assert tts.tts_star(np.full(10, -1), grid) == (math.inf, None)


def test_fit_exponential_recovers_parameters():
    n = np.array([16, 18, 20, 22, 24])
    A, k = tts.fit_exponential(n, 3.5 * np.exp(0.846 * n))
    assert abs(k - 0.846) < 1e-9 and abs(A - 3.5) < 1e-6


def test_bootstrap_interval_covers_the_median():
    rng = np.random.Generator(np.random.PCG64(3))
    cover = 0
    for rep in range(60):
        x = rng.exponential(1.0, size=200)          # true median ln 2
        lo, hi = tts.bootstrap_median_ci(x, n_boot=400, seed=rep)
        cover += lo <= math.log(2) <= hi
    assert cover >= 51                               # nominal 95%: 57 of 60


def test_bootstrap_interval_with_unsolved_instances():
    """Instances that never succeed have infinite TTS; the interval's ends are
    order statistics (infinite, not NaN) when enough of them are."""
    x = np.array([1.0, 2.0, 3.0, np.inf, np.inf, np.inf, np.inf])
    lo, hi = tts.bootstrap_median_ci(x, n_boot=500, seed=1)
    assert not np.isnan(lo) and hi == np.inf
