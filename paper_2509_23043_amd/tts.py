"""Time-to-solution (TTS) harness for factorization (Supp. TTS methodology).

The measurement the paper uses to compare PT and TAPT on integer
factorization:

* a run of length t_a sweeps succeeds when its lowest ladder energy reaches
  the ground energy of the clamped multiplier (every ground state is a valid
  factorization, A x B = C), so the empirical success probability s(t_a) is
  the fraction of independent runs whose first hit is at most t_a;
* R(P_target) = ceil(log(1 - P_target) / log(1 - s)) independent runs reach
  P_target = 0.99 (Supp. Eqs. for P_fail and R);
* TTS_MCS(t_a) = t_a R(0.99), minimised over the run length t_a;
* TTS in seconds = TTS_MCS* x the measured time per trajectory per sweep;
* the median over instances at each product bit length n, with bootstrap
  confidence intervals, is fitted to TTS(n) = A exp(k n) by least squares on
  log TTS.

The runs themselves are batched contexts of the library (every step in the
HIP kernels); this module only schedules them and does the statistics.
"""
from __future__ import annotations

import math

import numpy as np

P_TARGET = 0.99


def success_probability(first_hits, t_a):
    """Fraction of runs whose first hit (sweep, -1 = never) is <= t_a."""
    h = np.asarray(first_hits)
    return float(np.mean((h >= 0) & (h <= t_a))) if h.size else 0.0


def repetitions(s, p_target=P_TARGET):
    """Independent runs needed to reach p_target: ceil(log(1-p)/log(1-s));
    1 when s = 1 and infinite when s = 0."""
    if s >= 1.0:
        return 1
    if s <= 0.0:
        return math.inf
    return math.ceil(math.log(1.0 - p_target) / math.log(1.0 - s))


def tts_mcs(t_a, s, p_target=P_TARGET):
    """TTS in sweeps for run length t_a with success probability s."""
    r = repetitions(s, p_target)
    return math.inf if r == math.inf else t_a * r


def tts_star(first_hits, t_grid, p_target=P_TARGET):
    """min over t_a in t_grid of TTS_MCS(t_a): returns (tts, t_a*); (inf, None)
    when no run succeeds within the grid."""
    best, arg = math.inf, None
    for t in t_grid:
        v = tts_mcs(t, success_probability(first_hits, t), p_target)
        if v < best:
            best, arg = v, t
    return best, arg


def fit_exponential(n, tts):
    """Least-squares fit of log TTS = log A + k n; returns (A, k)."""
    n = np.asarray(n, np.float64)
    y = np.log(np.asarray(tts, np.float64))
    k, logA = np.polyfit(n, y, 1)
    return float(math.exp(logA)), float(k)


def bootstrap_median_ci(values, n_boot=2000, alpha=0.05, seed=0):
    """Percentile bootstrap interval of the median (infinite values allowed)."""
    v = np.asarray(values, np.float64)
    rng = np.random.Generator(np.random.PCG64(seed))
    meds = np.median(v[rng.integers(0, len(v), size=(n_boot, len(v)))], axis=1)
    # order statistics without interpolation, so that infinite medians stay infinite
    return (float(np.quantile(meds, alpha / 2, method="lower")),
            float(np.quantile(meds, 1 - alpha / 2, method="higher")))


def run_instance(problem, betas, runs, t_max, seed, target, banks=None, prop_period=1, chunk_sweeps=2000,
                 replicas_per_wg=0):
    """``runs`` independent PT runs (TAPT when ``banks`` maps slots to
    proposal banks, proposals every ``prop_period`` sweeps from the first),
    each t_max sweeps, batched in persistent launches.

    Returns (first_hits int64 [runs], seconds per trajectory per sweep from
    the chunk kernels' HIP events)."""
    from . import binding
    kw = dict(M=1, target=int(target))
    if banks:
        kw.update(prop_start=prop_period, prop_period=prop_period)
    ctxs = []
    try:
        for k in range(runs):
            c = binding.Context(problem, betas, seed=int(seed) + k, **kw)
            for r, b in (banks or {}).items():
                c.propose(r, b)
            ctxs.append(c)
        hits = []
        kern_ms = 0.0
        i = 0
        step = len(ctxs)
        while i < len(ctxs):
            group = ctxs[i:i + step]
            try:
                bt = binding.Batch(group, replicas_per_wg=replicas_per_wg, chunk_sweeps=chunk_sweeps)
            except binding.TaptError:
                if step == 1:
                    raise
                step = max(1, step // 2)   # more workgroups than can be resident: split
                continue
            bt.kernel_time()
            bt.sweep(int(t_max))
            ms, _ = bt.kernel_time()
            kern_ms += ms
            bt.close()
            hits += [c.summary()["first_hit"] for c in group]
            i += len(group)
    finally:
        for c in ctxs:
            c.close()
    return np.asarray(hits, np.int64), kern_ms * 1e-3 / (runs * t_max)
