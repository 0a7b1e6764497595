"""Adaptive temperature ladder: inverse temperatures that give roughly uniform
swap acceptance between neighbouring slots (Methods, "Parallel tempering";
the ladder is then fixed for every PT and TAPT run of a problem family).

Each round measures the swap acceptance A_r of every pair (r, r+1) and moves
the interior betas, ends fixed. For two slots a short distance apart,
-log A_r grows like the square of the gap times a local weight w_r (the
energy fluctuations between them), so w_r is estimated as
-log A_r / (beta_{r+1} - beta_r)^2 and the new gaps are made proportional to
w_r^(-1/2), which equalises the predicted -log A_r. A damping factor mixes
the new gaps with the old ones. The sampling runs in the library's kernels;
this module only does the bookkeeping between rounds.
"""
from __future__ import annotations

import numpy as np

A_FLOOR = 1e-4      # acceptance floor: a pair that never swapped still gets a finite weight


def rebalance(betas, acceptance, damping=0.5):
    """One update of the interior betas from the pair acceptances (ends and
    order preserved). ``acceptance``: [R-1] fractions in [0, 1]."""
    b = np.asarray(betas, np.float64)
    A = np.clip(np.asarray(acceptance, np.float64), A_FLOOR, 1.0 - 1e-12)
    gap = np.diff(b)
    w = -np.log(A) / gap ** 2
    target = w ** -0.5
    target *= (b[-1] - b[0]) / target.sum()
    new_gap = (1.0 - damping) * target + damping * gap
    new_gap *= (b[-1] - b[0]) / new_gap.sum()
    out = np.concatenate([[b[0]], b[0] + np.cumsum(new_gap)])
    out[-1] = b[-1]
    return out


def measure_acceptance(problem, betas, sweeps, runs=4, seed=0, M=1):
    """Swap acceptance of every pair over ``runs`` independent PT runs of
    ``sweeps`` sweeps (one batched launch sequence)."""
    from . import binding
    ctxs = [binding.Context(problem, betas, seed=seed + k, M=M) for k in range(runs)]
    try:
        bt = binding.Batch(ctxs, chunk_sweeps=min(int(sweeps), 2000))
        bt.sweep(int(sweeps))
        bt.close()
        att = np.zeros(len(betas) - 1)
        acc = np.zeros(len(betas) - 1)
        for c in ctxs:
            k = c.counters()
            att += k["swap_att"]
            acc += k["swap_acc"]
    finally:
        for c in ctxs:
            c.close()
    return acc / np.maximum(att, 1)


def adapt(problem, betas, rounds=8, sweeps=2000, runs=4, seed=0, damping=0.5, measure=None):
    """Iterate measure -> rebalance. Returns (betas, history) with history a
    list of (betas, acceptance) per round, the last one measured on the
    returned ladder. ``measure(betas, seed)`` replaces the library sampler
    (the tests pass the CPU reference)."""
    if measure is None:
        measure = lambda b, s: measure_acceptance(problem, b, sweeps, runs, s)
    b = np.asarray(betas, np.float64)
    hist = []
    for k in range(rounds):
        A = measure(b, seed + 1000 * k)
        hist.append((b.copy(), A))
        b = rebalance(b, A, damping)
    hist.append((b.copy(), measure(b, seed + 1000 * rounds)))
    return b, hist
