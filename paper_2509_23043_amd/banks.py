"""Long-run MCMC proposal banks (Supp. Table S3 and the bank protocol after it).

The paper's MCMC proposal generator draws every bank sample from its own
randomly initialised Metropolis chain at the slot's beta, run for a burn-in
(10^4 sweeps for the 3D spin glass, 10^5 for factorization) after which one
configuration is kept. Here the chains are the slots of independent-chain
contexts (``M=0``: no swap or proposal stage, every slot at the same beta),
up to 1024 per context, batched into persistent launches. Every step runs in
the HIP kernels; this module only groups contexts and collects the states.
"""
from __future__ import annotations

import time

import numpy as np

from . import binding


def _batches(ctxs, make_batch):
    """Yield batches over consecutive groups of ctxs. Independent chains never
    wait for each other, so the runtime queues their workgroups and one batch
    normally takes them all; a refused batch (device memory) is halved."""
    i, k = 0, len(ctxs)
    while i < len(ctxs):
        k = min(k, len(ctxs) - i)
        try:
            bt = make_batch(ctxs[i:i + k])
        except binding.TaptError:
            if k == 1:
                raise
            k = max(1, k // 2)
            continue
        yield ctxs[i:i + k], bt
        i += k


def generate_bank(problem, beta, n_samples, burn_in, seed, chains_per_context=1024, replicas_per_wg=0,
                  replicas_per_thread=0, kernel="auto", chunk_sweeps=2000, timing=None):
    """n_samples configurations, each the state of its own independent chain
    at ``beta`` after ``burn_in`` sweeps from a random start.

    Returns (configs int8 [n_samples, n], energies int32 [n_samples]). With
    ``timing`` a dict, it receives the device time of the sweeps (``sweep_s``,
    from HIP events on the batch streams), the wall time (``wall_s``) and the
    number of single-spin update attempts (``attempts``)."""
    n = int(problem["n"])
    sizes = []
    left = int(n_samples)
    while left > 0:
        sizes.append(min(chains_per_context, left))
        left -= sizes[-1]
    ctxs = [binding.Context(problem, np.full(R, float(beta)), seed=seed + k, M=0) for k, R in enumerate(sizes)]
    configs, energies = [], []
    kern_ms = 0.0
    t0 = time.perf_counter()
    try:
        make = lambda group: binding.Batch(group, replicas_per_wg=replicas_per_wg,
                                           replicas_per_thread=replicas_per_thread, chunk_sweeps=chunk_sweeps,
                                           kernel=kernel)
        for group, bt in _batches(ctxs, make):
            bt.kernel_time()
            bt.sweep(int(burn_in))
            ms, _ = bt.kernel_time()
            kern_ms += ms
            bt.close()
            for c in group:
                s, _ = c.state()
                configs.append(s)
                energies.append(c.energies())
    finally:
        for c in ctxs:
            c.close()
    wall = time.perf_counter() - t0
    if timing is not None:
        nfree = ctxs[0].nfree
        timing.update(sweep_s=kern_ms * 1e-3, wall_s=wall, attempts=int(n_samples) * int(burn_in) * nfree)
    return np.concatenate(configs)[:n_samples], np.concatenate(energies)[:n_samples]
