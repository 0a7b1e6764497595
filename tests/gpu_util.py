"""Helpers for the GPU parity tests."""
import sys

import numpy as np

import oracle
from paper_2509_23043_amd import binding


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def compare(ctx, ref, check_best=True):
    """Bit-exact comparison of a context with an oracle run."""
    spins, t = ctx.state()
    assert t == ref.t, (t, ref.t)
    assert np.array_equal(ctx.energies(), ref.E), (ctx.energies(), ref.E)
    assert np.array_equal(spins, ref.spins)
    c = ctx.counters()
    R = ref.R
    if R > 1:
        assert np.array_equal(c["swap_att"], ref.swap_att[:R - 1])
        assert np.array_equal(c["swap_acc"], ref.swap_acc[:R - 1])
    assert np.array_equal(c["prop_att"], ref.prop_att)
    assert np.array_equal(c["prop_acc"], ref.prop_acc)
    assert np.array_equal(c["flips"], ref.flips)
    if check_best:
        s = ctx.summary()
        assert s["best"] == ref.best, (s["best"], ref.best)
        assert s["best_t"] == ref.best_t, (s["best_t"], ref.best_t)
        assert s["best_slot"] == ref.best_slot
        assert s["first_hit"] == ref.first_hit
        assert np.array_equal(s["best_spins"], ref.best_spins)


def make_pair(problem, betas, seed, banks=None, **kw):
    ctx = binding.Context(problem, betas, seed=seed, **kw)
    if banks:
        for r, b in banks.items():
            ctx.propose(r, b)
    ref = oracle.Run(problem, betas, seed=seed, banks=banks, **kw)
    return ctx, ref
