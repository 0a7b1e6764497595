"""Adaptive ladder: the update rule against closed forms, and the whole loop
with the CPU reference as the sampler."""
import numpy as np

import oracle
from paper_2509_23043_amd import inputs, ladder


def test_uniform_acceptance_is_a_fixed_point():
    b = inputs.geometric_ladder(10)
    gap = np.diff(b)
    A = np.exp(-0.7 * np.ones(9))            # uniform -log A
    # weights -log A / gap^2 give target gaps proportional to the current ones
    out = ladder.rebalance(b, A, damping=0.0)
    assert np.allclose(out, b) and out[0] == b[0] and out[-1] == b[-1]


def test_rebalance_keeps_ends_and_order():
    b = inputs.geometric_ladder(12)
    rng = np.random.Generator(np.random.PCG64(1))
    out = ladder.rebalance(b, rng.uniform(0.0, 1.0, 11))
    assert out[0] == b[0] and out[-1] == b[-1] and np.all(np.diff(out) > 0)


def test_equalises_a_model_with_known_weights():
    """A model system with -log A_r = kappa(beta) gap^2 and kappa = 0.5 /
    beta^2 (a constant heat capacity: energy variance C / beta^2): the
    iteration drives -log A_r to equal values, and the equal-cost ladder has
    gaps proportional to beta, i.e. it is geometric."""
    b = np.linspace(0.2, 3.0, 16)
    model = lambda bb: np.exp(-0.5 / ((bb[1:] + bb[:-1]) / 2) ** 2 * np.diff(bb) ** 2)
    for _ in range(40):
        b = ladder.rebalance(b, model(b), damping=0.5)
    cost = -np.log(model(b))
    assert cost.std() / cost.mean() < 0.02
    ratio = b[1:] / b[:-1]
    assert ratio.std() / ratio.mean() < 0.02


def test_adapt_with_reference_sampler_evens_out_acceptance():
    """The loop on a 4^3 spin glass with the CPU reference as the sampler:
    the spread of the pair acceptances falls well below that of a linear
    ladder."""
    g = inputs.ea_lattice(4, 5)

    def measure(b, seed):
        run = oracle.Run(g, b, seed=seed, M=1)
        run.run(1500)
        return run.swap_acc[:len(b) - 1] / np.maximum(run.swap_att[:len(b) - 1], 1)

    b0 = np.linspace(0.2, 3.0, 10)
    b, hist = ladder.adapt(g, b0, rounds=6, seed=3, measure=measure)
    A0, A1 = hist[0][1], hist[-1][1]
    assert np.all(np.diff(b) > 0) and b[0] == b0[0] and b[-1] == b0[-1]
    assert A1.std() < 0.6 * A0.std(), (A0, A1)
