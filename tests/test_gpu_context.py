"""GPU vs oracle parity of contextual proposals (the context ablation of the
paper's supplement): candidates built on the device from the bank entry and
the slot's current spins, completed by MCMC sweeps, judged by Eq. 2."""
import numpy as np
import pytest

import oracle
from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce, compare

pytestmark = pytest.mark.gpu


def _pair(problem, betas, seed, banks, frac, sweeps, **kw):
    ctx = binding.Context(problem, betas, seed=seed, **kw)
    for r, b in banks.items():
        ctx.propose(r, b)
    ctx.set_context(frac, sweeps)
    ref = oracle.Run(problem, betas, seed=seed, banks=banks, ctx_fraction=frac, ctx_sweeps=sweeps, **kw)
    return ctx, ref


@pytest.mark.parametrize("G,frac,sweeps,rule", [(8, 0.25, 3, "metropolis"), (2, 0.5, 2, "gibbs"),
                                                (3, 0.0, 4, "metropolis"), (1, 0.125, 1, "metropolis")])
def test_lattice_contextual(G, frac, sweeps, rule):
    announce(f"contextual proposals, EA L=4 R=8, G={G} fraction={frac} sweeps={sweeps} rule={rule}")
    g = inputs.ea_lattice(4, 21)
    betas = inputs.geometric_ladder(8)
    banks = {r: inputs.random_bank(64, 5, seed=400 + r) for r in range(6)}
    ctx, ref = _pair(g, betas, 91, banks, frac, sweeps, rule=rule, prop_start=2, prop_period=2, target=-60)
    bt = binding.Batch([ctx], replicas_per_wg=G, chunk_sweeps=35)
    bt.sweep(90)
    ref.run(90)
    compare(ctx, ref)
    assert ref.prop_acc.sum() > 0


@pytest.mark.parametrize("G", [8, 2])
def test_multiplier_contextual(G):
    announce(f"contextual proposals, 6-bit multiplier R=8, G={G}")
    C = inputs.semiprimes(6, 1, seed=41)[0][0]
    g = inputs.multiplier(6, C)
    betas = inputs.geometric_ladder(8)
    banks = {r: inputs.random_bank(g["n"], 4, seed=500 + r, clamp=g["clamp"]) for r in range(5)}
    ctx, ref = _pair(g, betas, 17, banks, 0.25, 3, prop_start=1, prop_period=3)
    bt = binding.Batch([ctx], replicas_per_wg=G, chunk_sweeps=40)
    bt.sweep(120)
    ref.run(120)
    compare(ctx, ref)


def test_pm_eligible_lattice_takes_the_contextual_kernel():
    """An 8^3 +-J lattice would run in the +-J kernel; with contextual
    proposals it runs in the workgroup-synchronous one, several instances and
    a cross-workgroup split included."""
    announce("contextual proposals, 3 x EA +-J L=8 R=8, G=4")
    betas = inputs.geometric_ladder(8)
    ctxs, refs = [], []
    for k in range(3):
        g = inputs.ea_lattice(8, 60 + k)
        banks = {r: inputs.random_bank(512, 3, seed=600 + 10 * k + r) for r in range(6)}
        c, r = _pair(g, betas, 300 + k, banks, 0.25, 2, prop_start=2, prop_period=4)
        ctxs.append(c)
        refs.append(r)
    bt = binding.Batch(ctxs, replicas_per_wg=4, chunk_sweeps=30)
    bt.sweep(60)
    for c, r in zip(ctxs, refs):
        r.run(60)
        compare(c, r)


def test_full_context_equals_no_proposals():
    announce("contextual proposals with fraction 1: the chain without proposals")
    g = inputs.ea_lattice(4, 22)
    betas = inputs.geometric_ladder(6)
    banks = {r: inputs.random_bank(64, 3, seed=700 + r) for r in range(4)}
    ctx, _ = _pair(g, betas, 5, banks, 1.0, 2, prop_start=1, prop_period=1)
    plain = binding.Context(g, betas, seed=5)
    binding.Batch([ctx], chunk_sweeps=50).sweep(50)
    binding.Batch([plain], chunk_sweeps=50).sweep(50)
    s1, _ = ctx.state()
    s2, _ = plain.state()
    assert np.array_equal(s1, s2) and np.array_equal(ctx.energies(), plain.energies())
    c = ctx.counters()
    assert np.array_equal(c["prop_acc"], c["prop_att"]) and c["prop_att"][:4].tolist() == [50] * 4


def test_contextual_errors():
    announce("contextual proposals: argument and path errors")
    g = inputs.ea_lattice(4, 23)
    betas = inputs.geometric_ladder(4)
    ctx = binding.Context(g, betas, seed=1, prop_start=1, prop_period=1)
    for bad in ((-0.1, 1), (1.5, 1), (0.5, -1), (0.5, 65536)):
        with pytest.raises(binding.TaptError):
            ctx.set_context(*bad)
    bt = binding.Batch([ctx], chunk_sweeps=10)
    ctx.set_context(0.5, 2)
    with pytest.raises(binding.TaptError):
        ctx.sweep(1)                 # plain path: unsupported
    with pytest.raises(binding.TaptError):
        bt.sweep(10)                 # batch built before the mode changed
    bt.close()
    other = binding.Context(inputs.ea_lattice(6, 1), betas, seed=2)
    with pytest.raises(binding.TaptError):
        binding.Batch([ctx, other])  # contextual batches take one size
    binding.Batch([ctx], chunk_sweeps=10).sweep(10)
    ctx.set_context(0.0, 0)
    ctx.sweep(1)


def test_exact_count_context_on_a_large_lattice():
    """L = 10 (1000 free sites), fraction 0.125: every contextual proposal
    clamps exactly 125 sites, selected on the device by a radix select of the
    Philox keys, and the chain equals the oracle's."""
    announce("contextual proposals, EA L=10 R=4, G=2, fraction 0.125, 2 completion sweeps, 48 sweeps")
    g = inputs.ea_lattice(10, 23)
    betas = inputs.geometric_ladder(4)
    banks = {r: inputs.random_bank(1000, 3, seed=800 + r) for r in range(3)}
    ctx, ref = _pair(g, betas, 29, banks, 0.125, 2, prop_start=4, prop_period=4)
    bt = binding.Batch([ctx], replicas_per_wg=2, chunk_sweeps=24)
    bt.sweep(48)
    ref.run(48)
    compare(ctx, ref)
    assert ref.prop_att.sum() == 3 * 12
