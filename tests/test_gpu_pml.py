"""GPU vs oracle parity of the +-J row kernel (kernel "pml"): one beta slot per
wavefront, rows of L sites, lattices of every even L from 6 to 16 in one
launch. Bit-exact spins, energies, counters and best record against the
oracle for the same seeds; the launch plan is checked so that each case runs
the kernel it names."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce, compare

pytestmark = pytest.mark.gpu


def _run(cases, G, sweeps, chunk=40, M=1, rule="metropolis", bank_every=2, bank_size=4, target=None):
    """cases: [(L, R, seed)]; every context with proposals on every
    bank_every-th slot (none when M = 0), compared with its own oracle run."""
    import oracle
    ctxs, refs = [], []
    for L, R, seed in cases:
        g = inputs.ea_lattice(L, 7000 + 13 * L + seed)
        betas = inputs.geometric_ladder(R) if M else np.full(R, 0.9)
        banks = ({r: inputs.random_bank(g["n"], bank_size, seed=7100 + 31 * seed + r) for r in range(0, R, bank_every)}
                 if M else None)
        kw = dict(M=M, rule=rule)
        if M:
            kw.update(prop_start=2 * M, prop_period=3 * M)
        if target is not None:
            kw["target"] = target
        c = binding.Context(g, betas, seed=7200 + seed, **kw)
        for r, b in (banks or {}).items():
            c.propose(r, b)
        ctxs.append(c)
        refs.append(oracle.Run(g, betas, seed=7200 + seed, banks=banks, **kw))
    bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=chunk, kernel="pml")
    plan = bt.describe()
    assert [d["kernel"] for d in plan] == ["pml"], plan
    bt.sweep(sweeps)
    bt.close()
    for c, ref in zip(ctxs, refs):
        ref.run(sweeps)
        compare(c, ref)
        c.close()
    return plan


@pytest.mark.parametrize("L", [6, 8, 10, 12, 14, 16])
def test_pml_each_size(L):
    """One lattice size, a ladder split over three workgroups (6 slots, 2 per
    workgroup: every cycle has pairs inside a workgroup and across its
    boundaries), proposals on every other slot."""
    announce(f"pml: L={L}, R=6, G=2, 60 sweeps in launches of 40")
    _run([(L, 6, 1), (L, 6, 2)], 2, 60)


def test_pml_mixed_sizes_one_launch():
    """Six lattice sizes in one launch, ladders of 8..12 slots over workgroups
    of up to 8 slots (uneven splits), M = 2."""
    announce("pml: L = 6..16 in one launch, R = 8..12, G = 8, M = 2")
    cases = [(6, 12, 3), (8, 9, 4), (10, 8, 5), (12, 10, 6), (14, 11, 7), (16, 12, 8)]
    plan = _run(cases, 8, 64, chunk=30, M=2)
    announce(f"plan {plan}")


@pytest.mark.parametrize("rule", ["metropolis", "gibbs"])
def test_pml_one_slot_per_workgroup(rule):
    """Every pair crosses a workgroup boundary (one slot per workgroup); the
    heat-bath rule as well as Metropolis."""
    announce(f"pml: L=10 and 12, R=5, G=1, {rule}")
    _run([(10, 5, 9), (12, 5, 10)], 1, 50, rule=rule)


def test_pml_independent_chains():
    """Independent chains (M = 0: no exchange, the bank-generation runs)."""
    announce("pml: independent chains, L = 6 and 14, R = 8, G = 4")
    _run([(6, 8, 11), (14, 8, 12)], 4, 50, M=0)


def test_pml_first_hit_and_long_launch():
    """A target energy (first hit recorded) and one launch of 300 sweeps."""
    announce("pml: L=8 R=8 G=4 target -600, 300 sweeps in one launch")
    _run([(8, 8, 13)], 4, 300, chunk=300, target=-600)
