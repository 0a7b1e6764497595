"""GPU vs oracle parity of the one-slot-per-wavefront sparse kernel (kernel
"csrw"): bit-exact spins, energies, counters and best record against the
oracle, with the launch plan checked."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce
from tests.test_gpu_row_sweeper import _pad_isolated, _random_graph, _run_and_compare

pytestmark = pytest.mark.gpu


def _plan_kernel(problems, betas, G):
    ctxs = [binding.Context(g, betas, seed=1) for g in problems]
    try:
        bt = binding.Batch(ctxs, replicas_per_wg=G, kernel="csrw")
        plan = bt.describe()
        bt.close()
        return plan
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("m,R,G", [(8, 32, 8), (8, 29, 4), (6, 16, 1), (8, 12, 5), (10, 16, 8), (12, 12, 4)])
def test_multipliers_csrw(m, R, G):
    """Multipliers (clamped product bits, five colour classes, fields): slots
    per workgroup 8, 4 (an uneven split: R = 29), 1 (every pair across a
    workgroup boundary) and 5; 10- and 12-bit ones have input sites of degree
    20 and 24 (three bond chunks) and, at 12 bits, classes of more than 64
    sites (two rank groups each)."""
    announce(f"csrw: 2 x {m}-bit multipliers, R={R} G={G}")
    probs = [inputs.multiplier(m, C) for C, _, _ in inputs.semiprimes(m, 2, seed=6500 + m)]
    assert [d["kernel"] for d in _plan_kernel(probs, inputs.geometric_ladder(R), G)] == ["csrw"]
    _run_and_compare(probs, inputs.geometric_ladder(R), G, 120, expect="-", kernel="csrw")


@pytest.mark.parametrize("seed,hubs,jmax", [(1, 0, 7), (2, 0, 7), (3, 4, 7), (4, 3, 40)])
def test_random_graphs_csrw(seed, hubs, jmax):
    """Random sparse graphs with fields, clamped sites and DSATUR colourings,
    6 slots per workgroup: |J| up to 7 and degree <= 16; hub sites of degree
    above 16 (up to four bond chunks); couplings up to 40 (bytes in the dot
    products)."""
    probs = [_random_graph(150, 6600 + 10 * seed + k, hubs=hubs, jmax=jmax) for k in range(2)]
    for g in probs:
        dmax = np.diff(g["row_ptr"])[g["clamp"] == 0].max()
        assert (dmax <= 16) if hubs == 0 else (16 < dmax <= 64), dmax
        assert np.abs(g["J"]).max() <= jmax
    announce(f"csrw: random graphs n=150 seed={seed} hubs={hubs} |J|<={jmax}, "
             f"colours {[int(g['color'].max()) + 1 for g in probs]}")
    _run_and_compare(probs, inputs.geometric_ladder(12), 6, 150, expect="-", kernel="csrw")


@pytest.mark.parametrize("M,chunk", [(3, 50), (4, 30), (2, 7)])
def test_csrw_cycle_lengths(M, chunk):
    """Several sweeps per exchange cycle (M = 2, 3, 4), with launches of 50,
    30 and 7 sweeps that end inside a cycle: the next sweep's uniforms are drawn
    during a cycle end's wait only when that sweep belongs to the same launch."""
    announce(f"csrw: M={M}, launches of {chunk} sweeps, 2 x 8-bit multipliers, R=16 G=4")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6770)]
    _run_and_compare(probs, inputs.geometric_ladder(16), 4, 130, M=M, chunk=chunk, expect="-", kernel="csrw")


@pytest.mark.parametrize("rule", ["metropolis", "gibbs"])
def test_csrw_rules_and_extreme_betas(rule):
    """The flip decision from the flip probability in FP32, with the table read
    only near a uniform's edge, under both rules and at the ends of the range
    of beta: a slot that accepts almost everything (beta = 0.001), one that
    accepts almost nothing uphill (beta = 40: the probability underflows FP32
    for most fields), and couplings up to 40 (fields up to several hundred)."""
    betas = np.array([0.001, 0.05, 0.2, 0.6, 1.5, 3.0, 8.0, 40.0])
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 1, seed=6750)]
    probs.append(_random_graph(150, 6760, hubs=3, jmax=40))
    announce(f"csrw: {rule}, betas {betas.tolist()}, 8-bit multiplier and a random graph with |J| <= 40")
    _run_and_compare(probs, betas, 4, 150, expect="-", kernel="csrw", rule=rule)


def test_csrw_independent_chains_and_refusal():
    """Independent chains (M = 0); a graph with a colour class of more than
    256 sites is refused."""
    announce("csrw: independent chains, 2 x 8-bit multipliers, R=16 G=8; refusal at a class of 300+ sites")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6700)]
    _run_and_compare(probs, np.full(16, 1.3), 8, 100, M=0, expect="-", kernel="csrw")
    big = _pad_isolated(_random_graph(120, 6710, hubs=0), 280)
    assert np.bincount(big["color"][big["clamp"] == 0]).max() > 256
    c = binding.Context(big, inputs.geometric_ladder(8), seed=1)
    bt = binding.Batch([c], replicas_per_wg=4, kernel="csrw")   # falls back: a class of more than 256 sites
    assert [d["kernel"] for d in bt.describe()] != ["csrw"], bt.describe()
    bt.close()
    c.close()
