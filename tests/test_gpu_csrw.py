"""GPU vs oracle parity of the one-slot-per-wavefront sparse kernel (kernel
"csrw"): bit-exact spins, energies, counters and best record against the
oracle, with the launch plan checked."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce
from tests.test_gpu_row_sweeper import _random_graph, _run_and_compare

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


@pytest.mark.parametrize("m,R,G", [(8, 32, 8), (8, 29, 4), (6, 16, 1), (8, 12, 5)])
def test_multipliers_csrw(m, R, G):
    """Multipliers (clamped product bits, five colour classes, fields): slots
    per workgroup 8, 4 (an uneven split: R = 29), 1 (every pair across a
    workgroup boundary) and 5."""
    announce(f"csrw: 2 x {m}-bit multipliers, R={R} G={G}")
    probs = [inputs.multiplier(m, C) for C, _, _ in inputs.semiprimes(m, 2, seed=6500 + m)]
    assert [d["kernel"] for d in _plan_kernel(probs, inputs.geometric_ladder(R), G)] == ["csrw"]
    _run_and_compare(probs, inputs.geometric_ladder(R), G, 120, expect="-", kernel="csrw")


@pytest.mark.parametrize("seed", [1, 2])
def test_random_graphs_csrw(seed):
    """Random sparse graphs with |J| up to 7, fields, clamped sites and DSATUR
    colourings (degree <= 16), 6 slots per workgroup."""
    probs = [_random_graph(150, 6600 + 10 * seed + k, hubs=0) for k in range(2)]
    for g in probs:
        assert np.diff(g["row_ptr"])[g["clamp"] == 0].max() <= 16
    announce(f"csrw: random graphs n=150 seed={seed}, colours {[int(g['color'].max()) + 1 for g in probs]}")
    _run_and_compare(probs, inputs.geometric_ladder(12), 6, 150, expect="-", kernel="csrw")


def test_csrw_independent_chains_and_refusal():
    """Independent chains (M = 0); a 10-bit multiplier (degree 20) is refused."""
    announce("csrw: independent chains, 2 x 8-bit multipliers, R=16 G=8; refusal at degree 20")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6700)]
    _run_and_compare(probs, np.full(16, 1.3), 8, 100, M=0, expect="-", kernel="csrw")
    g10 = inputs.multiplier(10, inputs.semiprimes(10, 1, seed=6710)[0][0])
    c = binding.Context(g10, inputs.geometric_ladder(8), seed=1)
    bt = binding.Batch([c], replicas_per_wg=4, kernel="csrw")   # falls back: degree 20 > 16
    assert [d["kernel"] for d in bt.describe()] != ["csrw"], bt.describe()
    bt.close()
    c.close()
