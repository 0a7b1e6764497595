"""GPU vs oracle parity of the packed-row sparse sweeper (CsrRowSweep): the
fine tilings of general graphs, where each thread keeps one (site, storage)
item per colour class. Bit-exact spins, energies, counters and best record
against the oracle; the launch plan is checked so that each case runs the
sweeper it names."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce, compare

pytestmark = pytest.mark.gpu


def _random_graph(n, seed, hubs=3, jmax=7):
    """Sparse symmetric graph: a random base of degree about 6, a few hub
    sites of degree about 25 (two lanes per item), couplings in
    [-jmax, jmax] without 0, fields in [-5, 5], about 5 % clamped sites."""
    rng = np.random.default_rng(seed)
    Jd = np.zeros((n, n), np.int64)
    for _ in range(3 * n):
        i, j = rng.integers(0, n, 2)
        if i != j:
            v = int(rng.integers(1, jmax + 1)) * (1 if rng.random() < 0.5 else -1)
            Jd[i, j] = Jd[j, i] = v
    for hub in rng.choice(n, hubs, replace=False):
        for j in rng.choice(n, 20, replace=False):
            if j != hub:
                v = int(rng.integers(1, jmax + 1)) * (1 if rng.random() < 0.5 else -1)
                Jd[hub, j] = Jd[j, hub] = v
    rp, col, J = inputs.dense_to_csr(Jd)
    h = rng.integers(-5, 6, n)
    clamp = np.where(rng.random(n) < 0.05, rng.choice([-1, 1], n), 0)
    return inputs.graph(n, rp, col, J, h=h, clamp=clamp)


def _plan(bt):
    return [(d["kernel"], d["sweeper"], d["block"]) for d in bt.describe()]


def _run_and_compare(problems, betas, G, sweeps, M=1, chunk=50, bank_every=3, expect="csr-row"):
    import oracle
    R = len(betas)
    ctxs, cases = [], []
    for i, g in enumerate(problems):
        banks = ({r: inputs.random_bank(g["n"], 5, seed=5800 + 32 * i + r, clamp=g["clamp"])
                  for r in range(0, R - 2, bank_every)} if M else None)
        kw = dict(M=M)
        if M:
            kw.update(prop_start=2 * M, prop_period=3 * M)
        c = binding.Context(g, betas, seed=5900 + i, **kw)
        for r, b in (banks or {}).items():
            c.propose(r, b)
        ctxs.append(c)
        cases.append((g, banks, kw, 5900 + i))
    bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=chunk)
    plan = _plan(bt)
    assert all(p[1] == expect for p in plan), plan
    bt.sweep(sweeps)
    bt.close()
    for c, (g, banks, kw, seed) in zip(ctxs, cases):
        ref = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
        ref.run(sweeps)
        compare(c, ref)
        c.close()
    return plan


@pytest.mark.parametrize("m,R,G", [(8, 32, 4), (8, 29, 8), (8, 24, 1), (10, 24, 4), (6, 16, 3)])
def test_multipliers_row_sweeper(m, R, G):
    """Multipliers: one lane per item (m = 6, 8: degree <= 16) and two lanes
    per item (m = 10: degree 20, bonds summed by DPP); an uneven split of the
    ladder (R = 29 over workgroups of 8 and 7 slots); one slot per workgroup."""
    announce(f"row sweeper: 2 x {m}-bit multipliers, R={R} G={G}")
    betas = inputs.geometric_ladder(R)
    probs = [inputs.multiplier(m, C) for C, _, _ in inputs.semiprimes(m, 2, seed=6100 + m)]
    plan = _run_and_compare(probs, betas, G, 120)
    announce(f"plan {plan}")


@pytest.mark.parametrize("seed", [1, 2])
def test_random_graphs_row_sweeper(seed):
    """Random sparse graphs with |J| up to 7, fields, clamped sites, hub sites
    of degree about 25 (two lanes per item) and DSATUR colourings."""
    probs = [_random_graph(150, 6200 + 10 * seed + k) for k in range(2)]
    for g in probs:
        deg = np.diff(g["row_ptr"])[g["clamp"] == 0]
        assert 16 < deg.max() <= 32 and np.abs(g["J"]).max() <= 7
    announce(f"row sweeper: random graphs n=150 seed={seed}, max degree "
             f"{max(int(np.diff(g['row_ptr']).max()) for g in probs)}, colours {[int(g['color'].max()) + 1 for g in probs]}")
    _run_and_compare(probs, inputs.geometric_ladder(12), 4, 150)


def test_row_sweeper_independent_chains():
    """Independent chains (M = 0: no exchange, the bank-generation runs)."""
    announce("row sweeper: independent chains, 2 x 8-bit multipliers, R=16 G=4")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6300)]
    _run_and_compare(probs, np.full(16, 1.3), 4, 100, M=0)


def test_coarse_tiling_and_large_couplings_leave_row_sweeper():
    """Where the packed rows do not apply the runtime keeps the other
    sweepers, with the same chain: 16 slots per workgroup of an 8-bit
    multiplier need 640 threads (the four-storages-per-lane sweeper runs), and
    a coupling of 9 does not fit the 4-bit field (the CSR sweeper runs)."""
    announce("row sweeper: fallbacks (G=16 multiplier, |J| = 9 graph)")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 1, seed=6400)]
    _run_and_compare(probs, inputs.geometric_ladder(32), 16, 60, expect="csr-quad")
    _run_and_compare([_random_graph(100, 6450, hubs=0, jmax=9)], inputs.geometric_ladder(8), 4, 60, expect="csr")
