"""GPU vs oracle parity of the packed-row sparse sweepers: one storage per
lane (CsrRowSweep, kernel "row") and four interleaved storages per lane
(CsrRowQuadSweep, kernel "row4"), where each thread keeps one item per colour
class for the whole launch; and of the runtime's choice among all sparse
sweepers. Bit-exact spins, energies, counters and best record against the
oracle; the launch plan is checked so that each case runs the sweeper it
names."""
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


def _run_and_compare(problems, betas, G, sweeps, M=1, chunk=50, bank_every=3, expect="csr-row", kernel="row",
                     rule="metropolis"):
    import oracle
    R = len(betas)
    ctxs, cases = [], []
    for i, g in enumerate(problems):
        banks = ({r: inputs.random_bank(g["n"], 5, seed=5800 + 32 * i + r, clamp=g["clamp"])
                  for r in range(0, R - 2, bank_every)} if M else None)
        kw = dict(M=M, rule=rule)
        if M:
            kw.update(prop_start=2 * M, prop_period=3 * M)
        c = binding.Context(g, betas, seed=5900 + i, **kw)
        for r, b in (banks or {}).items():
            c.propose(r, b)
        ctxs.append(c)
        cases.append((g, banks, kw, 5900 + i))
    bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=chunk, kernel=kernel)
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


SWEEPER = {"row": "csr-row", "row4": "csr-row4"}


@pytest.mark.parametrize("kernel", ["row", "row4"])
@pytest.mark.parametrize("m,R,G", [(8, 32, 4), (8, 29, 8), (8, 24, 1), (10, 24, 4), (6, 16, 3), (8, 26, 13),
                                   (8, 32, 32)])
def test_multipliers_row_sweepers(kernel, m, R, G):
    """Multipliers: one lane per item (m = 6, 8: degree <= 16) and two lanes
    per item (m = 10: degree 20, sums combined by DPP); an uneven split of
    the ladder (R = 29 over workgroups of 8 and 7 slots); one slot per
    workgroup; slot counts that leave padding storages in the last quad
    (G = 1, 3, 13); a whole ladder in one workgroup (G = 32)."""
    if kernel == "row" and G > 12:
        pytest.skip("one storage per lane: 40 sites x 32 slots exceed a block")
    announce(f"{kernel} sweeper: 2 x {m}-bit multipliers, R={R} G={G}")
    betas = inputs.geometric_ladder(R)
    probs = [inputs.multiplier(m, C) for C, _, _ in inputs.semiprimes(m, 2, seed=6100 + m)]
    plan = _run_and_compare(probs, betas, G, 120, expect=SWEEPER[kernel], kernel=kernel)
    announce(f"plan {plan}")


@pytest.mark.parametrize("kernel", ["row", "row4"])
@pytest.mark.parametrize("seed", [1, 2])
def test_random_graphs_row_sweepers(kernel, seed):
    """Random sparse graphs with |J| up to 7, fields, clamped sites, hub sites
    of degree about 25 (two lanes per item) and DSATUR colourings."""
    probs = [_random_graph(150, 6200 + 10 * seed + k) for k in range(2)]
    for g in probs:
        deg = np.diff(g["row_ptr"])[g["clamp"] == 0]
        assert 16 < deg.max() <= 32 and np.abs(g["J"]).max() <= 7
    announce(f"{kernel} sweeper: random graphs n=150 seed={seed}, max degree "
             f"{max(int(np.diff(g['row_ptr']).max()) for g in probs)}, colours {[int(g['color'].max()) + 1 for g in probs]}")
    _run_and_compare(probs, inputs.geometric_ladder(12), 5, 150, expect=SWEEPER[kernel], kernel=kernel)


@pytest.mark.parametrize("kernel", ["row", "row4"])
def test_row_sweepers_independent_chains(kernel):
    """Independent chains (M = 0: no exchange, the bank-generation runs)."""
    announce(f"{kernel} sweeper: independent chains, 2 x 8-bit multipliers, R=16 G=4")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6300)]
    _run_and_compare(probs, np.full(16, 1.3), 4, 100, M=0, expect=SWEEPER[kernel], kernel=kernel)


def _pad_isolated(g, k):
    """g with k more free sites that have no bonds: they join colour 0,
    which then holds more than the 256 sites of the one-slot-per-wavefront
    sparse kernel's limit."""
    n = g["n"] + k
    rp = np.concatenate([g["row_ptr"], np.full(k, g["row_ptr"][-1])])
    out = inputs.graph(n, rp, g["col"], g["J"], h=np.concatenate([g["h"], np.zeros(k, np.int64)]),
                       clamp=np.concatenate([g["clamp"], np.zeros(k, np.int8)]))
    return out


def test_runtime_sparse_sweeper_choice():
    """The runtime's choice among the sweepers of the workgroup-synchronous
    kernel, each against the oracle (general graphs that fit it take the
    one-slot-per-wavefront kernel first): that kernel for 8- and 10-bit
    multipliers (auto; the 10-bit one has sites of degree 20); the one-storage
    rows for a graph with a colour class of more than 256 sites where a site's
    bound exceeds 255 (a field of 250); the four-storages-per-lane LDS sweeper
    where no packed rows fit a block (|J| = 9, a colour class of more than 256
    sites, 20 slots per workgroup); the LDS-resident CSR sweepers when the
    caller asks for the workgroup-synchronous kernel (the lane-sharing one at
    512 threads for 2 slots per workgroup); and a coupling of 9 refused by the
    one-storage rows and run in the four-storage rows (with a class of more
    than 256 sites)."""
    announce("sparse sweeper choice: csrw / row / quad / csr / csr-wide / row4, refusal")
    mult = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 1, seed=6400)]
    plan = _run_and_compare(mult, inputs.geometric_ladder(32), 8, 60, expect="-", kernel="auto")
    assert plan[0][0] == "csrw", plan
    m10a = [inputs.multiplier(10, C) for C, _, _ in inputs.semiprimes(10, 1, seed=6405)]
    plan = _run_and_compare(m10a, inputs.geometric_ladder(16), 4, 60, expect="-", kernel="auto")
    assert plan[0][0] == "csrw", plan
    big = _random_graph(120, 6470, hubs=0)
    big["h"] = big["h"].copy()
    big["h"][int(np.argmax(big["clamp"] == 0))] = 250
    big = _pad_isolated(big, 260)
    assert np.bincount(big["color"][big["clamp"] == 0]).max() > 256
    _run_and_compare([big], inputs.geometric_ladder(8), 1, 60, expect="csr-row", kernel="auto")
    g9q = _pad_isolated(_random_graph(100, 6460, hubs=0, jmax=9), 240)
    assert np.bincount(g9q["color"][g9q["clamp"] == 0]).max() > 256
    _run_and_compare([g9q], inputs.geometric_ladder(20), 20, 40, expect="csr-quad", kernel="auto")
    _run_and_compare(mult, inputs.geometric_ladder(16), 4, 60, expect="csr", kernel="block")
    _run_and_compare(mult, inputs.geometric_ladder(16), 2, 60, expect="csr-wide", kernel="block")
    g9 = _random_graph(100, 6450, hubs=0, jmax=9)
    c = binding.Context(g9, inputs.geometric_ladder(8), seed=1)
    with pytest.raises(binding.TaptError):
        binding.Batch([c], replicas_per_wg=4, kernel="row")
    c.close()
    g9p = _pad_isolated(g9, 260)   # a class of more than 256 sites: not the one-slot-per-wavefront kernel
    assert np.bincount(g9p["color"][g9p["clamp"] == 0]).max() > 256
    _run_and_compare([g9p], inputs.geometric_ladder(8), 4, 60, expect="csr-row4", kernel="auto")   # |J| = 9


def test_independent_chains_auto_choice():
    """Independent chains (M = 0) of multipliers with the kernel left open take
    the workgroup-synchronous kernel at its coarsest tiling and the
    four-storages-per-lane LDS sweeper (neither the packed rows nor the
    one-slot-per-wavefront kernel); with exchanges (M = 1) the same circuits
    take the one-slot-per-wavefront kernel. Both against the oracle."""
    announce("sparse auto choice: independent chains -> csr-quad, exchanging chains -> csrw")
    probs = [inputs.multiplier(8, C) for C, _, _ in inputs.semiprimes(8, 2, seed=6480)]
    plan = _run_and_compare(probs, np.full(32, 1.1), 0, 60, M=0, expect="csr-quad", kernel="auto")
    assert plan[0][0] == "chunk", plan
    plan = _run_and_compare(probs, inputs.geometric_ladder(16), 0, 60, M=1, expect="-", kernel="auto")
    assert plan[0][0] == "csrw", plan
