"""GPU vs oracle parity: the HIP path must realise the same chain bit for bit
(spins, integer energies, counters, best record) for the same seeds."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce, compare, make_pair

pytestmark = pytest.mark.gpu


def _cfg1():
    return inputs.ea_lattice(4, 1), inputs.geometric_ladder(16)


def test_plain_path_cfg1():
    announce("plain path, EA L=4 R=16, 200 sweeps")
    g, b = _cfg1()
    ctx, ref = make_pair(g, b, seed=1001)
    ctx.sweep(200)
    ref.run(200)
    compare(ctx, ref)


@pytest.mark.parametrize("G,rpt,K", [(16, 1, 1000), (16, 2, 64), (5, 1, 37), (4, 2, 200), (3, 4, 50), (1, 1, 100)])
def test_batched_tilings_cfg1(G, rpt, K):
    announce(f"batched EA L=4 R=16, G={G} rpt={rpt} K={K}, 300 sweeps")
    g, b = _cfg1()
    ctx, ref = make_pair(g, b, seed=1001)
    bt = binding.Batch([ctx], replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=K)
    bt.sweep(300)
    ref.run(300)
    compare(ctx, ref)


def test_cfg1_full_1000_sweeps_graph():
    announce("batched EA L=4 R=16, 1000 sweeps, hipGraph replay")
    g, b = _cfg1()
    ctx, ref = make_pair(g, b, seed=1001, target=-100)
    bt = binding.Batch([ctx], chunk_sweeps=128, use_graph=True)
    bt.sweep(1000)
    ref.run(1000)
    compare(ctx, ref)


def test_graph_replays_match_eager_after_every_replay():
    """hipGraph path: each replay (one chunk) is checked against an eager batch
    of the same contexts, with eager work and synchronisations between replays."""
    announce("hipGraph replays vs eager batch, EA L=4 R=16 x 3 instances, split ladders, 6 replays")
    g, b = _cfg1()
    banks = {r: inputs.random_bank(64, 5, seed=900 + r) for r in range(10)}
    kw = dict(prop_start=4, prop_period=8)
    pairs = []
    for k in range(3):
        a = binding.Context(g, b, seed=40 + k, **kw)
        e = binding.Context(g, b, seed=40 + k, **kw)
        for r, bk in banks.items():
            a.propose(r, bk)
            e.propose(r, bk)
        pairs.append((a, e))
    bg = binding.Batch([p[0] for p in pairs], replicas_per_wg=5, chunk_sweeps=24, use_graph=True)
    be = binding.Batch([p[1] for p in pairs], replicas_per_wg=5, chunk_sweeps=24)
    for rep in range(6):
        bg.sweep(24)
        be.sweep(24)
        for a, e in pairs:
            sa, ta = a.state()
            se, te = e.state()
            assert ta == te == 24 * (rep + 1)
            assert np.array_equal(sa, se), rep
            assert np.array_equal(a.energies(), e.energies()), rep
            assert a.summary()["best"] == e.summary()["best"]
    bg.close()
    be.close()


@pytest.mark.parametrize("path", ["plain", "batched", "split"])
def test_proposals(path):
    announce(f"proposals, {path}")
    g, b = _cfg1()
    banks = {r: inputs.random_bank(64, 9, seed=200 + r) for r in range(14)}
    ctx, ref = make_pair(g, b, seed=77, banks=banks, prop_start=4, prop_period=6, prop_stop=150)
    if path == "plain":
        ctx.sweep(180)
    else:
        bt = binding.Batch([ctx], replicas_per_wg=16 if path == "batched" else 6, chunk_sweeps=45)
        bt.sweep(180)
    ref.run(180)
    compare(ctx, ref)


@pytest.mark.parametrize("rule,M", [("gibbs", 1), ("metropolis", 3), ("gibbs", 4)])
def test_rules_and_cycle_length(rule, M):
    announce(f"rule={rule} M={M}")
    g, b = _cfg1()
    banks = {r: inputs.random_bank(64, 5, seed=300 + r) for r in range(0, 12, 2)}
    kw = dict(rule=rule, M=M, prop_start=2 * M, prop_period=2 * M)
    ctx, ref = make_pair(g, b, seed=5, banks=banks, **kw)
    ctx2, _ = make_pair(g, b, seed=5, banks=banks, **kw)
    ctx.sweep(121)
    bt = binding.Batch([ctx2], replicas_per_wg=5, chunk_sweeps=40)
    bt.sweep(121)
    ref.run(121)
    compare(ctx, ref)
    compare(ctx2, ref)


@pytest.mark.parametrize("L,R", [(6, 8), (8, 12), (10, 6), (12, 4), (14, 3), (16, 4)])
def test_lattice_sizes(L, R):
    announce(f"lattice L={L} R={R}")
    g = inputs.ea_lattice(L, 10 + L)
    b = inputs.geometric_ladder(R)
    ctx, ref = make_pair(g, b, seed=L)
    ctx2, _ = make_pair(g, b, seed=L)
    bt = binding.Batch([ctx2], chunk_sweeps=25)
    bt.sweep(60)
    ctx.sweep(60)
    ref.run(60)
    compare(ctx, ref)
    compare(ctx2, ref)


@pytest.mark.parametrize("m", [3, 4, 6])
def test_factorization_csr(m):
    announce(f"multiplier m={m} (CSR kernel, clamps, DSATUR colors)")
    ps = inputs.primes_in(1 << (m - 1), 1 << m)
    C = ps[0] * ps[-1]
    g = inputs.multiplier(m, C)
    b = inputs.geometric_ladder(12)
    egnd = -3 * m * m - 4 * m * (m - 1)
    banks = {r: np.stack([inputs.multiplier_assignment(g, ps[0], ps[-1])] * 2 + [inputs.random_bank(g["n"], 1, seed=r, clamp=g["clamp"])[0]])
             for r in range(3)}
    ctx, ref = make_pair(g, b, seed=m, banks=banks, prop_start=20, prop_period=20, target=egnd)
    ctx2, _ = make_pair(g, b, seed=m, banks=banks, prop_start=20, prop_period=20, target=egnd)
    ctx.sweep(100)
    bt = binding.Batch([ctx2], replicas_per_wg=5, chunk_sweeps=30)
    bt.sweep(100)
    ref.run(100)
    compare(ctx, ref)
    compare(ctx2, ref)


def test_gadget_sequential_colors():
    announce("full adder, one color per spin (sequential sweep)")
    g = inputs.gadget_graph("fa")
    b = np.array([0.5, 1.7, 4.6])
    ctx, ref = make_pair(g, b, seed=3, rule="gibbs")
    ctx.sweep(500)
    ref.run(500)
    compare(ctx, ref)


def test_mixed_batch_and_switching_paths():
    announce("mixed batch (lattices of 3 sizes + CSR), then plain, then batched again")
    probs = [(inputs.ea_lattice(4, 2), inputs.geometric_ladder(7)),
             (inputs.ea_lattice(6, 3), inputs.geometric_ladder(9)),
             (inputs.ea_lattice(8, 4), inputs.geometric_ladder(10)),
             (inputs.multiplier(4, 11 * 13), inputs.geometric_ladder(8))]
    pairs = [make_pair(g, b, seed=40 + k) for k, (g, b) in enumerate(probs)]
    bt = binding.Batch([p[0] for p in pairs], replicas_per_wg=4, chunk_sweeps=33)
    bt.sweep(70)
    for ctx, _ in pairs:
        ctx.sweep(11)
    bt.sweep(40)
    for ctx, ref in pairs:
        ref.run(121)
        compare(ctx, ref)


def test_resume_from_saved_state():
    announce("save / restore / continue")
    g, b = _cfg1()
    ctx, ref = make_pair(g, b, seed=9)
    ctx.sweep(50)
    spins, t = ctx.state()
    ctx2 = binding.Context(g, b, seed=9)
    ctx2.set_state(spins, t)
    bt = binding.Batch([ctx2], replicas_per_wg=8, chunk_sweeps=20)
    bt.sweep(70)
    ref.run(120)
    s2, t2 = ctx2.state()
    assert t2 == 120
    assert np.array_equal(s2, ref.spins)
    assert np.array_equal(ctx2.energies(), ref.E)


def test_bank_energies_and_energy_kernel():
    announce("energy kernel vs oracle energy")
    import torch
    import oracle
    g = inputs.ea_lattice(8, 5)
    ctx = binding.Context(g, inputs.geometric_ladder(4), seed=1)
    cfg = inputs.random_bank(512, 33, seed=9)
    dev = torch.from_numpy(cfg).cuda()
    out = torch.zeros(33, dtype=torch.int32, device="cuda")
    ctx.energy_device(dev.data_ptr(), 33, out.data_ptr())
    torch.cuda.synchronize()
    run = oracle.Run(g, [1.0], seed=0)
    want = np.array([run.energy(c) for c in cfg])
    assert np.array_equal(out.cpu().numpy(), want)


def test_invalid_inputs_rejected():
    announce("argument validation")
    g, b = _cfg1()
    with pytest.raises(binding.TaptError):
        binding.Context(g, b[::-1], seed=1)
    ctx = binding.Context(g, b, seed=1)
    bad = np.zeros((2, 64), np.int8)
    with pytest.raises(binding.TaptError):
        ctx.propose(0, bad)
    m = inputs.multiplier(3, 35)
    ctxm = binding.Context(m, b[:4], seed=1)
    wrong = inputs.random_bank(m["n"], 2, seed=1)          # ignores the clamps
    if np.any((m["clamp"] != 0) & (wrong[0] != m["clamp"])):
        with pytest.raises(binding.TaptError):
            ctxm.propose(0, wrong)


@pytest.mark.parametrize("G,rpt,kernel", [(4, 4, "auto"), (4, 1, "auto"), (2, 1, "auto"), (8, 1, "pm1"), (8, 1, "pm")])
def test_many_instances_split_ladders(G, rpt, kernel):
    """64 EA L=8 instances with R=32 split into 32/G workgroups each, several
    launches; sampled instances checked against the oracle. (8, 1, pm1) is
    the benchmark's own launch configuration."""
    announce(f"64 instances, L=8 R=32, G={G} rpt={rpt} kernel={kernel}, 3 launches of 40 sweeps")
    from tests.gpu_util import make_pair
    betas = inputs.geometric_ladder(32)
    pairs = []
    for i in range(64):
        g = inputs.ea_lattice(8, 2000 + i)
        banks = {r: inputs.random_bank(512, 4, seed=7000 + 64 * i + r) for r in range(0, 30, 7)} if i % 8 == 0 else None
        kw = dict(prop_start=20, prop_period=20) if banks else {}
        ctx = binding.Context(g, betas, seed=3000 + i, **kw)
        if banks:
            for r, b in banks.items():
                ctx.propose(r, b)
        pairs.append((ctx, g, banks, kw))
    bt = binding.Batch([p[0] for p in pairs], replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=40,
                       kernel=kernel)
    bt.sweep(120)
    import oracle
    for i in (0, 8, 37, 63):
        ctx, g, banks, kw = pairs[i]
        ref = oracle.Run(g, betas, seed=3000 + i, banks=banks, **kw)
        ref.run(120)
        compare(ctx, ref)


def test_mixed_sizes_one_launch():
    """Lattices L = 6..16 with ladders of 24..48 slots and a multiplier, all in
    one launch of the mixed kernel; every instance checked against the oracle."""
    announce("mixed sizes L=6,8,10,12,16 (R=24..48) + 5-bit multiplier, one mixed launch, 60 sweeps")
    sizes = [(6, 24), (8, 30), (10, 36), (12, 42), (16, 48)]
    cases = []
    for k, (L, R) in enumerate(sizes):
        g = inputs.ea_lattice(L, 3000 + k)
        banks = {r: inputs.random_bank(g["n"], 3, seed=8000 + 64 * k + r) for r in range(0, R - 2, 5)}
        cases.append((g, inputs.geometric_ladder(R), banks, dict(prop_start=20, prop_period=20), 3000 + k))
    m = inputs.multiplier(5, 17 * 29)
    cases.append((m, inputs.geometric_ladder(16), None, {}, 99))
    ctxs = []
    for g, b, banks, kw, seed in cases:
        ctx = binding.Context(g, b, seed=seed, **kw)
        for r, bank in (banks or {}).items():
            ctx.propose(r, bank)
        ctxs.append(ctx)
    bt = binding.Batch(ctxs, chunk_sweeps=25)
    bt.sweep(60)
    import oracle
    for ctx, (g, b, banks, kw, seed) in zip(ctxs, cases):
        ref = oracle.Run(g, b, seed=seed, banks=banks, **kw)
        ref.run(60)
        compare(ctx, ref)


@pytest.mark.parametrize("kernel,G,rule,M", [("pm", 8, "metropolis", 1), ("pm", 2, "gibbs", 1), ("pm", 4, "metropolis", 3),
                                             ("pm", 16, "gibbs", 2), ("wave", 8, "metropolis", 1), ("wave", 3, "gibbs", 2),
                                             ("block", 8, "metropolis", 1), ("pm1", 8, "metropolis", 1),
                                             ("pm1", 1, "gibbs", 1), ("pm1", 5, "metropolis", 3), ("pm1", 3, "gibbs", 2)])
def test_l8_kernels(kernel, G, rule, M):
    """The persistent kernels that run 8^3 lattices (the +-J kernel with two
    slots or one slot per wavefront, wave-per-replica, workgroup-synchronous),
    on the benchmark's shape (R = 32, proposals from banks) for several
    instances."""
    announce(f"L=8 R=32 x 6 instances, kernel={kernel} G={G} rule={rule} M={M}, 2 launches of 90 sweeps")
    betas = inputs.geometric_ladder(32)
    cases = []
    for i in range(6):
        g = inputs.ea_lattice(8, 4100 + i)
        banks = {r: inputs.random_bank(512, 5, seed=9100 + 40 * i + r) for r in range(0, 30, 3)}
        cases.append((g, banks, 6100 + i))
    kw = dict(rule=rule, M=M, prop_start=6 * M, prop_period=6 * M, target=-700)
    ctxs = []
    for g, banks, seed in cases:
        c = binding.Context(g, betas, seed=seed, **kw)
        for r, b in banks.items():
            c.propose(r, b)
        ctxs.append(c)
    bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=90, kernel=kernel)
    bt.sweep(180)
    import oracle
    for c, (g, banks, seed) in zip(ctxs, cases):
        ref = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
        ref.run(180)
        compare(c, ref)


def test_mixed_sizes_full_batch():
    """The mixed-size workload at its full count: 8 instances of each of
    L = 6, 8, 10, 12, 16 with ladders of 24..48 slots, proposals every 50
    sweeps, one persistent launch; one instance per size checked against
    the oracle, every instance against its own recomputed energies."""
    announce("mixed sizes x 8 instances each (40 contexts, 1440 replicas), one launch, 2 x 50 sweeps")
    import oracle
    sizes = [(6, 24), (8, 30), (10, 36), (12, 42), (16, 48)]
    ctxs, cases = [], []
    for k, (L, R) in enumerate(sizes):
        betas = inputs.geometric_ladder(R)
        for i in range(8):
            g = inputs.ea_lattice(L, 3000 + 10 * k + i)
            banks = {r: inputs.random_bank(g["n"], 3, seed=8000 + 100 * k + 10 * i + r) for r in range(0, R - 2, 8)}
            kw = dict(prop_start=50, prop_period=50)
            c = binding.Context(g, betas, seed=300 + 10 * k + i, **kw)
            for r, b in banks.items():
                c.propose(r, b)
            ctxs.append(c)
            cases.append((g, betas, banks, kw, 300 + 10 * k + i, i == 0))
    bt = binding.Batch(ctxs, chunk_sweeps=50)
    bt.sweep(100)
    for c, (g, betas, banks, kw, seed, check) in zip(ctxs, cases):
        spins, t = c.state()
        assert t == 100
        erun = oracle.Run(g, [1.0], seed=0)
        want = np.array([erun.energy(spins[r]) for r in range(len(betas))])
        assert np.array_equal(c.energies(), want)
        if check:
            ref = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
            ref.run(100)
            compare(c, ref)


def test_factorization_batch_8bit():
    """8 x 8-bit multipliers (200 spins, 176 free) with R = 32 in one launch,
    the factorization batch's shape; two instances checked against the oracle."""
    announce("8-bit multipliers x 8 products, R=32, one launch, 120 sweeps")
    import oracle
    betas = inputs.geometric_ladder(32)
    egnd = -3 * 64 - 4 * 8 * 7
    ctxs, cases = [], []
    for i, (C, p, q) in enumerate(inputs.semiprimes(8, 8, seed=4000)):
        g = inputs.multiplier(8, C)
        banks = {r: inputs.random_bank(g["n"], 4, seed=4100 + 32 * i + r, clamp=g["clamp"]) for r in range(0, 23, 4)}
        kw = dict(prop_start=20, prop_period=20, target=egnd)
        c = binding.Context(g, betas, seed=4200 + i, **kw)
        for r, b in banks.items():
            c.propose(r, b)
        ctxs.append(c)
        cases.append((g, banks, kw, 4200 + i))
    bt = binding.Batch(ctxs, chunk_sweeps=60)
    bt.sweep(120)
    for i in (0, 5):
        g, banks, kw, seed = cases[i]
        ref = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
        ref.run(120)
        compare(ctxs[i], ref)


@pytest.mark.parametrize("case", ["plain", "block", "pm", "pm1", "csr"])
def test_independent_chains(case):
    """Independent chains (no cycle end, equal betas allowed): the
    bank-generation runs of Supp. Table S3, on every kernel family."""
    announce(f"independent chains, {case}")
    import oracle
    if case == "csr":
        ps = inputs.primes_in(8, 16)
        g = inputs.multiplier(4, ps[0] * ps[-1])
        betas = np.full(8, 1.5)
    elif case in ("pm", "pm1"):
        g = inputs.ea_lattice(8, 41)
        betas = np.full(16, 1.0)
    else:
        g = inputs.ea_lattice(6 if case == "plain" else 10, 42)
        betas = np.array([0.8, 0.8, 1.6, 1.6, 2.4, 0.5])
    seeds = (900, 901)
    ctxs = [binding.Context(g, betas, seed=s, M=0) for s in seeds]
    if case == "plain":
        ctxs[0].sweep(30)
        ctxs[0].sweep(30)
        ctxs = ctxs[:1]
    else:
        kern = {"block": "block", "pm": "pm", "pm1": "pm1", "csr": "auto"}[case]
        G = {"block": 4, "pm": 8, "pm1": 4, "csr": 4}[case]
        bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=30, kernel=kern)
        bt.sweep(60)
    for c, s in zip(ctxs, seeds):
        ref = oracle.Run(g, betas, seed=s, M=0)
        ref.run(60)
        compare(c, ref)
        assert ref.swap_att.sum() == 0


def test_generate_bank_matches_independent_oracle_chains():
    """banks.generate_bank: sample j is slot j mod 1024 of context j // 1024,
    an independent chain at beta after the burn-in, bit for bit."""
    announce("generate_bank: 2100 chains of L=4 at beta 1.3, 40 sweeps, 3 contexts")
    import oracle
    from paper_2509_23043_amd import banks
    g = inputs.ea_lattice(4, 61)
    timing = {}
    cfg, E = banks.generate_bank(g, 1.3, 2100, 40, seed=300, timing=timing)
    assert cfg.shape == (2100, 64) and E.shape == (2100,)
    assert timing["attempts"] == 2100 * 40 * 64
    for c, R in ((0, 1024), (2, 52)):
        ref = oracle.Run(g, np.full(R, 1.3), seed=300 + c, M=0)
        ref.run(40)
        for slot in (0, R // 2, R - 1):
            j = 1024 * c + slot
            assert np.array_equal(cfg[j], ref.spins[slot]) and E[j] == ref.E[slot], (c, slot)


def test_tts_runs_match_oracle_first_hits():
    """tts.run_instance: every run's first hit (the sweep its ladder first
    reaches the multiplier's ground energy) equals the oracle's, for PT and
    for TAPT with proposal banks every sweep."""
    announce("tts.run_instance: m=3 multiplier, 6 runs x 400 sweeps, PT and TAPT")
    import oracle
    from paper_2509_23043_amd import tts
    m = 3
    g = inputs.multiplier(m, 5 * 7)
    egnd = -3 * m * m - 4 * m * (m - 1)
    betas = inputs.geometric_ladder(6)
    bank = {r: inputs.random_bank(g["n"], 16, seed=50 + r, clamp=g["clamp"]) for r in range(4)}
    for banks in (None, bank):
        hits, dt = tts.run_instance(g, betas, 6, 400, seed=700, target=egnd, banks=banks)
        assert dt > 0
        for k in range(6):
            kw = dict(M=1, target=egnd)
            if banks:
                kw.update(prop_start=1, prop_period=1)
            ref = oracle.Run(g, betas, seed=700 + k, banks=banks, **kw)
            ref.run(400)
            assert hits[k] == ref.first_hit, (k, hits[k], ref.first_hit)


def test_ladder_acceptance_matches_oracle_and_adapts():
    """ladder.measure_acceptance sums the library's swap counters over its
    runs, equal to the oracle's; ladder.adapt on the library evens out the
    acceptance of a linear ladder."""
    announce("adaptive ladder: L=4 counters vs oracle, then 4 rounds on L=6")
    import oracle
    from paper_2509_23043_amd import ladder
    g = inputs.ea_lattice(4, 9)
    b = np.linspace(0.3, 2.5, 8)
    A = ladder.measure_acceptance(g, b, 300, runs=3, seed=40)
    att = np.zeros(7)
    acc = np.zeros(7)
    for k in range(3):
        ref = oracle.Run(g, b, seed=40 + k, M=1)
        ref.run(300)
        att += ref.swap_att[:7]
        acc += ref.swap_acc[:7]
    assert np.array_equal(A, acc / np.maximum(att, 1))
    g6 = inputs.ea_lattice(6, 10)
    b0 = np.linspace(0.2, 3.0, 12)
    b1, hist = ladder.adapt(g6, b0, rounds=4, sweeps=2000, runs=4, seed=7)
    assert hist[-1][1].std() < 0.7 * hist[0][1].std(), (hist[0][1], hist[-1][1])


@pytest.mark.parametrize("R,G,M", [(32, 16, 1), (32, 32, 1), (26, 13, 1), (48, 24, 2), (64, 32, 0)])
def test_multipliers_quad_sweeper(R, G, M):
    """Coarse tilings of sparse graphs (at least 12 slots per workgroup) run
    the four-storages-per-lane sweeper: interleaved storages, padding storages
    when G is not a multiple of 4 (G = 13), six quads per site (G = 24),
    independent chains (M = 0, the bank-generation runs); 8-bit multipliers
    against the oracle."""
    announce(f"quad sweeper: 3 x 8-bit multipliers, R={R} G={G} M={M}")
    import oracle
    betas = inputs.geometric_ladder(R) if M else np.full(R, 1.3)
    egnd = -3 * 64 - 4 * 8 * 7
    ctxs, cases = [], []
    for i, (C, p, q) in enumerate(inputs.semiprimes(8, 3, seed=4700 + R)):
        g = inputs.multiplier(8, C)
        banks = ({r: inputs.random_bank(g["n"], 5, seed=4800 + 32 * i + r, clamp=g["clamp"]) for r in range(0, R - 4, 3)}
                 if M else None)
        kw = dict(M=M, target=egnd)
        if M:
            kw.update(prop_start=2 * M, prop_period=2 * M)
        c = binding.Context(g, betas, seed=4900 + i, **kw)
        for r, b in (banks or {}).items():
            c.propose(r, b)
        ctxs.append(c)
        cases.append((g, banks, kw, 4900 + i))
    bt = binding.Batch(ctxs, replicas_per_wg=G, chunk_sweeps=50, kernel="block")
    assert [d["sweeper"] for d in bt.describe()] == ["csr-quad"], bt.describe()
    bt.sweep(100)
    for c, (g, banks, kw, seed) in zip(ctxs, cases):
        ref = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
        ref.run(100)
        compare(c, ref)
