"""pt_batch_run_static: the batched run that allocates no device memory must
give what pt_batch_create + pt_batch_sweep give, bit for bit, on two calls in
a row (the second on a smaller batch), and refuse a launch larger than its
static scratch."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _state(c):
    s, t = c.state()
    return s, t, c.energies(), c.counters(), c.summary()


def _same(a, b):
    sa, ta, ea, ca, ua = _state(a)
    sb, tb, eb, cb, ub = _state(b)
    assert ta == tb
    assert np.array_equal(sa, sb)
    assert np.array_equal(ea, eb)
    for k in ca:
        assert np.array_equal(ca[k], cb[k]), k
    for k in ("best", "best_t", "best_slot", "first_hit"):
        assert ua[k] == ub[k], k
    assert np.array_equal(ua["best_spins"], ub["best_spins"])


def _pairs(specs):
    out = []
    for g, betas, seed, banks, kw in specs:
        pair = []
        for _ in range(2):
            c = binding.Context(g, betas, seed=seed, **kw)
            for r, b in (banks or {}).items():
                c.propose(r, b)
            pair.append(c)
        out.append(pair)
    return out


def test_static_run_matches_batch_twice_then_smaller():
    announce("pt_batch_run_static vs pt_batch_sweep: 6 x L=8 R=32 (pm1, G=8), then 3 mixed contexts")
    betas = inputs.geometric_ladder(32)
    specs = []
    for i in range(6):
        g = inputs.ea_lattice(8, 4300 + i)
        banks = {r: inputs.random_bank(512, 6, seed=9300 + 40 * i + r) for r in range(0, 30, 4)}
        specs.append((g, betas, 600 + i, banks, dict(prop_start=10, prop_period=10, target=-700)))
    pairs = _pairs(specs)
    ref = binding.Batch([p[0] for p in pairs], replicas_per_wg=8, chunk_sweeps=50, kernel="pm1")
    ref.sweep(120)
    binding.run_static([p[1] for p in pairs], 120, replicas_per_wg=8, chunk_sweeps=50, kernel="pm1")
    for a, b in pairs:
        _same(a, b)
    # second call on the same contexts: continues from where the first ended
    ref.sweep(70)
    binding.run_static([p[1] for p in pairs], 70, replicas_per_wg=8, chunk_sweeps=50, kernel="pm1")
    for a, b in pairs:
        _same(a, b)
    ref.close()
    # a smaller batch of other shapes right after (automatic tiling, mixed kernel)
    m4 = inputs.multiplier(4, 11 * 13)
    small = [(inputs.ea_lattice(6, 77), inputs.geometric_ladder(10), 41, None, {}),
             (m4, inputs.geometric_ladder(8), 42, {0: inputs.random_bank(m4["n"], 3, seed=5, clamp=m4["clamp"])},
              dict(prop_start=5, prop_period=5))]
    pairs2 = _pairs(small)
    ref2 = binding.Batch([p[0] for p in pairs2], chunk_sweeps=40)
    ref2.sweep(90)
    binding.run_static([p[1] for p in pairs2], 90, chunk_sweeps=40)
    for a, b in pairs2:
        _same(a, b)
    ref2.close()


def test_static_run_refuses_oversized_launch():
    announce("pt_batch_run_static refuses a launch larger than its scratch")
    # 80 8^3 ladders of 1024 independent chains on the +-J kernel need
    # 80 x 1024 x 512 B of per-slot snapshots alone (40 MiB), more than the
    # scratch holds
    g = inputs.ea_lattice(8, 1)
    ctxs = [binding.Context(g, np.full(1024, 0.7), seed=k, M=0) for k in range(80)]
    with pytest.raises(binding.TaptError) as e:
        binding.run_static(ctxs, 2, replicas_per_wg=8, kernel="pm1")
    assert e.value.code == binding.PT_ENOMEM, e.value
