"""Serving (continuous batching): every request's result equals the same
chain run alone and the oracle's, whatever else shares the device."""
import time

import numpy as np
import pytest

import oracle
from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _problems():
    """(name, graph, betas, banks, opts, target) of a small mixed pool."""
    out = []
    for k, L in enumerate((4, 6, 8)):
        g = inputs.ea_lattice(L, 600 + k)
        b = inputs.geometric_ladder(8 + 4 * k)
        banks = {r: inputs.random_bank(g["n"], 6, seed=900 + 10 * k + r) for r in range(0, len(b) - 2, 3)}
        out.append((f"ea{L}", g, b, banks, dict(prop_start=10, prop_period=10), -int(1.2 * g["n"])))
    m = 4
    g = inputs.multiplier(m, 11 * 13)
    b = inputs.geometric_ladder(10)
    banks = {r: inputs.random_bank(g["n"], 4, seed=950 + r, clamp=g["clamp"]) for r in range(6)}
    out.append(("fact4", g, b, banks, dict(prop_start=20, prop_period=20), -3 * m * m - 4 * m * (m - 1)))
    return out


def _register(srv, pool):
    ids, ctxs = [], []
    for name, g, b, banks, kw, _ in pool:
        ctx = binding.Context(g, b, seed=0, **kw)
        for r, bank in banks.items():
            ctx.propose(r, bank)
        ids.append(srv.register(ctx))
        ctxs.append(ctx)
    return ids, ctxs


def _drain(srv, n, timeout=120.0):
    res = {}
    t_end = time.time() + timeout
    while len(res) < n:
        assert time.time() < t_end, "serving did not finish"
        for r in srv.poll(64, wait_ms=200):
            res[r["id"]] = r
    return res


def _requests():
    """(problem index, seed, cap, with target) of a mixed request list."""
    rq = []
    for j in range(14):
        p = j % 4
        rq.append((p, 7000 + j, 300 + 170 * (j % 5), j % 3 != 2))
    return rq


def _key(r):
    return (r["status"], r["hit"], r["first_hit"], r["best_energy"], r["best_slot"], r["best_t"], r["sweeps"])


@pytest.mark.parametrize("pipeline", [False, True])
def test_serving_alone_vs_mix_and_oracle(pipeline):
    """The mix one round at a time and pipelined (each round enqueued before
    the last is retired: finished requests ride along as no-ops)."""
    announce(f"serving: 14 mixed requests (EA L=4,6,8 + 4-bit factorization), alone vs mix vs oracle, "
             f"pipeline={pipeline}")
    pool = _problems()
    rqs = _requests()
    K = 100
    # the mix: everything submitted at once
    srv = binding.Server(chunk_sweeps=K, pipeline=pipeline)
    ids, _ctxs = _register(srv, pool)
    sub = {}
    for j, (p, seed, cap, with_t) in enumerate(rqs):
        sub[srv.submit(ids[p], seed, cap, target=pool[p][5] if with_t else None, user_tag=j)] = j
    mix = _drain(srv, len(rqs))
    st = srv.stats()
    srv.stop()
    assert st["completed"] == len(rqs) and st["rejected"] == 0
    assert st["peak_active"] > 1
    # lattices of L = 4, the row kernel's lattices and the multipliers run in lanes of their own
    assert st["peak_lanes"] >= 2, st
    by_tag = {r["user_tag"]: r for r in mix.values()}
    # three of them alone, each on a fresh server
    for j in (0, 5, 11):
        p, seed, cap, with_t = rqs[j]
        srv = binding.Server(chunk_sweeps=K)
        ids1, _c = _register(srv, pool)
        srv.submit(ids1[p], seed, cap, target=pool[p][5] if with_t else None, user_tag=j)
        alone = list(_drain(srv, 1).values())[0]
        srv.stop()
        assert _key(alone) == _key(by_tag[j]), (j, alone, by_tag[j])
        assert np.array_equal(alone["best_spins"], by_tag[j]["best_spins"])
    # every result against the oracle run for the same number of sweeps
    for j, (p, seed, cap, with_t) in enumerate(rqs):
        r = by_tag[j]
        name, g, b, banks, kw, target = pool[p]
        assert r["status"] == 0
        if with_t and r["hit"]:
            assert r["sweeps"] == min(cap, -(-r["first_hit"] // K) * K)
        else:
            assert r["sweeps"] == cap
        ref = oracle.Run(g, b, seed=seed, banks=banks, target=target if with_t else None, **kw)
        ref.run(r["sweeps"])
        assert r["best_energy"] == ref.best and r["best_t"] == ref.best_t and r["best_slot"] == ref.best_slot
        assert r["first_hit"] == ref.first_hit
        assert np.array_equal(r["best_spins"], ref.best_spins), name


def test_serving_memory_admission():
    announce("serving: memory budget admits two requests at a time")
    pool = _problems()[:2]
    K = 50
    srv = binding.Server(chunk_sweeps=K, mem_budget=1)   # too small for any request
    ids, _c = _register(srv, pool)
    srv.submit(ids[0], 1, 100)
    r = _drain(srv, 1)
    srv.stop()
    assert list(r.values())[0]["status"] == binding.PT_ENOMEM
    # the state bytes of one request, then a budget of two and a half
    srv = binding.Server(chunk_sweeps=K)
    ids, _c = _register(srv, pool)
    srv.submit(ids[0], 1, 50)
    _drain(srv, 1)
    one = srv.stats()["mem_peak"]
    srv.stop()
    assert one > 0
    srv = binding.Server(chunk_sweeps=K, mem_budget=2 * one + one // 2)
    ids, _c = _register(srv, pool)
    for j in range(6):
        srv.submit(ids[0], 100 + j, 150 + 50 * j)
    res = _drain(srv, 6)
    st = srv.stats()
    srv.stop()
    assert st["peak_active"] <= 2 and st["completed"] == 6
    for r in res.values():
        assert r["status"] == 0 and r["sweeps"] == 150 + 50 * (r["id"] - 1)
        assert r["t_admit"] >= r["t_submit"] and r["t_done"] >= r["t_admit"]


def test_serving_lanes_overflow():
    """More requests of one kind than one co-resident launch holds: 40 +-J
    L = 6 lattices of 64 slots (8 workgroups of the row kernel each) are
    admitted together and run in several lanes per round, pipelined; every
    result equals the oracle's."""
    announce("serving: 40 requests of L=6 R=64 over several launch lanes, 3 checked against the oracle")
    g = inputs.ea_lattice(6, 640)
    b = inputs.geometric_ladder(64)
    banks = {r: inputs.random_bank(g["n"], 4, seed=960 + r) for r in range(0, 60, 4)}
    kw = dict(prop_start=20, prop_period=20)
    K, cap = 50, 150
    srv = binding.Server(chunk_sweeps=K, pipeline=True)
    ctx = binding.Context(g, b, seed=0, **kw)
    for r, bank in banks.items():
        ctx.propose(r, bank)
    pid = srv.register(ctx)
    for j in range(40):
        srv.submit(pid, 8000 + j, cap, user_tag=j)
    res = {r["user_tag"]: r for r in _drain(srv, 40).values()}
    st = srv.stats()
    srv.stop()
    assert st["completed"] == 40 and st["rejected"] == 0
    assert st["peak_active"] > 32 and st["peak_lanes"] >= 2, st
    for j in (0, 21, 39):
        r = res[j]
        assert r["status"] == 0 and r["sweeps"] == cap
        ref = oracle.Run(g, b, seed=8000 + j, banks=banks, **kw)
        ref.run(cap)
        assert r["best_energy"] == ref.best and r["best_t"] == ref.best_t and r["best_slot"] == ref.best_slot
        assert np.array_equal(r["best_spins"], ref.best_spins), j


@pytest.mark.parametrize("pipeline", [False, True])
def test_serving_sparse_lanes_by_pace(pipeline):
    """Sparse requests of two paces (6-bit multipliers: one rank group per
    colour class; 12-bit: two) beyond one co-resident launch (64 slots each,
    8 workgroups): admitted together into mixed lanes, then refilled pace by
    pace (pipelined: while a round over the old lanes runs). Every result
    equals the oracle's for the sweeps it ran."""
    announce(f"serving: 24 + 24 multiplier requests (m = 6 and 12, R = 64) over several lanes, pipeline={pipeline}")
    K, cap = 50, 100
    probs = []
    for m in (6, 12):
        C, _p, _q = inputs.semiprimes(m, 1, seed=7700 + m)[0]
        g = inputs.multiplier(m, C)
        b = inputs.geometric_ladder(64)
        banks = {r: inputs.random_bank(g["n"], 4, seed=7800 + 10 * m + r, clamp=g["clamp"]) for r in range(0, 48, 6)}
        probs.append((g, b, banks, dict(prop_start=25, prop_period=25)))
    srv = binding.Server(chunk_sweeps=K, pipeline=pipeline)
    pids = []
    for g, b, banks, kw in probs:
        ctx = binding.Context(g, b, seed=0, **kw)
        for r, bank in banks.items():
            ctx.propose(r, bank)
        pids.append(srv.register(ctx))
    for j in range(48):
        srv.submit(pids[j % 2], 9100 + j, cap, user_tag=j)
    res = {r["user_tag"]: r for r in _drain(srv, 48).values()}
    st = srv.stats()
    srv.stop()
    assert st["completed"] == 48 and st["rejected"] == 0 and st["peak_lanes"] >= 2, st
    for j in (0, 1, 46, 47):
        g, b, banks, kw = probs[j % 2]
        r = res[j]
        assert r["status"] == 0 and r["sweeps"] == cap
        ref = oracle.Run(g, b, seed=9100 + j, banks=banks, **kw)
        ref.run(cap)
        assert r["best_energy"] == ref.best and r["best_t"] == ref.best_t and r["best_slot"] == ref.best_slot
        assert np.array_equal(r["best_spins"], ref.best_spins), j
