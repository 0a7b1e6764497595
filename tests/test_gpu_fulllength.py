"""Full-length parity: the benchmark workloads run to their stated lengths, in
the launch configuration the benchmark times, compared with the oracle
element by element (spins and energies by slot, every counter, the best
record and the first hit).

- 64 EA +-J L=8 instances, R=32, 10^5 sweeps in 10^4-sweep launches
  of the +-J kernel with one slot per wavefront and 8 slots per workgroup;
  8 instances compared with stored oracle runs of the same length.
- the 40-instance mixed-size batch (L = 6..16, R = 24..48), 10^5
  sweeps in one launch sequence under the autotuner's tiling (and the
  runtime's automatic tiling); one instance per size compared with stored
  oracle runs.
- 64 8-bit factorization instances, R=32, 10^4 sweeps under the
  autotuner's tiling; every instance compared with an oracle run made beside
  the test on the host's cores.

The stored runs are written by tests/golden/make_fulllength.py (oracle only).
"""
import multiprocessing as mp
import os
import time

import numpy as np
import pytest

from paper_2509_23043_amd import autotune, binding
from tests import fulllength as F
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _pool():
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    return mp.get_context("spawn").Pool(workers)


def _all_banks(cases, cfg, oracle_banks):
    """Oracle banks for the compared instances, seeded iid ones elsewhere."""
    return {c["k"]: oracle_banks.get(c["k"]) or F.filler_banks(c, cfg) for c in cases}


def _contexts(cases, cfg, banks):
    ctxs = []
    for c in cases:
        ctx = binding.Context(c["g"], c["betas"], seed=c["seed"], **F.run_kwargs(cfg, c))
        for r, b in (banks or {}).get(c["k"], {}).items():
            ctx.propose(r, b)
        ctxs.append(ctx)
    return ctxs


def _tuned(cases, cfg):
    """The autotuner's tiling for this batch (M fixed at the workload's 1),
    timed on scratch contexts without banks."""
    def make(M):
        return _contexts(cases, cfg, None)
    res = autotune.tune(make, Ms=(1,), warm=100, timed=400)
    return res["replicas_per_wg"], res["replicas_per_thread"], res["kernel"]


def _run_and_compare(cases, cfg, banks, refs, tiling, label):
    G, rpt, kern = tiling
    announce(f"{label}: {len(cases)} instances, tiling G={G} rpt={rpt} kernel={kern}, "
             f"{cfg['sweeps']} sweeps in launches of {cfg['chunk']}")
    ctxs = _contexts(cases, cfg, banks)
    bt = binding.Batch(ctxs, replicas_per_wg=G, replicas_per_thread=rpt, chunk_sweeps=cfg["chunk"], kernel=kern)
    t0 = time.perf_counter()
    bt.sweep(cfg["sweeps"])
    dt = time.perf_counter() - t0
    announce(f"{label}: GPU run {dt:.2f} s")
    for k, ref in refs.items():
        F.compare_result(ctxs[k], ref, f"{label} instance {k}")
    bt.close()
    for c in ctxs:
        c.close()


def test_ea_l8_x64_full_length_bench_launch():
    cfg = F.EA_L8
    golden, refs = F.load_golden(cfg)
    assert golden["sweeps"] == cfg["sweeps"] == 100_000 and len(refs) == 8
    cases = F.ea_cases(cfg)
    announce("8^3 x 64: oracle banks of the 8 compared instances")
    with _pool() as pool:
        banks = _all_banks(cases, cfg, F.oracle_banks([c for c in cases if c["k"] in refs], cfg, pool))
    _run_and_compare(cases, cfg, banks, refs, (8, 1, "pm1"), "8^3 x 64")


def test_ea_mixed_x40_full_length_tuned_launch():
    cfg = F.EA_MIXED
    golden, refs = F.load_golden(cfg)
    assert golden["sweeps"] == cfg["sweeps"] == 100_000 and len(refs) == 5
    cases = F.ea_cases(cfg)
    assert sorted({cases[k]["L"] for k in refs}) == [6, 8, 10, 12, 16]
    announce("mixed sizes x 40: oracle banks of the 5 compared instances")
    with _pool() as pool:
        banks = _all_banks(cases, cfg, F.oracle_banks([c for c in cases if c["k"] in refs], cfg, pool))
    tuned = _tuned(cases, cfg)
    _run_and_compare(cases, cfg, banks, refs, tuned, "mixed sizes (autotuned)")
    if tuned != (0, 0, "auto"):
        _run_and_compare(cases, cfg, banks, refs, (0, 0, "auto"), "mixed sizes (automatic tiling)")


def test_mult8x8_x64_full_length_all_products():
    cfg = F.MULT8
    cases = F.fact_cases(cfg)
    assert len(cases) == 64 and len({c["C"] for c in cases}) == 64
    announce("8x8-bit multipliers x 64: oracle banks and 10^4-sweep oracle runs of all 64 products")
    t0 = time.perf_counter()
    with _pool() as pool:
        banks = F.oracle_banks(cases, cfg, pool)
        res = F.run_oracle(cases, cfg, banks, pool)
    announce(f"8x8-bit multipliers x 64: oracle {time.perf_counter() - t0:.1f} s, "
             f"{sum(r['first_hit'] >= 0 for r in res)} of 64 reached the ground energy")
    for r in res:
        assert r["energy_mismatch"] == 0
    refs = {c["k"]: r for c, r in zip(cases, res)}
    # a ground state found by the oracle factors the product
    from paper_2509_23043_amd import inputs
    for c, r in zip(cases, res):
        if r["first_hit"] >= 0:
            assert r["best"] == c["target"]
            A = inputs.bits_to_int(r["best_spins"], c["g"]["a_idx"])
            B = inputs.bits_to_int(r["best_spins"], c["g"]["b_idx"])
            assert A * B == c["C"] and {A, B} == {c["p"], c["q"]}, (c["C"], A, B)
    tuned = _tuned(cases, cfg)
    _run_and_compare(cases, cfg, banks, refs, tuned, "8x8-bit multipliers (autotuned)")
    assert np.all([refs[k]["t"] == cfg["sweeps"] for k in refs])
