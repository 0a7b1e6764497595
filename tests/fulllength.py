"""Workloads of the full-length parity tests: the benchmark configurations run
to their stated lengths, in the launch configuration the benchmark times.

Proposal banks of the instances that are compared with the oracle are drawn
by the oracle itself: bank entry k of slot r is the state of an independent
chain at beta_r (sweeps_per_cycle 0, the long-run MCMC of Supp. Table S3)
after BANK_SWEEPS sweeps from its own random start. So no input and no
expected value comes from the HIP path. The other instances of a batch carry
seeded iid banks; they only fill the launch.

Expected results of the 10^5-sweep runs (the 8^3 and the mixed-size
spin-glass batches) are stored under
tests/golden/ by tests/golden/make_fulllength.py, which calls only the oracle
and this module; the factorization batch (10^4 sweeps) is short
enough for the oracle to run beside the test on the host's cores.
"""
from __future__ import annotations

import base64
import json
import os
import time

import numpy as np

from paper_2509_23043_amd import inputs

from paper_2509_23043_amd.workloads import EA_L8, EA_MIXED, MULT8, ea_cases, fact_cases, run_kwargs  # noqa: F401

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BANK_SWEEPS = 20
BANK_SEED = 7_000_000

# instances compared with the oracle (batch order)
COMPARED = {"ea_l8_x64": (0, 9, 18, 27, 36, 45, 54, 63), "ea_mixed_x40": (0, 8, 16, 24, 32)}


def _bank_job(args):
    """Bank of one slot: B independent oracle chains at that slot's beta."""
    g, beta, B, seed = args
    import oracle
    run = oracle.Run(g, np.full(B, beta), seed=seed, M=0, check_energy=False)
    run.run(BANK_SWEEPS)
    return run.spins.copy()


def oracle_banks(cases, cfg, pool=None):
    """{case k: {slot r: int8 [B, n]}} for the given cases, one oracle job per
    (case, slot), seeded by (case, slot)."""
    jobs, keys = [], []
    for c in cases:
        for r in range(c["n_prop"]):
            jobs.append((c["g"], float(c["betas"][r]), cfg["B"], BANK_SEED + 1000 * c["k"] + r))
            keys.append((c["k"], r))
    res = pool.map(_bank_job, jobs) if pool is not None else [_bank_job(j) for j in jobs]
    out = {}
    for (k, r), b in zip(keys, res):
        out.setdefault(k, {})[r] = b
    return out


def filler_banks(case, cfg):
    """Seeded iid banks of an instance that is not compared (launch filler)."""
    g = case["g"]
    return {r: inputs.random_bank(g["n"], cfg["B"], seed=BANK_SEED + 1000 * case["k"] + r, clamp=g.get("clamp"))
            for r in range(case["n_prop"])}


def _oracle_job(args):
    """Full run of one case on the oracle; the result as plain arrays."""
    g, betas, seed, banks, kw, sweeps = args
    import oracle
    t0 = time.perf_counter()
    run = oracle.Run(g, betas, seed=seed, banks=banks, **kw)
    run.run(sweeps)
    return dict(t=run.t, E=run.E.copy(), spins=run.spins.copy(), swap_att=run.swap_att.copy(),
                swap_acc=run.swap_acc.copy(), prop_att=run.prop_att.copy(), prop_acc=run.prop_acc.copy(),
                flips=run.flips.copy(), best=run.best, best_t=run.best_t, best_slot=run.best_slot,
                first_hit=run.first_hit, best_spins=run.best_spins.copy(), energy_mismatch=run.energy_mismatch,
                seconds=time.perf_counter() - t0)


def run_oracle(cases, cfg, banks, pool=None, check_energy=True):
    jobs = [(c["g"], c["betas"], c["seed"], banks[c["k"]], dict(run_kwargs(cfg, c), check_energy=check_energy),
             cfg["sweeps"]) for c in cases]
    return pool.map(_oracle_job, jobs) if pool is not None else [_oracle_job(j) for j in jobs]


# ---- golden files: spins as packed bits, counters as lists ----

def _pack(spins):
    return base64.b64encode(np.packbits(np.asarray(spins) > 0, axis=None).tobytes()).decode()


def _unpack(s, shape):
    bits = np.unpackbits(np.frombuffer(base64.b64decode(s), np.uint8))[:int(np.prod(shape))]
    return (bits.astype(np.int8) * 2 - 1).reshape(shape)


def to_json(res):
    d = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in res.items()}
    d["spins"] = _pack(res["spins"])
    d["best_spins"] = _pack(res["best_spins"])
    d["R"], d["n"] = int(res["spins"].shape[0]), int(res["spins"].shape[1])
    return d


def from_json(d):
    R, n = d["R"], d["n"]
    out = dict(d)
    out["spins"] = _unpack(d["spins"], (R, n))
    out["best_spins"] = _unpack(d["best_spins"], (n,))
    for k in ("E", "swap_att", "swap_acc", "prop_att", "prop_acc", "flips"):
        out[k] = np.asarray(d[k], np.int64 if k == "E" else np.uint64)
    return out


def golden_path(cfg):
    return os.path.join(GOLDEN, f"fulllength_{cfg['name']}.json")


def load_golden(cfg):
    d = json.load(open(golden_path(cfg)))
    return d, {int(k): from_json(v) for k, v in d["results"].items()}


def compare_result(ctx, ref, label=""):
    """Element-by-element comparison of a context with a stored oracle result."""
    spins, t = ctx.state()
    R = spins.shape[0]
    assert t == ref["t"], (label, t, ref["t"])
    E = ctx.energies()
    bad = np.nonzero(E != ref["E"])[0]
    assert bad.size == 0, (label, "energies differ at slots", bad[:8], E[bad[:8]], ref["E"][bad[:8]])
    rows = np.nonzero(np.any(spins != ref["spins"], axis=1))[0]
    assert rows.size == 0, (label, "spins differ in slots", rows[:8])
    c = ctx.counters()
    for key in ("swap_att", "swap_acc"):
        assert np.array_equal(c[key], ref[key][:R - 1]), (label, key)
    for key in ("prop_att", "prop_acc", "flips"):
        assert np.array_equal(c[key], ref[key]), (label, key)
    s = ctx.summary()
    assert (s["best"], s["best_t"], s["best_slot"], s["first_hit"]) == \
        (ref["best"], ref["best_t"], ref["best_slot"], ref["first_hit"]), (label, s, ref["best"], ref["best_t"])
    assert np.array_equal(s["best_spins"], ref["best_spins"]), (label, "best configuration")
