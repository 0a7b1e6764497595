"""The benchmark workloads as seeded problem descriptions.

Shared by bench.py and the full-length parity tests, so that both run the same
instances, ladders, seeds, schedules and targets. Like ``inputs``, this module
only describes problems: it holds none of the sampler's arithmetic.

- ``EA_L8``: 64 synthetic 3D EA +-J instances, L=8 (512 spins), R=32 geometric
  0.2..3.0, Metropolis, M=1, 10^5 sweeps, 256-entry banks on the 30 hottest
  slots, proposals every 100 sweeps.
- ``EA_MIXED``: EA +-J L in {6, 8, 10, 12, 16} x 8 instances with ladders of
  24/30/36/42/48 slots, M=1, 10^5 sweeps, banks on all but the two coldest
  slots, proposals every 50 sweeps; one persistent launch under the
  autotuner's tiling.
- ``MULT8``: 64 distinct products of two distinct primes in [128, 256) as 8x8-bit
  array multipliers (200 spins, 176 free, DSATUR colors), R=32, M=1, banks on
  the round(13 R / 18) = 23 hottest slots (the paper's 13 of 18), proposals
  every 100 sweeps, target the ground energy -3m^2 - 4m(m-1).

Spin-glass targets (first-hit bookkeeping only): E <= -1.70 N on the energy
grid of 4.
"""
from __future__ import annotations

from . import inputs

EA_L8 = dict(name="ea_l8_x64", sizes=((8, 32),), per_size=64, inst_seed=2000, run_seed=3000, B=256, period=100,
            sweeps=100_000, chunk=10_000)
EA_MIXED = dict(name="ea_mixed_x40", sizes=((6, 24), (8, 30), (10, 36), (12, 42), (16, 48)), per_size=8, inst_seed=3000,
            run_seed=3500, B=256, period=50, sweeps=100_000, chunk=10_000)
MULT8 = dict(name="mult8x8_x64", m=8, count=64, prod_seed=4000, run_seed=4500, R=32, n_prop=23, B=256, period=100,
            sweeps=10_000, chunk=10_000, solve_cap=100_000)


def ea_target(n):
    """E <= -1.70 N rounded to the energy grid of 4 (towards zero)."""
    return -4 * int(1.70 * n / 4)


def ea_cases(cfg):
    """Every instance of a spin-glass workload, in batch order: dicts with
    k, g (problem), betas, seed (run seed), target, n_prop (banked slots)."""
    out = []
    k = 0
    for L, R in cfg["sizes"]:
        betas = inputs.geometric_ladder(R)
        for i in range(cfg["per_size"]):
            inst = cfg["inst_seed"] + i if len(cfg["sizes"]) == 1 else cfg["inst_seed"] + 100 * L + i
            g = inputs.ea_lattice(L, inst)
            out.append(dict(k=k, g=g, betas=betas, seed=cfg["run_seed"] + k, target=ea_target(g["n"]),
                            n_prop=R - 2, L=L))
            k += 1
    return out


def fact_cases(cfg=MULT8):
    """Every product of the factorization workload: dicts as ea_cases plus
    C, p, q and m."""
    m = cfg["m"]
    egnd = -3 * m * m - 4 * m * (m - 1)
    betas = inputs.geometric_ladder(cfg["R"])
    picks, seen = [], set()
    for C, p, q in inputs.semiprimes(m, 8 * cfg["count"], seed=cfg["prod_seed"]):
        if C not in seen and len(picks) < cfg["count"]:
            seen.add(C)
            picks.append((C, p, q))
    out = []
    for k, (C, p, q) in enumerate(picks):
        out.append(dict(k=k, g=inputs.multiplier(m, C), betas=betas, seed=cfg["run_seed"] + k, target=egnd,
                        n_prop=cfg["n_prop"], C=C, p=p, q=q, m=m))
    return out


def run_kwargs(cfg, case):
    """Options of one run: M=1, the workload's proposal period from sweep
    `period` on, the case's first-hit target."""
    return dict(M=1, prop_start=cfg["period"], prop_period=cfg["period"], target=case["target"])
