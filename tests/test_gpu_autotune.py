"""Autotuner on the GPU: its choice runs the oracle's chain bit for bit, for
the M it picked, and the tiling it picked gives the same chain as any other."""
import pytest

import oracle
from paper_2509_23043_amd import autotune, binding, inputs
from tests.gpu_util import announce, compare

pytestmark = pytest.mark.gpu


def _cases():
    out = []
    for k, (L, R) in enumerate(((6, 12), (8, 16))):
        g = inputs.ea_lattice(L, 70 + k)
        banks = {r: inputs.random_bank(g["n"], 4, seed=700 + 20 * k + r) for r in range(0, R - 2, 4)}
        out.append((g, inputs.geometric_ladder(R), banks, 500 + k))
    g = inputs.multiplier(4, 11 * 13)
    out.append((g, inputs.geometric_ladder(10), None, 520))
    return out


def _make(M, seed_offset=0):
    ctxs = []
    for g, b, banks, seed in _cases():
        c = binding.Context(g, b, seed=seed + seed_offset, M=M, prop_start=20, prop_period=20)
        for r, bank in (banks or {}).items():
            c.propose(r, bank)
        ctxs.append(c)
    return ctxs


def test_autotune_choice_is_result_invariant(tmp_path):
    announce("autotune over tilings and M in {1, 2} on a mixed batch; chosen vs default vs oracle")
    res = autotune.tune(_make, Ms=(1, 2), cache=str(tmp_path / "t.json"), warm=40, timed=80)
    assert res["scan"] and not res["cached"]
    M = res["M"]
    tuned = _make(M)
    bt = binding.Batch(tuned, replicas_per_wg=res["replicas_per_wg"],
                       replicas_per_thread=res["replicas_per_thread"], chunk_sweeps=60)
    bt.sweep(120)
    default = _make(M)
    bt2 = binding.Batch(default, chunk_sweeps=35)
    bt2.sweep(120)
    for c1, c2, (g, b, banks, seed) in zip(tuned, default, _cases()):
        ref = oracle.Run(g, b, seed=seed, banks=banks, M=M, prop_start=20, prop_period=20)
        ref.run(120)
        compare(c1, ref)
        compare(c2, ref)
    again = autotune.tune(_make, Ms=(1, 2), cache=str(tmp_path / "t.json"))
    assert again["cached"] and again["M"] == M
