"""Checkpoint / resume (pt_save, pt_restore) and long ladders, on the GPU.

A resumed chain must equal the uninterrupted oracle chain bit for bit:
spins, energies, every counter, the bank cursors (seen through the proposal
counters after the resume) and the best record."""
import numpy as np
import pytest

from paper_2509_23043_amd import binding, inputs
from tests.gpu_util import announce, compare, make_pair

pytestmark = pytest.mark.gpu


def _banked(seed, **kw):
    g = inputs.ea_lattice(4, 1)
    b = inputs.geometric_ladder(16)
    banks = {r: inputs.random_bank(64, 9, seed=200 + r) for r in range(14)}
    kw = dict(prop_start=4, prop_period=6, target=-90, **kw)
    return g, b, banks, kw


@pytest.mark.parametrize("first,second", [("plain", "batched"), ("batched", "plain"), ("batched", "batched")])
def test_resume_with_proposals_is_bit_identical(first, second):
    announce(f"checkpoint after 50 sweeps ({first}), resume in a fresh context ({second}) for 70 more")
    g, b, banks, kw = _banked(77)
    ctx, ref = make_pair(g, b, seed=77, banks=banks, **kw)

    def run(c, n, how):
        if how == "plain":
            c.sweep(n)
        else:
            bt = binding.Batch([c], replicas_per_wg=6, chunk_sweeps=25)
            bt.sweep(n)
            bt.close()

    run(ctx, 50, first)
    blob = ctx.save()
    ctx2 = binding.Context(g, b, seed=77, **kw)
    for r, bk in banks.items():
        ctx2.propose(r, bk)
    ctx2.restore(blob)
    run(ctx2, 70, second)
    ref.run(120)
    compare(ctx2, ref)
    assert ctx2.counters()["prop_att"].sum() == ref.prop_att.sum() > 0


def test_restore_refuses_mismatches_and_leaves_state():
    announce("checkpoint refused on another seed, other bank sizes and corrupt energies")
    g, b, banks, kw = _banked(5)
    ctx = binding.Context(g, b, seed=5, **kw)
    for r, bk in banks.items():
        ctx.propose(r, bk)
    ctx.sweep(30)
    blob = ctx.save()
    other = binding.Context(g, b, seed=6, **kw)
    for r, bk in banks.items():
        other.propose(r, bk)
    with pytest.raises(binding.TaptError):
        other.restore(blob)
    fewer = binding.Context(g, b, seed=5, **kw)
    for r, bk in banks.items():
        fewer.propose(r, bk[:8])
    with pytest.raises(binding.TaptError):
        fewer.restore(blob)
    # an energy that is not the energy of its spins: refused, state unchanged
    same = binding.Context(g, b, seed=5, **kw)
    for r, bk in banks.items():
        same.propose(r, bk)
    before = same.save()
    bad = bytearray(blob)
    hdr = 72                                      # header bytes before E[0]
    e0 = int.from_bytes(bad[hdr:hdr + 4], "little", signed=True)
    bad[hdr:hdr + 4] = (e0 + 4).to_bytes(4, "little", signed=True)
    with pytest.raises(binding.TaptError):
        same.restore(bytes(bad))
    assert same.save() == before
    same.restore(blob)
    assert same.save() == blob


def test_long_fine_ladder_tables_are_whole():
    """600 slots on a geometric 0.2..3.0 ladder: the swap tables of Eq. 1 hold
    about 5e6 entries together. Every one must reach the device untruncated,
    or swaps that Eq. 1 accepts with nonzero probability would be refused."""
    announce("EA L=4, R=600 geometric ladder, 40 sweeps, plain path; batch refused or equal")
    g = inputs.ea_lattice(4, 3)
    b = inputs.geometric_ladder(600)
    ctx, ref = make_pair(g, b, seed=11)
    ctx.sweep(40)
    ref.run(40)
    compare(ctx, ref)
    assert ref.swap_acc.sum() > 0
    # a batch stages each workgroup's swap tables in LDS; tables this long
    # (about 24500 entries for the hottest pair) do not fit, and the batch
    # must say so rather than run with cut tables
    ctx2, _ = make_pair(g, b, seed=11)
    try:
        bt = binding.Batch([ctx2], chunk_sweeps=20)
        bt.sweep(40)
    except binding.TaptError as e:
        assert e.code == binding.PT_EUNSUPPORTED, e
        return
    compare(ctx2, ref)
