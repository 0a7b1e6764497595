"""Host logic of the bank-generation helpers (no GPU calls)."""


def test_batches_halve_until_the_runtime_accepts():
    """banks._batches covers every context once, in order, halving a group the
    runtime refuses (here: groups above 3 contexts) down to one context."""
    from paper_2509_23043_amd import banks, binding

    def make(group):
        if len(group) > 3:
            raise binding.TaptError(7, "too many workgroups")
        return tuple(group)

    ctxs = list(range(10))
    out = list(banks._batches(ctxs, make))
    assert [c for g, _ in out for c in g] == ctxs
    assert all(len(g) <= 3 and bt == tuple(g) for g, bt in out)

    def refuse(group):
        raise binding.TaptError(7, "never")

    try:
        list(banks._batches([1, 2], refuse))
        assert False, "a single refused context must raise"
    except binding.TaptError:
        pass
