"""Host logic of the autotuner: candidate set, cache key, cache round trip
(timing replaced by a stub, no GPU)."""
import json
import types

from paper_2509_23043_amd import autotune


def _ctx(kind, L, n, R, pm=False):
    return types.SimpleNamespace(kind=kind, L=L, n=n, R=R, nfree=n, pm=pm, close=lambda: None)


def test_candidates_cover_caps_and_threads():
    c = autotune.candidates([_ctx("lattice", 8, 512, 32)])
    assert (8, 1, "block") in c and (32, 4, "block") in c and (64, 2, "block") in c and (8, 1, "wave") in c
    assert all(rpt <= G for G, rpt, _ in c)
    assert not any(k == "pm" for _, _, k in c)
    c3 = autotune.candidates([_ctx("lattice", 8, 512, 32, pm=True)])
    assert (8, 1, "pm") in c3 and (16, 1, "pm") in c3 and (8, 1, "pm1") in c3 and (16, 1, "pm1") not in c3
    c2 = autotune.candidates([_ctx("lattice", 4, 64, 3)])
    assert max(G for G, _, _ in c2) <= 6 and all(k == "block" for _, _, k in c2)


def test_batch_key_is_a_multiset(monkeypatch):
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    a = [_ctx("lattice", 8, 512, 32), _ctx("csr", 0, 200, 32), _ctx("lattice", 8, 512, 32)]
    b = [a[1], a[0], a[2]]
    assert autotune.batch_key(a) == autotune.batch_key(b)
    assert "lattice:8:R32x2" in autotune.batch_key(a)
    assert autotune.batch_key(a) != autotune.batch_key(a[:2])


def test_tune_picks_fastest_and_caches(monkeypatch, tmp_path):
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    rates = {(1, 8, 1, "block"): 100.0, (2, 8, 1, "block"): 150.0, (1, 16, 2, "block"): 120.0}
    calls = []

    def fake_time(ctxs, G, rpt, kern, warm, timed):
        M = ctxs[0].M
        calls.append((M, G, rpt, kern))
        return rates.get((M, G, rpt, kern))

    monkeypatch.setattr(autotune, "time_tiling", fake_time)

    def make(M):
        c = _ctx("lattice", 8, 512, 32)
        c.M = M
        return [c]

    monkeypatch.setattr(autotune, "mean_best_energy", lambda make, M, tiling, sweeps: {1: -100.0, 2: -101.0}[M])
    cache = str(tmp_path / "tune.json")
    r = autotune.tune(make, Ms=(1, 2), cache=cache)
    assert (r["M"], r["replicas_per_wg"], r["replicas_per_thread"]) == (2, 8, 1)
    assert not r["cached"] and len(r["scan"]) == 3
    n_calls = len(calls)
    r2 = autotune.tune(make, Ms=(1, 2), cache=cache)
    assert r2["cached"] and r2["M"] == 2 and len(calls) == n_calls
    assert r["key"] in json.load(open(cache))


def test_faster_M_that_samples_worse_is_refused(monkeypatch):
    """M changes the chain: a faster M whose held-out runs end at a higher
    mean best energy than the reference M's loses to the reference."""
    monkeypatch.setattr(autotune, "arch", lambda: "gfx950")
    rates = {(1, 8, 1, "block"): 100.0, (2, 8, 1, "block"): 150.0}
    monkeypatch.setattr(autotune, "time_tiling", lambda ctxs, G, rpt, kern, warm, timed:
                        rates.get((ctxs[0].M, G, rpt, kern)))
    seen = []

    def quality(make, M, tiling, sweeps):
        seen.append((M, tiling["replicas_per_wg"], sweeps))
        return {1: -120.0, 2: -110.0}[M]

    monkeypatch.setattr(autotune, "mean_best_energy", quality)

    def make(M, seed_offset=0):
        c = _ctx("lattice", 8, 512, 32)
        c.M = M
        return [c]

    r = autotune.tune(make, Ms=(1, 2), quality_sweeps=500)
    assert r["M"] == 1 and r["replicas_per_wg"] == 8
    assert sorted(seen) == [(1, 8, 500), (2, 8, 500)]
    assert r["quality"] == {"1": -120.0, "2": -110.0}
