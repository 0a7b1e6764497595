"""Write the expected results of the full-length parity tests.

Runs the CPU oracle (and nothing else) on the compared instances of the
spin-glass workloads at their stated lengths (10^5 sweeps, M=1, banks drawn by
the oracle's own independent chains) and stores every output the GPU tests
compare: final spins and energies by slot, swap, proposal and flip counters,
the best record and the first hit. One oracle process per instance, longest
first.

    python tests/golden/make_fulllength.py [--workers N] [ea_l8_x64 ea_mixed_x40]
"""
import argparse
import json
import multiprocessing as mp
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from tests import fulllength as F  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=len(os.sched_getaffinity(0)))
    ap.add_argument("cfgs", nargs="*", default=["ea_l8_x64", "ea_mixed_x40"])
    args = ap.parse_args()
    cfgs = {"ea_l8_x64": F.EA_L8, "ea_mixed_x40": F.EA_MIXED}
    todo = []
    for name in args.cfgs:
        cfg = cfgs[name]
        cases = [c for c in F.ea_cases(cfg) if c["k"] in F.COMPARED[name]]
        todo.append((cfg, cases))
    ctx = mp.get_context("spawn")
    with ctx.Pool(args.workers) as pool:
        jobs = []
        for cfg, cases in todo:
            t0 = time.perf_counter()
            banks = F.oracle_banks(cases, cfg, pool)
            print(f"{cfg['name']}: banks of {len(cases)} instances in {time.perf_counter() - t0:.1f} s", flush=True)
            for c in cases:
                jobs.append((cfg, c, banks[c["k"]]))
        # longest runs first
        jobs.sort(key=lambda j: -len(j[1]["betas"]) * j[1]["g"]["n"])
        t0 = time.perf_counter()
        pending = [(cfg, c, pool.apply_async(F._oracle_job, ((c["g"], c["betas"], c["seed"], b,
                                                                dict(F.run_kwargs(cfg, c), check_energy=True),
                                                                cfg["sweeps"]),)))
                   for cfg, c, b in jobs]
        results = {}
        for cfg, c, fut in pending:
            res = fut.get()
            assert res["energy_mismatch"] == 0, (cfg["name"], c["k"])
            print(f"{cfg['name']} instance {c['k']} (n={c['g']['n']}, R={len(c['betas'])}): "
                  f"{res['seconds']:.0f} s, best {res['best']} at {res['best_t']}, first hit {res['first_hit']}",
                  flush=True)
            results.setdefault(cfg["name"], {})[c["k"]] = F.to_json(res)
    for cfg, cases in todo:
        out = dict(workload=cfg["name"], sweeps=cfg["sweeps"], bank_sweeps=F.BANK_SWEEPS, bank_seed=F.BANK_SEED,
                   compared=list(F.COMPARED[cfg["name"]]), host=platform.processor() or platform.machine(),
                   wall_s=round(time.perf_counter() - t0, 1),
                   results={str(k): v for k, v in sorted(results[cfg["name"]].items())})
        with open(F.golden_path(cfg), "w") as f:
            json.dump(out, f, separators=(",", ":"))
            f.write("\n")
        print(f"wrote {F.golden_path(cfg)}", flush=True)


if __name__ == "__main__":
    main()
