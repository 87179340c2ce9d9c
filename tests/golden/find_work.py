"""Writes find_work.json: what the finder's algorithm does on the benchmark's finder
workloads, counted by the FP64 oracle's search (it calls only oracle/ and synth/).

For each workload: seeds, hits, and the oracle's counts of predictions that reach
their layer, hits inside a search window (each given a chi2), updates of surviving
hit branches, and seed refits.  The counts do not depend on how hits are binned (the
binned search equals the brute-force one).  bench.py multiplies them by the flops of
each operation to obtain the search kernel's algorithmic work.

    python tests/golden/find_work.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def count(k):
    geom, ev = synth.find_workload(k)
    t0 = time.time()
    r = oracle.find(geom, ev)
    w = [int(v) for v in r["work"]]
    return {"seeds": int(ev.seed_hits.shape[1]), "hits": int(ev.hits.shape[1]), "events": int(ev.hit_off.shape[0]),
            "predictions": w[0], "window_hits": w[1], "updates": w[2], "seed_refits": w[3],
            "oracle_seconds": round(time.time() - t0, 1), "oracle_threads": oracle.num_threads()}


def main():
    out = {"chi2_cut": 30.0, "nsigma": 3.0, "keep": 6, "max_miss": 3,
           "one_event_5000_tracks": count(3), "batched_64_events": count(5)}
    with open(os.path.join(HERE, "find_work.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
