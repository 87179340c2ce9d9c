"""Benchmark of the batched Kalman fit on one MI355X.

Workload (the headline metric's configuration): 1e6 tracks through 17 barrel layers
at radii 4..110 cm, B = 3.8 T, x/X0 = 0.02 per layer with Gaussian multiple
scattering, pT log-uniform 0.5..50 GeV, |eta| < 1.5, hits smeared 0.01 cm (r phi) and
0.1 cm (z), seeds built on the GPU from the first three hits with a ten-times
inflated prior.  Synthetic, seeded data (see synth/).

One step = one kf_fit launch over all tracks (inputs resident in HBM).  The metric is
Kalman propagate+update steps per second: every hit used by the filter is one step.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FP32 operations of one track (FMA = 2, each sqrt/rsqrt/division/
# transcendental = 1), counted from the step as written with the known zeros removed:
# propagation to the layer (crossing 47, fixed-arc transport of state and covariance
# 180), scattering noise 27, measurement and update (frame 12, hit placement 9,
# S and its inverse 85, residual and chi2 29, gain and Joseph update 345, chi2
# accumulation 1).  The three-hit seed costs 60.
FLOPS_PROPAGATE = 47 + 180
FLOPS_SCATTER = 27
FLOPS_UPDATE = 12 + 9 + 85 + 29 + 345 + 1
FLOPS_SEED = 60
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_HBM_GBS = 8000.0


def algorithmic_flops(n_hits_per_track, xX0_positive=True):
    n = np.asarray(n_hits_per_track, np.int64)
    n = n[n > 0]
    per = FLOPS_SEED + FLOPS_UPDATE * n + (FLOPS_PROPAGATE + (FLOPS_SCATTER if xX0_positive else 0)) * (n - 1)
    return float(per.sum())


def algorithmic_bytes(n_tracks, n_layers, n_steps):
    # hits read (12 B per used hit) + mask (4 B) + outputs: state 24, cov 84, chi2 4,
    # ndf 4, status 4 bytes per track
    return float(n_steps * 12 + n_tracks * (4 + 24 + 84 + 12))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tracks", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the fit shards tracks across GPUs with no exchange, "
              f"so --gpus {args.gpus} is not run here", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1906_11744_amd import Context

    t0 = time.time()
    geom, ts = synth.fit_workload(2, n=args.tracks)
    print(f"# generated {args.tracks} tracks in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    ctx = Context(geom)
    hits = torch.from_numpy(np.ascontiguousarray(ts.hits)).to(dev)
    mask = torch.from_numpy(ts.hit_mask.view(np.int32)).to(dev)
    xX0 = torch.from_numpy(geom.xX0.astype(np.float32)).to(dev)
    n = args.tracks
    out = None
    for _ in range(max(1, args.warmup)):
        out = ctx.fit(hits, mask, xX0=xX0, out=out)
    torch.cuda.synchronize()
    ndf = out["ndf"].cpu().numpy()
    status = out["status"].cpu().numpy().view(np.uint32)
    n_hits = np.where(status & 16, 0, (ndf + 5) // 2)
    steps_per_launch = int(n_hits.sum())
    flops = algorithmic_flops(n_hits)
    nbytes = algorithmic_bytes(n, geom.n_layers, steps_per_launch)

    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        ctx.fit(hits, mask, xX0=xX0, out=out)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    per = np.array([a.elapsed_time(b) for a, b in ev]) * 1e-3   # s per launch
    ms_per_step = wall / args.steps * 1e3
    value = steps_per_launch * args.steps / wall
    avg = float(per.mean())
    achieved_tflops = flops / avg / 1e12

    res = {
        "metric": "KF propagate+update steps/s (FP32 vs oracle tol)",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fit: 1e6 tracks x 17 barrel layers (4-110 cm), B=3.8 T, x/X0=0.02, "
                               "pT log-uniform 0.5-50 GeV, |eta|<1.5, seeds from first 3 hits (10x cov)",
                   "tracks": n, "layers": geom.n_layers, "kalman_steps_per_launch": steps_per_launch},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "fit_kernel", "avg_launch_ms": avg * 1e3,
                     "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                     "hbm_frac": nbytes / avg / 1e9 / PEAK_HBM_GBS},
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = min(n, 200_000)
        idx = np.arange(sample)
        h = np.ascontiguousarray(ts.hits[:, :, idx])
        m = ts.hit_mask[idx]
        t1 = time.perf_counter()
        ref = oracle.fit(geom, h, m)
        dt = time.perf_counter() - t1
        ref_steps = int(np.where(ref["status"] & 16, 0, (ref["ndf"] + 5) // 2).sum())
        res["cpu_baseline"] = {"value": ref_steps / dt, "unit": "steps/s", "cores": oracle.num_threads(),
                               "kind": "oracle",
                               "sample": f"first {sample} tracks of the same workload, FP64 C++ oracle, "
                                         f"{dt:.1f} s"}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
