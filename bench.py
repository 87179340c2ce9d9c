"""Benchmark of the batched Kalman fit on one MI355X.

Workload (the headline metric's configuration): 1e6 tracks through 17 barrel layers
at radii 4..110 cm, B = 3.8 T, x/X0 = 0.02 per layer with Gaussian multiple
scattering, pT log-uniform 0.5..50 GeV, |eta| < 1.5, hits smeared 0.01 cm (r phi) and
0.1 cm (z), seeds built on the GPU from the first three hits with a ten-times
inflated prior.  Synthetic, seeded data (see synth/).

One step = one kf_fit launch over all tracks (inputs resident in HBM).  The metric is
Kalman propagate+update steps per second: every hit used by the filter is one step.
The same JSON line also reports track finding (events/s for one event of 5 000 tracks
and for 64 events of uneven pileup in one call versus one call per event), the
adjoint's cost relative to the forward fit on 1e5 tracks, and the fixed-interval
smoother over the 1e6-track fit.  Prints one JSON line.
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

# Algorithmic FP32 operations (FMA = 2, add/mul = 1, each reciprocal, square root,
# logarithm or other transcendental = 1), counted from the formulas as the kernel
# evaluates them with the known zeros of J and H removed:
#   crossing 60, fixed-arc transport of state and covariance 194, frame 14,
#   Highland scattering 27, S and its equilibrated inverse (with H and H C) 83,
#   hit placement 9, residual and chi2 50, gain + state + Joseph covariance 356,
#   chi2 accumulation 1; the three-hit seed 91.
# A track with hits on layers 0..n-1 costs SEED + FIRST + (n - 1) * STEP.  The count
# agrees with the hardware's SQ_INSTS_VALU_FLOPS_FP32 of the fit kernel to 1%.
FLOPS_SEED = 91
FLOPS_PLACE = 9                                    # a hit placed on a layer its alignment moves
FLOPS_FIRST = 14 + 83 + FLOPS_PLACE + 50 + 356 + 1  # update at the seed layer
FLOPS_PROPAGATE = 60 + 194 + 14                    # crossing, transport, frame
FLOPS_SCATTER = 27
FLOPS_UPDATE = 83 + FLOPS_PLACE + 50 + 356 + 1
# The finder's algorithmic work, per operation of its algorithm (counts of each on the
# benchmark workloads are the oracle's, in tests/golden/find_work.json):
#   a prediction that reaches its layer: crossing, transport, frame, scattering, S and its
#     inverse, the window's half widths (2 square roots, a division, 3 products, 2 adds);
#   a hit inside a window: rectangle test (4) and its residual and chi2 (50);
#   an update of a surviving hit branch: gain, state and Joseph covariance (its residual
#     and S^-1 were formed by the scan and the prediction);
#   a seed refit: the three-hit seed, the update at layer 0, then two predictions and
#     updates (no alignment: no hit placement).
FLOPS_FIND_PREDICT = 60 + 194 + 14 + 27 + 83 + 8
FLOPS_FIND_WINDOW_HIT = 4 + 50
FLOPS_FIND_UPDATE = 356
FLOPS_FIND_SEED = 91 + (14 + 83 + 50 + 356 + 1) + 2 * (60 + 194 + 14 + 27 + 83 + 50 + 356 + 1)
FIND_WORK = os.path.join(ROOT, "tests", "golden", "find_work.json")
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (256 CU x 2.4 GHz x 256 flop/clk, packed FP32)
PEAK_FP32_UNPACKED_TFLOPS = 78.6  # the same without packed FP32 (64 FMA lanes per CU per clock)
PEAK_HBM_GBS = 8000.0

# HBM traffic of one fit_kernel launch on the 1e6-track workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch, mean over every launch of the run), each scaled by
# what the same counter reads for a device copy of 1 GiB (FETCH_SIZE 524 300 KiB,
# WRITE_SIZE 1 048 576 KiB).  Valid only while the fit kernel's sources hash to `sources`.
FIT_TRAFFIC = {"sources": "df523bda9e7396ef", "tracks": 1_000_000,
               "fetch_kib": 108222.4, "write_kib": 117298.2,
               "fetch_scale": 1048576.0 / 524300.0, "write_scale": 1.0}
FIT_SOURCES = ("paper_1906_11744_amd/csrc/kf_fit.hip", "paper_1906_11744_amd/csrc/kf_device.h")


# The same for one smooth_kernel launch on that workload.
SMOOTH_TRAFFIC = {"sources": "069c027262fcc2b9", "tracks": 1_000_000,
                  "fetch_kib": 902497.8, "write_kib": 1800781.2,
                  "fetch_scale": 1048576.0 / 524300.0, "write_scale": 1.0}
SMOOTH_SOURCES = ("paper_1906_11744_amd/csrc/kf_smooth.hip", "paper_1906_11744_amd/csrc/kf_smooth.h",
                  "paper_1906_11744_amd/csrc/kf_adjoint.h")


def _traffic_bytes(table, sources, n_tracks):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != table["sources"] or n_tracks != table["tracks"]:
        return None
    return 1024.0 * (table["fetch_kib"] * table["fetch_scale"] + table["write_kib"] * table["write_scale"])


# The same for one find_kernel launch on the 64-event batch (773 995 seeds) with the refit
# of each seed's best candidate: the median over the run's launches (most of them are of
# the configuration the autotuner keeps; the others are its trials); valid only while
# the finder's sources hash to `sources`.
FIND_TRAFFIC = {"sources": "b3bdc3bfb3b7b275", "tracks": 773995, "fetch_kib": 4252272.7, "write_kib": 3137996.8,
                "fetch_scale": 1048576.0 / 524300.0, "write_scale": 1.0}
FIND_SOURCES = ("paper_1906_11744_amd/csrc/kf_find.hip", "paper_1906_11744_amd/csrc/kf_device.h",
                "paper_1906_11744_amd/csrc/kf_internal.h")


def find_traffic_bytes(n_seeds):
    """Measured HBM bytes per search-kernel launch on the 64-event batch, or None."""
    if FIND_TRAFFIC["sources"] is None:
        return None
    return _traffic_bytes(FIND_TRAFFIC, FIND_SOURCES, n_seeds)


def find_algorithmic_flops(work):
    """Flops of the finder's algorithm for the operation counts `work` (find_work.json)."""
    return float(work["predictions"] * FLOPS_FIND_PREDICT + work["window_hits"] * FLOPS_FIND_WINDOW_HIT +
                 work["updates"] * FLOPS_FIND_UPDATE + work["seed_refits"] * FLOPS_FIND_SEED)


def fit_traffic_bytes(n_tracks):
    """Measured HBM bytes per fit launch, or None if the kernel or workload differs."""
    return _traffic_bytes(FIT_TRAFFIC, FIT_SOURCES, n_tracks)


def smooth_traffic_bytes(n_tracks):
    """Measured HBM bytes per smoother launch, or None if the kernel or workload differs."""
    return _traffic_bytes(SMOOTH_TRAFFIC, SMOOTH_SOURCES, n_tracks)


def algorithmic_flops(n_hits_per_track, xX0_positive=True, aligned=False):
    """Flops per launch; without alignment the hit placement is the identity, which the
    kernel skips, and is not counted."""
    n = np.asarray(n_hits_per_track, np.int64)
    n = n[n > 0]
    place = 0 if aligned else FLOPS_PLACE
    per = (FLOPS_SEED + FLOPS_FIRST - place +
           (FLOPS_PROPAGATE + (FLOPS_SCATTER if xX0_positive else 0) + FLOPS_UPDATE - place) * (n - 1))
    return float(per.sum())


def algorithmic_bytes(n_tracks, n_layers, n_steps):
    # hits read (12 B per used hit) + mask (4 B) + outputs: state 24, cov 84, chi2 4,
    # ndf 4, status 4 bytes per track
    return float(n_steps * 12 + n_tracks * (4 + 24 + 84 + 12))


# The GPU lowers its clocks within milliseconds of going idle and needs some tens of
# milliseconds of sustained load to raise them again (measured on the fit: ~235 us per
# launch cold, ~204 us after ~200 back-to-back launches).  Every timed function is
# first run back to back for this long, untimed, before its warm-up steps.
SETTLE_S = 0.2


def _settle(fn, seconds=SETTLE_S):
    """Run fn() back to back until `seconds` of wall clock have passed (synchronising
    every few calls so the host does not run ahead of the GPU); returns the calls made."""
    import torch
    t0 = time.perf_counter()
    calls = 0
    while True:
        for _ in range(4):
            fn()
        calls += 4
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            return calls


class Timing(tuple):
    """(region, per_launch, wall): seconds per call of a back-to-back region bracketed by
    one event pair, seconds per call from an event pair around each call, and wall-clock
    seconds per call of the region."""
    __slots__ = ()

    def __new__(cls, region, per_launch, wall):
        return super().__new__(cls, (region, per_launch, wall))

    region = property(lambda self: self[0])
    per_launch = property(lambda self: self[1])
    wall = property(lambda self: self[2])


def _time_launches(fn, steps, warmup):
    """Time `steps` back-to-back calls of fn() on the current stream (the library
    launches on it), after the clocks have settled and `warmup` untimed calls: one HIP
    event pair around the whole region (device time, including the GPU's gap between
    consecutive calls) and the host's wall clock around it, both between two
    synchronisations; then a second pass with an event pair around each call."""
    import torch
    _settle(fn)
    for _ in range(max(1, warmup)):
        fn()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    region = e0.elapsed_time(e1) * 1e-3 / steps
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    per_launch = sum(a.elapsed_time(b) for a, b in ev) * 1e-3 / steps
    return Timing(region, per_launch, wall / steps)


class _HipEvents:
    """Raw hipEvent_t handles from the HIP runtime torch has loaded (one runtime per
    process: both name the same soname), for kf_ctx_set_launch_events."""

    def __init__(self, count):
        import ctypes as C
        self._C = C
        self.hip = C.CDLL("libamdhip64.so.7")
        self.ev = []
        for _ in range(count):
            e = C.c_void_p()
            if self.hip.hipEventCreate(C.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e)

    def elapsed_ms(self, a, b):
        ms = self._C.c_float()
        rc = self.hip.hipEventElapsedTime(self._C.byref(ms), a, b)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return ms.value

    def close(self):
        for e in self.ev:
            self.hip.hipEventDestroy(e)
        self.ev = []


def _time_kernel(ctx, fn, steps, warmup):
    """Mean duration (s) of the library kernel launched by each of `steps` back-to-back
    calls of fn() (after `warmup`): the events of kf_ctx_set_launch_events, one pair per
    call, bracket that kernel's own execution on the stream."""
    import torch
    he = _HipEvents(2 * steps)
    _settle(fn)
    for _ in range(max(1, warmup)):
        fn()
    torch.cuda.synchronize()
    try:
        for k in range(steps):
            ctx.set_launch_events(he.ev[2 * k], he.ev[2 * k + 1])
            fn()
        ctx.set_launch_events(None, None)
        torch.cuda.synchronize()
        total = sum(he.elapsed_ms(he.ev[2 * k], he.ev[2 * k + 1]) for k in range(steps))
    finally:
        ctx.set_launch_events(None, None)
        torch.cuda.synchronize()
        he.close()
    return total * 1e-3 / steps


def bench_find(steps, warmup):
    """Track finding: one event of 5 000 tracks, and 64 events of uneven pileup in one
    call (find + refit of each seed's best candidate) against a loop of per-event calls."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    res = {}
    geom, ev = synth.find_workload(3)
    kf = Context(geom)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    xX0 = t(geom.xX0.astype(np.float32))
    args = (t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event))
    # the context's default configuration first (the geometry's bins, the default lanes
    # per seed and wide-window threshold), then the autotuned one
    out = kf.find(*args, xX0=xX0)
    kf.set_find_config(use_graph=1)
    avg_d, _, _ = _time_launches(lambda: kf.find(*args, xX0=xX0, out=out), steps, warmup)
    cfg_d = kf.find_config()
    kf.set_find_config(use_graph=0)
    out = kf.find(*args, xX0=xX0, autotune=True)
    avg, _, _ = _time_launches(lambda: kf.find(*args, xX0=xX0, out=out), steps, warmup)
    kf.set_find_config(use_graph=1)
    avg_g, _, _ = _time_launches(lambda: kf.find(*args, xX0=xX0, out=out), steps, warmup)
    res["single_event_5000_tracks"] = {"events_per_s": 1.0 / avg_g, "ms_per_event": avg_g * 1e3,
                                       "ms_per_event_without_graph": avg * 1e3,
                                       "seeds": int(ev.seed_hits.shape[1]), "config": kf.find_config(),
                                       "ms_per_event_default_config": avg_d * 1e3, "default_config": cfg_d}
    t0 = time.time()
    geom, ev = synth.find_workload(5)
    print(f"# generated 64 events ({ev.seed_hits.shape[1]} seeds, {ev.hits.shape[1]} hits) in "
          f"{time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    kf = Context(geom)
    xX0 = t(geom.xX0.astype(np.float32))
    args = (t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event))
    out = kf.find(*args, xX0=xX0, refit=True)
    kf.set_find_config(use_graph=1)
    avg_bd, _, _ = _time_launches(lambda: kf.find(*args, xX0=xX0, refit=True, out=out), max(3, steps // 4), warmup)
    cfg_bd = kf.find_config()
    kf.set_find_config(use_graph=0)
    out = kf.find(*args, xX0=xX0, refit=True, autotune=True, out=out)
    kf.set_find_config(use_graph=1)
    avg_b, _, _ = _time_launches(lambda: kf.find(*args, xX0=xX0, refit=True, out=out), max(3, steps // 4), warmup)
    # per-event calls on the same data
    E = ev.hit_off.shape[0]
    per_event = []
    for e in range(E):
        sel = np.nonzero(ev.seed_event == e)[0]
        lo, hi = int(ev.hit_off[e, 0]), int(ev.hit_off[e, -1])
        per_event.append((t(ev.hits[:, lo:hi]), t(ev.hit_off[e:e + 1] - lo),
                          t((ev.seed_hits[:, sel] - lo).astype(np.int32)),
                          t(np.zeros(sel.shape[0], np.int32))))
    cfg_batched = kf.find_config()
    kf.set_find_config(use_graph=0)   # a graph per event would be captured anew at every call
    outs = [kf.find(*a, xX0=xX0, refit=True) for a in per_event]

    def loop():
        for a, o in zip(per_event, outs):
            kf.find(*a, xX0=xX0, refit=True, out=o)
    avg_l, _, _ = _time_launches(loop, max(3, steps // 4), warmup)
    res["batched_64_events"] = {"events_per_s": E / avg_b, "ms_per_call": avg_b * 1e3, "config": cfg_batched,
                                "ms_per_call_default_config": avg_bd * 1e3, "default_config": cfg_bd,
                                "seeds": int(ev.seed_hits.shape[1]), "hits": int(ev.hits.shape[1]),
                                "fp64_fallback": _fallback_rates(out)}
    # the search kernel alone, on its own launch events (plain launches, the tuned
    # configuration), against the algorithmic flops of what the search does
    with open(FIND_WORK) as fh:
        work = json.load(fh)["batched_64_events"]
    if work["seeds"] == int(ev.seed_hits.shape[1]) and work["hits"] == int(ev.hits.shape[1]):
        kf.set_find_config(**dict(cfg_batched, use_graph=0))
        t_k = _time_kernel(kf, lambda: kf.find(*args, xX0=xX0, refit=True, out=out), max(3, steps // 4), warmup)
        flops = find_algorithmic_flops(work)
        ach = flops / t_k / 1e12
        res["batched_64_events"]["roofline"] = {
            "bound": "alu", "achieved": ach, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP32_TFLOPS, "traffic": find_traffic_bytes(work["seeds"]),
            "traffic_unit": "B per launch", "kernel": "find_kernel", "avg_launch_ms": t_k * 1e3,
            "algorithmic_flops_per_launch": flops, "work": {k: work[k] for k in
                                                            ("predictions", "window_hits", "updates", "seed_refits")},
            "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS, "frac_unpacked": ach / PEAK_FP32_UNPACKED_TFLOPS}
    res["per_event_loop_64_events"] = {"events_per_s": E / avg_l, "ms_total": avg_l * 1e3}
    res["batched_speedup"] = avg_l / avg_b
    return res


def _fallback_rates(out):
    """Share of the finder's candidates (every kept rank, counted where a candidate
    exists) and of the refitted best candidates whose status carries the FP64-fallback
    bit (at least one update took S^-1 and chi2 in FP64)."""
    n_cand = out["n_cand"].cpu().numpy()
    st = out["status"].cpu().numpy()
    live = np.arange(st.shape[0])[:, None] < n_cand[None, :]
    r = {"find_candidates": float(((st & 4) != 0)[live].mean()) if live.any() else 0.0,
         "find_rank0": float(((st[0] & 4) != 0)[n_cand > 0].mean()) if (n_cand > 0).any() else 0.0}
    if out.get("rf_status") is not None:
        rs = out["rf_status"].cpu().numpy()
        r["refit"] = float(((rs & 4) != 0)[n_cand > 0].mean()) if (n_cand > 0).any() else 0.0
    return r


def bench_grad(steps, warmup):
    """Differentiable fit: 1e5 misaligned tracks; forward (fit with checkpoints) and the
    adjoint (kf_fit_backward), each timed alone, in the uniform field and under the
    parameterised one."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, align=a_true)
    kf = Context(geom)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hits, mask = t(ts.hits), t(ts.hit_mask.view(np.int32))
    al, xX0 = t(np.zeros((geom.n_layers, 4), np.float32)), t(geom.xX0.astype(np.float32))
    fwd = kf.fit(hits, mask, align=al, xX0=xX0, ckpt=True)
    w = torch.ones(ts.hits.shape[2], dtype=torch.float32, device=dev)
    t_f, _, _ = _time_launches(lambda: kf.fit(hits, mask, align=al, xX0=xX0, ckpt=True, out=fwd), steps, warmup)
    t_b, _, _ = _time_launches(lambda: kf.fit_backward(hits, mask, fwd, w, align=al, xX0=xX0), steps, warmup)
    n = int(ts.hits.shape[2])
    ndf = fwd["ndf"].cpu().numpy()
    status = fwd["status"].cpu().numpy().view(np.uint32)
    n_steps = int(np.where(status & 16, 0, (ndf + 5) // 2).sum())
    # bytes each must move: the forward reads 12 B of hit per step and the mask, writes
    # the outputs (120 B per track) and a 27-float checkpoint per step; the adjoint
    # reads the checkpoint and the hit of every step and 16 B per track (mask, status,
    # ndf, dLoss/dchi2); its gradient output is negligible
    b_f = 120.0 * n_steps + 124.0 * n
    b_b = 120.0 * n_steps + 16.0 * n
    # the same inputs under the parameterised field (every step evaluates its field)
    kfb = Context(geom)
    kfb.set_field(*synth.FIELD_SOLENOID)
    fwdb = kfb.fit(hits, mask, align=al, xX0=xX0, ckpt=True)
    t_fb, _, _ = _time_launches(lambda: kfb.fit(hits, mask, align=al, xX0=xX0, ckpt=True, out=fwdb), steps, warmup)
    t_bb, _, _ = _time_launches(lambda: kfb.fit_backward(hits, mask, fwdb, w, align=al, xX0=xX0), steps, warmup)
    # sparse checkpoints: the forward keeps every k-th layer, the adjoint recomputes the rest
    sparse = {}
    for k in (2, 4, 17):
        fk = kf.fit(hits, mask, align=al, xX0=xX0, ckpt=True, ckpt_every=k)
        tkf, _, _ = _time_launches(lambda: kf.fit(hits, mask, align=al, xX0=xX0, ckpt=True, ckpt_every=k, out=fk),
                                   steps, warmup)
        tkb, _, _ = _time_launches(lambda: kf.fit_backward(hits, mask, fk, w, align=al, xX0=xX0), steps, warmup)
        sparse[str(k)] = {"checkpoint_bytes": int(fk["ckpt"].numel() * 4), "forward_ms": tkf * 1e3,
                          "backward_ms": tkb * 1e3, "backward_over_forward": tkb / tkf}
    # the material model (16-bin map per layer, silicon's energy loss) in forward and adjoint
    xmap = synth.material_map(geom).astype(np.float32)
    kfm = Context(geom)
    dmap = t(xmap)
    kfm.set_material(dmap, synth.ELOSS_SI_GEV_PER_X0)
    fwdm = kfm.fit(hits, mask, align=al, xX0=xX0, ckpt=True)
    t_fm, _, _ = _time_launches(lambda: kfm.fit(hits, mask, align=al, xX0=xX0, ckpt=True, out=fwdm), steps, warmup)
    t_bm, _, _ = _time_launches(lambda: kfm.fit_backward(hits, mask, fwdm, w, align=al, xX0=xX0), steps, warmup)
    return {"tracks": n, "kalman_steps": n_steps, "forward_ms": t_f * 1e3, "backward_ms": t_b * 1e3,
            "backward_over_forward": t_b / t_f, "checkpoint_bytes": int(fwd["ckpt"].numel() * 4),
            "field_forward_ms": t_fb * 1e3, "field_backward_ms": t_bb * 1e3,
            "material_forward_ms": t_fm * 1e3, "material_backward_ms": t_bm * 1e3,
            "sparse_checkpoints": sparse,
            "forward_algorithmic_bytes": b_f, "forward_GB_per_s": b_f / t_f / 1e9,
            "backward_algorithmic_bytes": b_b, "backward_GB_per_s": b_b / t_b / 1e9}


def bench_material(steps, warmup):
    """The fit with the detector model of Sec. 3: 1e6 tracks simulated through a 16-bin
    x/X0 map per layer with the mean energy loss of silicon, in the field B_z(r, z),
    fitted with the whole model (kf_ctx_set_material + kf_ctx_set_field); the same
    tracks fitted with the material model alone and with one x/X0 per layer in a
    uniform field, for the cost of each part."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    t0 = time.time()
    geom, ts, fld, (xmap, eloss) = synth.field_workload(1_000_000, material=True)
    print(f"# generated 1e6 tracks through the material map and field in {time.time() - t0:.1f} s", file=sys.stderr,
          flush=True)
    ctx = Context(geom)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hits, mask = t(ts.hits), t(ts.hit_mask.view(np.int32))
    xX0 = t(geom.xX0.astype(np.float32))
    dmap = t(xmap.astype(np.float32))
    ctx.set_material(dmap, eloss)
    ctx.set_field(*fld)
    out = ctx.fit(hits, mask, xX0=xX0)
    ndf = out["ndf"].cpu().numpy()
    status = out["status"].cpu().numpy().view(np.uint32)
    n_steps = int(np.where(status & 16, 0, (ndf + 5) // 2).sum())
    fn = lambda: ctx.fit(hits, mask, xX0=xX0, out=out)
    tm = _time_launches(fn, steps, warmup)
    t_full = _time_kernel(ctx, fn, steps, warmup)
    ctx.set_field(0.0, 0.0)
    t_mat = _time_kernel(ctx, fn, steps, warmup)
    ctx.set_material(None, 0.0)
    t_plain = _time_kernel(ctx, fn, steps, warmup)
    res = {"tracks": int(ts.hits.shape[2]), "kalman_steps": n_steps, "map_bins": int(xmap.shape[1]),
           "eloss_gev_per_x0": eloss, "field_c_r_c_z": list(fld), "steps_per_s": n_steps / tm.wall,
           "ms_per_call": tm.wall * 1e3, "kernel_ms": t_full * 1e3, "kernel_ms_material_only": t_mat * 1e3,
           "kernel_ms_one_xX0_per_layer_uniform_field": t_plain * 1e3, "model_cost_ratio": t_full / t_plain}
    # the finder on one event of 5 000 tracks simulated with the whole model
    ev = synth.make_events(geom, [5000], workload=10, material=(xmap, eloss), field=fld)
    args = (t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event))
    ctx.set_material(dmap, eloss)
    ctx.set_field(*fld)
    ctx.set_find_config(use_graph=1)
    fout = ctx.find(*args, xX0=xX0)
    t_fm = _time_launches(lambda: ctx.find(*args, xX0=xX0, out=fout), steps, warmup).region
    ctx.set_material(None, 0.0)
    ctx.set_field(0.0, 0.0)
    fout = ctx.find(*args, xX0=xX0)
    t_fp = _time_launches(lambda: ctx.find(*args, xX0=xX0, out=fout), steps, warmup).region
    res["find_one_event_5000_tracks"] = {"events_per_s": 1.0 / t_fm, "ms_per_event": t_fm * 1e3,
                                         "ms_per_event_one_xX0_per_layer_uniform_field": t_fp * 1e3}
    # the smoother over the 1e6-track fit under the whole model, against the plain model
    ctx.set_material(dmap, eloss)
    ctx.set_field(*fld)
    fwd = ctx.fit(hits, mask, xX0=xX0, ckpt=True)
    sout = ctx.smooth(hits, mask, fwd, xX0=xX0)
    t_sm = _time_kernel(ctx, lambda: ctx.smooth(hits, mask, fwd, xX0=xX0, out=sout), steps, warmup)
    ctx.set_material(None, 0.0)
    ctx.set_field(0.0, 0.0)
    fwd = ctx.fit(hits, mask, xX0=xX0, ckpt=True, out=fwd)
    t_sp = _time_kernel(ctx, lambda: ctx.smooth(hits, mask, fwd, xX0=xX0, out=sout), steps, warmup)
    res["smooth_1e6_tracks"] = {"kernel_ms": t_sm * 1e3, "kernel_ms_one_xX0_per_layer_uniform_field": t_sp * 1e3}
    return res


def bench_endcap(steps, warmup):
    """Barrel and endcap (17 bounded cylinders, 7 disks per side, |eta| < 2.5): the fit of
    1e5 tracks and the finder (with refit) on 8 events of 5 000 tracks."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    geom, ts = synth.endcap_workload(n=100_000)
    ctx = Context(geom)
    hits, mask, xX0 = t(ts.hits), t(ts.hit_mask.view(np.int32)), t(geom.xX0.astype(np.float32))
    out = ctx.fit(hits, mask, xX0=xX0)
    torch.cuda.synchronize()
    ndf = out["ndf"].cpu().numpy()
    status = out["status"].cpu().numpy().view(np.uint32)
    n_steps = int(np.where(status & 16, 0, (ndf + 5) // 2).sum())
    tm = _time_launches(lambda: ctx.fit(hits, mask, xX0=xX0, out=out), steps, warmup)
    tk = _time_kernel(ctx, lambda: ctx.fit(hits, mask, xX0=xX0, out=out), steps, warmup)
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    res = {"fit": {"tracks": 100_000, "kalman_steps": n_steps, "steps_per_s": n_steps / tm.wall,
                   "ms_per_call": tm.wall * 1e3, "kernel_ms": tk * 1e3,
                   "tracks_ending_on_a_disk": float(np.mean(geom.is_disk[last]))}}
    geom, ev = synth.endcap_find_workload(n_tracks=5000, n_events=8)
    cf = Context(geom)
    args = (t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event))
    xf = t(geom.xX0.astype(np.float32))
    fo = cf.find(*args, xX0=xf, refit=True)
    torch.cuda.synchronize()
    tf = _time_launches(lambda: cf.find(*args, xX0=xf, refit=True, out=fo), max(3, steps // 4), warmup)
    S = ev.seed_hits.shape[1]
    res["find"] = {"events": 8, "seeds": S, "hits": int(ev.hits.shape[1]), "ms_per_call": tf.wall * 1e3,
                   "seeds_per_s": S / tf.wall}
    return res


def bench_smooth(steps, warmup, n_tracks):
    """Fixed-interval smoother over the fit workload: the fit with checkpoints, then
    kf_smooth of every track (the smoothed state and covariance of every layer)."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    geom, ts = synth.fit_workload(2, n=n_tracks)
    ctx = Context(geom)
    hits = torch.from_numpy(np.ascontiguousarray(ts.hits)).to(dev)
    mask = torch.from_numpy(ts.hit_mask.view(np.int32)).to(dev)
    xX0 = torch.from_numpy(geom.xX0.astype(np.float32)).to(dev)
    fwd = ctx.fit(hits, mask, xX0=xX0, ckpt=True)
    out = ctx.smooth(hits, mask, fwd, xX0=xX0)
    torch.cuda.synchronize()
    layers = int((out["last"] - out["first"] + 1).clamp(min=0).sum().item())
    t_f, _, _ = _time_launches(lambda: ctx.fit(hits, mask, xX0=xX0, ckpt=True, out=fwd), steps, warmup)
    t_s, _, _ = _time_launches(lambda: ctx.smooth(hits, mask, fwd, xX0=xX0, out=out), steps, warmup)
    t_k = _time_kernel(ctx, lambda: ctx.smooth(hits, mask, fwd, xX0=xX0, out=out), steps, warmup)
    # HBM bytes the smoother must move: the checkpoint (27 floats) of every smoothed
    # layer read, the whole output (27 floats on every layer, zeros included) written,
    # mask/ndf/status read and first/last written
    nbytes = layers * 27 * 4 + geom.n_layers * n_tracks * 27 * 4 + n_tracks * 5 * 4
    gbs = nbytes / t_k / 1e9
    return {"tracks": n_tracks, "smoothed_layers": layers, "forward_with_checkpoints_ms": t_f * 1e3,
            "smooth_ms": t_s * 1e3, "smoothed_layers_per_s": layers / t_s,
            "roofline": {"kernel": "smooth_kernel", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                         "avg_launch_ms": t_k * 1e3,
                         "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": smooth_traffic_bytes(n_tracks),
                         "algorithmic_bytes": nbytes}}


def bench_dedup(steps, warmup):
    """Duplicate handling on the 64-event workload with 5% of its seeds duplicated
    (second measurements of seed hits): seed cleaning over all seeds, then the finder
    (with refit) over the kept seeds and duplicate removal over their rank-0 candidates."""
    import torch

    import synth
    from paper_1906_11744_amd import Context
    dev = torch.device("cuda:0")
    geom, ev = synth.find_workload(5)
    ev, _ = synth.inject_duplicate_seeds(geom, ev, 0.05)
    ctx = Context(geom)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hits, off, sh, se = t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event)
    xX0 = t(geom.xX0.astype(np.float32))
    keep = ctx.clean_seeds(hits, off, sh, se, xX0=xX0)
    t_clean, _, _ = _time_launches(lambda: ctx.clean_seeds(hits, off, sh, se, xX0=xX0, out=keep), steps, warmup)
    sel = torch.nonzero(keep == 1).flatten()
    sh2, se2 = sh[:, sel].contiguous(), se[sel].contiguous()
    out = ctx.find(hits, off, sh2, se2, xX0=xX0, refit=True)
    hi, nh, c2 = out["hit_idx"][0].contiguous(), out["n_hits"][0].contiguous(), out["chi2"][0].contiguous()
    E = int(off.shape[0])
    kt = ctx.remove_duplicates(hits, E, se2, hi, nh, c2, out["rf_state"], xX0=xX0)
    t_rm, _, _ = _time_launches(lambda: ctx.remove_duplicates(hits, E, se2, hi, nh, c2, out["rf_state"], xX0=xX0,
                                                              out=kt), steps, warmup)
    torch.cuda.synchronize()
    S, S2 = int(sh.shape[1]), int(sh2.shape[1])
    return {"events": E, "seeds": S, "seeds_removed_by_cleaning": S - S2,
            "tracks_removed_after_building": int((kt == 0).sum().item()),
            "clean_ms": t_clean * 1e3, "clean_seeds_per_s": S / t_clean,
            "remove_ms": t_rm * 1e3, "remove_tracks_per_s": S2 / t_rm}


def _cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo) and its logical CPUs."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip() + f" ({os.cpu_count()} logical CPUs on the host)"
    except OSError:
        pass
    return None


def _cpu_more(geom, ts):
    """More of the oracle on the host, each on a bounded sample: the fit on one thread
    (20 000 tracks of the fit workload, passes until 3 s), and the finder with every
    thread on the one-event workload (5 000 tracks) and on the first 24 000 seeds of the
    64-event batch (every event's hits), scaled to events by the batch's seeds per event."""
    import oracle
    import synth
    out = {}
    sub_hits = np.ascontiguousarray(ts.hits[:, :, :20000])
    sub_mask = np.ascontiguousarray(ts.hit_mask[:20000])
    try:
        oracle.set_num_threads(1)
        t0 = time.perf_counter()
        passes, st = 0, 0
        while True:
            r = oracle.fit(geom, sub_hits, sub_mask)
            passes += 1
            st += int(np.where(r["status"] & 16, 0, (r["ndf"] + 5) // 2).sum())
            dt = time.perf_counter() - t0
            if dt >= 3.0:
                break
        out["one_thread_value"] = st / dt
        out["one_thread_sample"] = f"{passes} pass(es) over 20 000 tracks of the workload, 1 thread, {dt:.1f} s"
    finally:
        oracle.set_num_threads(0)
    g3, ev3 = synth.find_workload(3)
    t0 = time.perf_counter()
    oracle.find(g3, ev3)
    dt = time.perf_counter() - t0
    out["find_one_event_5000_tracks"] = {"events_per_s": 1.0 / dt, "threads": oracle.num_threads()}
    g5, ev5 = synth.find_workload(5)
    from types import SimpleNamespace
    k = 24000
    sub = SimpleNamespace(hits=ev5.hits, hit_off=ev5.hit_off, seed_hits=np.ascontiguousarray(ev5.seed_hits[:, :k]),
                          seed_event=np.ascontiguousarray(ev5.seed_event[:k]))
    t0 = time.perf_counter()
    oracle.find(g5, sub)
    dt = time.perf_counter() - t0
    per_event = ev5.seed_hits.shape[1] / ev5.hit_off.shape[0]
    out["find_64_events"] = {"events_per_s": k / dt / per_event, "seeds_per_s": k / dt,
                             "threads": oracle.num_threads(),
                             "sample": f"first {k} of {ev5.seed_hits.shape[1]} seeds (binning of all 64 events "
                                       f"included), {dt:.1f} s"}
    return out


def cpu_scaling():
    """The oracle's finder over several events at once (its OpenMP loop runs over every
    seed of every event, so all events are in flight together) against the number of
    threads: the CPU reference point for the finder, the analogue of the paper's scan of
    events in flight.  8 events of the 64-event mix scaled to ~1 250 tracks each."""
    import os

    import oracle
    import synth
    geom, ev = synth.find_workload(5, n_tracks=1250, n_events=8)
    n_cpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = [t for t in (1, 2, 4, 8, 16, 32, 64) if t <= n_cpu]
    rows = []
    try:
        for t in threads:
            oracle.set_num_threads(t)
            t0 = time.perf_counter()
            oracle.find(geom, ev)
            dt = time.perf_counter() - t0
            rows.append({"threads": t, "s": dt, "events_per_s": ev.n_tracks.shape[0] / dt})
            print(f"# cpu scaling: {t} threads {dt:.2f} s", file=sys.stderr, flush=True)
    finally:
        oracle.set_num_threads(0)
    base = rows[0]["s"]
    for r in rows:
        r["speedup"] = base / r["s"]
    return {"events": int(ev.n_tracks.shape[0]), "seeds": int(ev.seed_hits.shape[1]),
            "tracks_per_event_mean": float(ev.n_tracks.mean()), "scan": rows}


def copy_calibration(steps):
    """A plain device copy of 1 GiB, `steps` times: the reference kernel whose HBM
    counters (FETCH_SIZE, WRITE_SIZE) calibrate those of the fit kernel."""
    import torch
    n = 1 << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    avg, _, _ = _time_launches(lambda: b.copy_(a), steps, 1)
    return {"copy_bytes_each_way": 4 * n, "avg_ms": avg * 1e3, "GB_per_s": 8 * n / avg / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tracks", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["all", "fit", "find", "grad", "smooth", "dedup", "material", "endcap",
                                       "cpu_scaling", "copy"],
                    default="all")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the fit shards tracks across GPUs with no exchange, "
              f"so --gpus {args.gpus} is not run here", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1906_11744_amd import Context

    res = None
    if args.only in ("all", "fit"):
        t0 = time.time()
        geom, ts = synth.fit_workload(2, n=args.tracks)
        print(f"# generated {args.tracks} tracks in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
        dev = torch.device("cuda:0")
        ctx = Context(geom)
        hits = torch.from_numpy(np.ascontiguousarray(ts.hits)).to(dev)
        mask = torch.from_numpy(ts.hit_mask.view(np.int32)).to(dev)
        xX0 = torch.from_numpy(geom.xX0.astype(np.float32)).to(dev)
        n = args.tracks
        out = ctx.fit(hits, mask, xX0=xX0)
        torch.cuda.synchronize()
        ndf = out["ndf"].cpu().numpy()
        status = out["status"].cpu().numpy().view(np.uint32)
        n_hits = np.where(status & 16, 0, (ndf + 5) // 2)
        steps_per_launch = int(n_hits.sum())
        flops = algorithmic_flops(n_hits)
        nbytes = algorithmic_bytes(n, geom.n_layers, steps_per_launch)
        tm = _time_launches(lambda: ctx.fit(hits, mask, xX0=xX0, out=out), args.steps, args.warmup)
        avg = _time_kernel(ctx, lambda: ctx.fit(hits, mask, xX0=xX0, out=out), args.steps, args.warmup)
        value = steps_per_launch / tm.wall
        achieved_tflops = flops / avg / 1e12
        res = {
            "metric": "KF propagate+update steps/s (FP32 vs oracle tol)",
            "value": value,
            "unit": "steps/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": tm.wall * 1e3,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "fit: 1e6 tracks x 17 barrel layers (4-110 cm), B=3.8 T, x/X0=0.02, "
                                   "pT log-uniform 0.5-50 GeV, |eta|<1.5, seeds from first 3 hits (10x cov)",
                       "tracks": n, "layers": geom.n_layers, "kalman_steps_per_launch": steps_per_launch},
            "fp64_fallback_tracks": float(((status & 4) != 0).mean()),
            "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved_tflops / PEAK_FP32_TFLOPS, "traffic": fit_traffic_bytes(n),
                         "traffic_unit": "B per launch",
                         "kernel": "fit_kernel", "avg_launch_ms": avg * 1e3,
                         "ms_per_call_with_kernel_gaps": tm.region * 1e3,
                         "ms_per_call_with_per_call_events": tm.per_launch * 1e3,
                         "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": nbytes,
                         "hbm_frac": nbytes / avg / 1e9 / PEAK_HBM_GBS,
                         "peak_unpacked": PEAK_FP32_UNPACKED_TFLOPS,
                         "frac_unpacked": achieved_tflops / PEAK_FP32_UNPACKED_TFLOPS},
        }
        # the small configuration (1 000 tracks, 10 layers, no material): 16 waves on
        # 1 024 SIMDs, so a launch is latency-bound; reported per call, not as a roofline
        g1, ts1 = synth.fit_workload(1)
        ctx1 = Context(g1)
        h1 = torch.from_numpy(np.ascontiguousarray(ts1.hits)).to(dev)
        m1 = torch.from_numpy(ts1.hit_mask.view(np.int32)).to(dev)
        o1 = ctx1.fit(h1, m1)
        tm1 = _time_launches(lambda: ctx1.fit(h1, m1, out=o1), args.steps, args.warmup)
        t1 = _time_kernel(ctx1, lambda: ctx1.fit(h1, m1, out=o1), args.steps, args.warmup)
        res["fit_1000_tracks_10_layers"] = {"us_per_call": tm1.region * 1e6, "us_kernel": t1 * 1e6,
                                            "us_per_call_with_per_call_events": tm1.per_launch * 1e6}
        if not args.no_cpu_baseline:
            # the oracle over the whole workload, pass after pass, until 10 s have elapsed
            import oracle
            h = np.ascontiguousarray(ts.hits)
            t1 = time.perf_counter()
            passes, ref_steps = 0, 0
            while True:
                ref = oracle.fit(geom, h, ts.hit_mask)
                passes += 1
                ref_steps += int(np.where(ref["status"] & 16, 0, (ref["ndf"] + 5) // 2).sum())
                dt = time.perf_counter() - t1
                if dt >= 10.0:
                    break
            res["cpu_baseline"] = {"value": ref_steps / dt, "unit": "steps/s", "cores": oracle.num_threads(),
                                   "kind": "oracle",
                                   "sample": f"{passes} pass(es) over all {n} tracks of the same workload, FP64 C++ "
                                             f"oracle (OpenMP over tracks), {dt:.1f} s",
                                   "cpu_model": _cpu_model()}
            res["cpu_baseline"].update(_cpu_more(geom, ts))
        del hits, mask, out
    else:
        res = {"metric": "KF propagate+update steps/s (FP32 vs oracle tol)", "value": None, "unit": "steps/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup}
    if args.only == "copy":
        res["copy_calibration"] = copy_calibration(args.steps)
    if args.only in ("all", "find"):
        res["find"] = bench_find(args.steps, args.warmup)
    if args.only in ("all", "grad"):
        res["adjoint"] = bench_grad(args.steps, args.warmup)
    if args.only in ("all", "smooth"):
        res["smooth"] = bench_smooth(args.steps, args.warmup, args.tracks)
    if args.only in ("all", "dedup"):
        res["dedup"] = bench_dedup(args.steps, args.warmup)
    if args.only in ("all", "material"):
        res["material"] = bench_material(args.steps, args.warmup)
    if args.only in ("all", "endcap"):
        res["endcap"] = bench_endcap(args.steps, args.warmup)
    if args.only in ("all", "cpu_scaling") and not args.no_cpu_baseline:
        res["cpu_finder_scaling"] = cpu_scaling()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
