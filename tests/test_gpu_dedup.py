"""GPU duplicate handling (kf_clean_seeds, kf_remove_duplicates, through the C ABI)
against the oracle's brute-force relation on the same inputs.

The keep masks are integers: they must be identical, except for items whose decision
the oracle flags as float-sensitive (a compared quantity within float rounding of its
cut).  Cases: one event and 64 events of uneven size with injected duplicate seeds
(second measurements of seed hits), misaligned layers, the azimuth wrap, clusters of
identical copies, a window so wide that every item shares one or two bins, invalid
seeds, empty input; the removal on the GPU finder's own rank-0 candidates."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _ctx(geom):
    need_gpu()
    from paper_1906_11744_amd import Context
    return Context(geom)


def _gpu_clean(ctx, ev, align=None):
    a = None if align is None else to_dev(np.asarray(align, np.float32))
    keep = ctx.clean_seeds(to_dev(ev.hits), to_dev(ev.hit_off), to_dev(ev.seed_hits), to_dev(ev.seed_event), align=a)
    torch.cuda.synchronize()
    return keep.cpu().numpy()


def _compare(g, r, sens, label):
    diff = g != r
    print(f"[{label}] n={g.size}: removed {int((r == 0).sum())}, differences {int(diff.sum())}, "
          f"of which float-sensitive {int((diff & sens).sum())}, sensitive items {int(sens.sum())}")
    assert not np.any(diff & ~sens), (label, np.nonzero(diff & ~sens)[0][:10])


def _cuts_of(ctx):
    c = ctx.dedup_cuts()
    seed = dict(psi_window=c["psi_window"], min_shared=c["min_shared"], min_shared_kin=c["min_shared_kin"],
                kap_rel=c["seed_kap_rel"], kap_abs=c["seed_kap_abs"], theta=c["seed_theta"], phi=c["seed_phi"],
                z=c["seed_z"])
    trk = dict(psi_window=c["psi_window"], shared_frac=c["trk_shared_frac"], kap_rel=c["trk_kap_rel"],
               kap_abs=c["trk_kap_abs"], theta=c["trk_theta"])
    # the oracle in FP64 on the float cuts the library holds
    return {k: float(v) if isinstance(v, float) else v for k, v in seed.items()}, \
        {k: float(v) for k, v in trk.items()}


def test_clean_one_event_with_injected_duplicates():
    geom, ev = synth.find_workload(3)
    ev2, dup_of = synth.inject_duplicate_seeds(geom, ev, 0.1)
    ctx = _ctx(geom)
    sc, _ = _cuts_of(ctx)
    g = _gpu_clean(ctx, ev2)
    r, sens = oracle.clean_seeds(geom, ev2, cuts=sc)
    _compare(g, r, sens, "one event, 10% injected")
    inj = dup_of >= 0
    assert np.all(g[~inj] == 1) and (g[inj] == 0).mean() > 0.75


def test_clean_64_events_misaligned():
    geom, ev = synth.find_workload(5)
    ev2, _ = synth.inject_duplicate_seeds(geom, ev, 0.05)
    align = synth.misalignment(geom.n_layers)
    ctx = _ctx(geom)
    sc, _ = _cuts_of(ctx)
    g = _gpu_clean(ctx, ev2, align=align)
    r, sens = oracle.clean_seeds(geom, ev2, cuts=sc, align=align)
    _compare(g, r, sens, "64 events, 5% injected, misaligned")
    assert (r == 0).sum() > 20000


def _tiny(geom):
    L = geom.n_layers
    angs0 = [math.pi - 0.001, -math.pi + 0.001, 0.5, 0.5004]
    angs12 = [math.pi - 0.001, 0.5]
    per = [angs0, angs12, angs12]
    hits, off = [], [0]
    for l in range(L):
        angs = per[l] if l < 3 else []
        r = geom.radius[l]
        hits += [(r * math.cos(a), r * math.sin(a), 0.1 * r) for a in angs]
        off.append(off[-1] + len(angs))
    o = off
    # seeds: 0 at the wrap, 1 its duplicate across the wrap, 2-4 copies of 0, 5 at 0.5,
    # 6 its duplicate by a second layer-0 measurement, 7 invalid (hit outside its layer
    # slice), 8 invalid event
    s = [[o[0], o[1], o[2]], [o[0] + 1, o[1], o[2]], [o[0], o[1], o[2]], [o[0], o[1], o[2]], [o[0], o[1], o[2]],
         [o[0] + 2, o[1] + 1, o[2] + 1], [o[0] + 3, o[1] + 1, o[2] + 1], [o[1], o[1], o[2]], [o[0], o[1], o[2]]]
    ev = synth.EventBatch(hits=np.ascontiguousarray(np.array(hits, np.float32).T), hit_off=np.array([off], np.int64),
                          hit_track=np.full(len(hits), -1, np.int64),
                          seed_hits=np.ascontiguousarray(np.array(s, np.int32).T),
                          seed_event=np.array([0] * 8 + [5], np.int32), seed_track=np.zeros(9, np.int64),
                          track_event=np.zeros(0, np.int32), track_hits=np.zeros((L, 0), np.int64),
                          n_tracks=np.array([0]))
    return ev


def test_clean_edge_cases():
    geom = synth.workload_geometry(2)
    ctx = _ctx(geom)
    ev = _tiny(geom)
    for window in (0.05, 2.5, 4.0, 7.0):   # nb = 125, 2, 1, 1 bins
        ctx.set_dedup_cuts(psi_window=window)
        sc, _ = _cuts_of(ctx)
        g = _gpu_clean(ctx, ev)
        r, sens = oracle.clean_seeds(geom, ev, cuts=sc)
        assert not sens.any()
        assert np.array_equal(g, r), (window, g, r)
        if window == 0.05:
            assert g.tolist() == [1, 0, 0, 0, 0, 1, 0, 1, 1]
    # empty input and no events
    keep = ctx.clean_seeds(to_dev(ev.hits), to_dev(ev.hit_off), to_dev(np.zeros((3, 0), np.int32)),
                           to_dev(np.zeros(0, np.int32)))
    assert keep.numel() == 0
    ev0 = dataclasses.replace(ev, hit_off=np.zeros((0, geom.n_layers + 1), np.int64))
    assert np.all(_gpu_clean(ctx, ev0) == 1)


def test_clean_is_deterministic():
    geom, ev = synth.find_workload(3, n_tracks=3000)
    ev2, _ = synth.inject_duplicate_seeds(geom, ev, 0.2)
    ctx = _ctx(geom)
    a = _gpu_clean(ctx, ev2)
    b = _gpu_clean(ctx, ev2)
    assert np.array_equal(a, b)


def test_remove_duplicates_on_gpu_finder_output():
    geom, ev = synth.find_workload(3, n_tracks=3000)
    ev2, _ = synth.inject_duplicate_seeds(geom, ev, 0.1)
    ctx = _ctx(geom)
    _, tc = _cuts_of(ctx)
    d = {k: to_dev(getattr(ev2, k)) for k in ("hits", "hit_off", "seed_hits", "seed_event")}
    out = ctx.find(d["hits"], d["hit_off"], d["seed_hits"], d["seed_event"],
                   xX0=to_dev(geom.xX0.astype(np.float32)), refit=True)
    keep = ctx.remove_duplicates(d["hits"], 1, d["seed_event"], out["hit_idx"][0].contiguous(),
                                 out["n_hits"][0].contiguous(), out["chi2"][0].contiguous(), out["rf_state"])
    torch.cuda.synchronize()
    g = keep.cpu().numpy()
    r, sens = oracle.remove_duplicates(geom, ev2.hits, 1, ev2.seed_event, out["hit_idx"][0].cpu().numpy(),
                                       out["n_hits"][0].cpu().numpy(), out["chi2"][0].cpu().numpy(),
                                       out["rf_state"].cpu().numpy(), cuts=tc)
    _compare(g, r, sens, "removal on the finder's rank-0 candidates, 3000 tracks + 10% duplicates")
    # the duplicate rate (a reference track matched by more than one kept track) drops
    # to zero and no reference track loses its match
    hi, nh = out["hit_idx"][0].cpu().numpy(), out["n_hits"][0].cpu().numpy()
    rate0, eff0 = _dup_rate_and_eff(ev2, hi, nh, np.ones(g.size, bool))
    rate, eff = _dup_rate_and_eff(ev2, hi, nh, g == 1)
    print(f"duplicate rate {rate0:.3f} -> {rate:.3f}, efficiency {eff0:.4f} -> {eff:.4f}")
    assert rate0 > 0.05 and rate == 0.0 and eff == eff0


def _dup_rate_and_eff(ev, hit_idx, n_hits, sel):
    """As the oracle's pin: reference tracks with >= 12 hits, kept tracks with >= 10
    hits matched to the true track giving at least half of their non-seed hits."""
    T = ev.track_hits.shape[1]
    ref = (ev.track_hits >= 0).sum(0) >= 12
    counts = np.zeros(T, int)
    for i in np.nonzero(sel & (n_hits >= 10))[0]:
        hs = hit_idx[3:, i]
        hs = hs[hs >= 0]
        tr = ev.hit_track[hs]
        ids, c = np.unique(tr[tr >= 0], return_counts=True)
        if ids.size and c.max() >= 0.5 * hs.size:
            counts[ids[np.argmax(c)]] += 1
    return (counts[ref] > 1).mean(), (counts[ref] >= 1).mean()


def test_remove_duplicates_edge_cases():
    geom = synth.workload_geometry(2)
    L = geom.n_layers
    ctx = _ctx(geom)
    ev = _tiny(geom)
    hit_idx = np.full((L, 5), -1, np.int32)
    hit_idx[0] = [0, 0, 2, 0, 0]
    hit_idx[1] = [4, 4, 5, 4, 4]
    hit_idx[3:, 0] = 100 + np.arange(3, L)
    hit_idx[3:, 1] = 100 + np.arange(3, L)
    hit_idx[3:8, 3] = 100 + np.arange(3, 8)
    n_hits = (hit_idx >= 0).sum(0).astype(np.int32)
    n_hits[4] = 0                                      # no track: kept, takes no part
    chi2 = np.array([3.0, 3.0, 1.0, 0.5, 0.1], np.float32)
    state = np.zeros((6, 5), np.float32)
    state[3] = 0.3
    state[5] = 1.0
    ev_idx = np.zeros(5, np.int32)
    _, tc = _cuts_of(ctx)
    g = ctx.remove_duplicates(to_dev(ev.hits), 1, to_dev(ev_idx), to_dev(hit_idx), to_dev(n_hits), to_dev(chi2),
                              to_dev(state)).cpu().numpy()
    r, sens = oracle.remove_duplicates(geom, ev.hits, 1, ev_idx, hit_idx, n_hits, chi2, state, cuts=tc)
    assert not sens.any()
    assert np.array_equal(g, r) and g.tolist() == [1, 0, 1, 0, 1], (g, r)
