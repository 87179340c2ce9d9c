"""Pins of the oracle's duplicate handling (seed cleaning and post-build removal).

* Injected duplicate seeds (a second measurement of one, two or all three of a true
  seed's hits, as overlapping modules give): cleaning removes every duplicate that
  shares two hits with its original and nearly every one that shares one, and no
  original seed (real tracks share no hits); duplicates sharing no hit are left to
  the post-build step.
* The whole chain (cleaning, building the kept seeds, removal) brings the duplicate
  rate, defined as in the paper (a reference track matched by more than one
  reconstructed track; matching by at least half of the non-seed hits), from ~9% to 0
  without losing efficiency.
* Hand-built cases: the priority order (more hits, lower chi2, lower index), events
  never interact, the azimuth window wraps at +-pi, identical copies leave one.
"""
import dataclasses
import math

import numpy as np

import oracle
import synth


def _variants(dup_of):
    d = np.nonzero(dup_of >= 0)[0]
    return d, np.arange(d.size) % 5


def test_cleaning_removes_injected_duplicate_seeds(oracle_lib):
    geom, ev = synth.find_workload(3)
    ev2, dup_of = synth.inject_duplicate_seeds(geom, ev, 0.1)
    keep, sens = oracle.clean_seeds(geom, ev2)
    inj = dup_of >= 0
    d, var = _variants(dup_of)
    assert inj.sum() > 400
    assert np.all(keep[~inj] == 1)                      # no original seed is lost
    for v in (0, 1, 2):                                 # two shared hits
        assert np.all(keep[d[var == v]] == 0), v
    assert np.mean(keep[d[var == 3]] == 0) > 0.95       # one shared hit + kinematics
    assert np.all(keep[d[var == 4]] == 1)               # no shared hit: not a seed-level duplicate
    assert sens.sum() <= 5


def _dup_rate_and_eff(ev, hit_idx, n_hits, sel):
    """Duplicate rate and efficiency over reference tracks (>= 12 hits), counting
    reconstructed tracks with >= 10 hits, matched to the true track that gives at least
    half of their hits outside the seed layers."""
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


def test_chain_removes_duplicates_without_losing_efficiency(oracle_lib):
    geom, ev = synth.find_workload(3, n_tracks=2000)
    r0 = oracle.find(geom, ev)
    _, eff0 = _dup_rate_and_eff(ev, r0["hit_idx"][0], r0["n_hits"][0], np.ones(ev.seed_hits.shape[1], bool))
    ev2, dup_of = synth.inject_duplicate_seeds(geom, ev, 0.1)
    S = ev2.seed_hits.shape[1]
    r = oracle.find(geom, ev2)
    rate_raw, eff_raw = _dup_rate_and_eff(ev2, r["hit_idx"][0], r["n_hits"][0], np.ones(S, bool))
    assert rate_raw > 0.05
    keep_s, _ = oracle.clean_seeds(geom, ev2)
    sel = np.nonzero(keep_s == 1)[0]
    ev3 = dataclasses.replace(ev2, seed_hits=np.ascontiguousarray(ev2.seed_hits[:, sel]),
                              seed_event=ev2.seed_event[sel], seed_track=ev2.seed_track[sel])
    r3 = oracle.find(geom, ev3, refit=True)
    keep_t, sens = oracle.remove_duplicates(geom, ev3.hits, 1, ev3.seed_event, r3["hit_idx"][0],
                                            r3["n_hits"][0], r3["chi2"][0].astype(np.float32),
                                            r3["rf_state"].astype(np.float32))
    rate, eff = _dup_rate_and_eff(ev3, r3["hit_idx"][0], r3["n_hits"][0], keep_t == 1)
    assert rate == 0.0
    assert abs(eff - eff0) < 1e-9 and abs(eff_raw - eff0) < 1e-9
    assert sens.sum() <= 2


def _tiny_event(geom, angles0, angles12, z=0.0):
    """One event: hits on layers 0-2 at the given azimuths (layer 0 list, then one
    azimuth shared by layers 1 and 2 per track), radial straight-line positions."""
    L = geom.n_layers
    per_layer = [list(angles0), list(angles12), list(angles12)]
    hits, off = [], [0]
    for l in range(L):
        angs = per_layer[l] if l < 3 else []
        r = geom.radius[l]
        for a in angs:
            hits.append((r * math.cos(a), r * math.sin(a), z + 0.1 * r))
        off.append(off[-1] + len(angs))
    H = len(hits)
    return synth.EventBatch(hits=np.ascontiguousarray(np.array(hits, np.float32).T),
                            hit_off=np.array([off], np.int64), hit_track=np.full(H, -1, np.int64),
                            seed_hits=np.zeros((3, 0), np.int32), seed_event=np.zeros(0, np.int32),
                            seed_track=np.zeros(0, np.int64), track_event=np.zeros(0, np.int32),
                            track_hits=np.zeros((L, 0), np.int64), n_tracks=np.array([0]))


def test_cleaning_wraps_the_azimuth_window_and_keeps_events_apart(oracle_lib):
    geom = synth.workload_geometry(2)
    # layer 0 hits at pi - 0.001 and -pi + 0.001 (0.002 apart across the wrap), one
    # shared pair of layer-1/2 hits at pi - 0.001
    ev = _tiny_event(geom, [math.pi - 0.001, -math.pi + 0.001], [math.pi - 0.001])
    o = ev.hit_off[0]
    s = np.array([[o[0], o[0] + 1, o[0], o[0]], [o[1]] * 4, [o[2]] * 4], np.int32)
    ev = dataclasses.replace(ev, seed_hits=s, seed_event=np.zeros(4, np.int32))
    keep, sens = oracle.clean_seeds(geom, ev)
    # seed 1 shares hits 1, 2 with seed 0 across the wrap; seeds 2, 3 are copies of 0
    assert keep.tolist() == [1, 0, 0, 0] and not sens.any()
    # the same seeds split over two events (event 1 repeats event 0's hits): a seed
    # only meets the seeds of its own event
    ev2 = dataclasses.replace(ev, hits=np.concatenate([ev.hits, ev.hits], axis=1),
                              hit_off=np.stack([ev.hit_off[0], ev.hit_off[0] + ev.hits.shape[1]]))
    H = ev.hits.shape[1]
    s2 = np.concatenate([s[:, :2], s[:, :2] + H], axis=1).astype(np.int32)
    ev2 = dataclasses.replace(ev2, seed_hits=s2, seed_event=np.array([0, 0, 1, 1], np.int32))
    keep2, _ = oracle.clean_seeds(geom, ev2)
    assert keep2.tolist() == [1, 0, 1, 0]


def test_removal_priority_order(oracle_lib):
    geom = synth.workload_geometry(2)
    L = geom.n_layers
    ev = _tiny_event(geom, [0.3, 0.31], [0.3])
    # four tracks over made-up hit indices on layers 0-2 (placed hits exist there) and
    # invented indices beyond (only equality matters for sharing)
    hit_idx = np.full((L, 4), -1, np.int32)
    base = np.arange(3, L)
    hit_idx[0] = [0, 0, 1, 0]
    hit_idx[1] = [2, 2, 2, 2]
    hit_idx[2] = [3, 3, 3, 3]
    hit_idx[3:, 0] = 1000 + base          # 17 hits
    hit_idx[3:, 1] = 1000 + base          # the same 17 hits, higher chi2
    hit_idx[3:12, 2] = 1000 + base[:9]    # 12 hits, 11 shared with track 0
    hit_idx[3:, 3] = 2000 + base          # 17 hits, 3 shared: not a duplicate
    n_hits = (hit_idx >= 0).sum(0).astype(np.int32)
    chi2 = np.array([10.0, 12.0, 1.0, 5.0], np.float32)
    state = np.zeros((6, 4), np.float32)
    state[3] = 0.5
    state[5] = 1.2
    keep, sens = oracle.remove_duplicates(geom, ev.hits, 1, np.zeros(4, np.int32), hit_idx, n_hits, chi2, state)
    assert keep.tolist() == [1, 0, 0, 1] and not sens.any()
    # equal hits and chi2: the lower index wins
    chi2[1] = chi2[0]
    keep, _ = oracle.remove_duplicates(geom, ev.hits, 1, np.zeros(4, np.int32), hit_idx, n_hits, chi2, state)
    assert keep.tolist() == [1, 0, 0, 1]
    # a kinematic disagreement (a crossing track sharing hits) keeps both
    state[3, 1] = -0.5
    keep, _ = oracle.remove_duplicates(geom, ev.hits, 1, np.zeros(4, np.int32), hit_idx, n_hits, chi2, state)
    assert keep.tolist() == [1, 1, 0, 1]
