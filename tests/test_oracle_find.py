"""Pins of the oracle's combinatorial finder (no GPU): brute force and special cases."""
import numpy as np

import oracle
import synth


def test_binned_search_equals_brute_force(oracle_lib):
    """Scanning only the phi/z bins that overlap each window gives exactly the result of
    testing every hit of the layer (including the ambiguity log)."""
    geom, ev = synth.find_workload(3, n_tracks=400)
    ob = oracle.find(geom, ev)
    oB = oracle.find(geom, ev, brute=True)
    for k in ob:
        np.testing.assert_array_equal(ob[k], oB[k], err_msg=k)


def test_binned_equals_brute_force_with_wide_windows(oracle_lib):
    """Large windows (many sigma) wrap around in phi and clamp in z."""
    geom, ev = synth.find_workload(3, n_tracks=150)
    ob = oracle.find(geom, ev, nsigma=400.0, chi2_cut=60.0)
    oB = oracle.find(geom, ev, nsigma=400.0, chi2_cut=60.0, brute=True)
    for k in ob:
        np.testing.assert_array_equal(ob[k], oB[k], err_msg=k)


def test_noiseless_event_finds_the_truth(oracle_lib):
    """No smearing, no scattering, no noise hits, keep 1: the best candidate of every
    seed is its own track, and its state is the fit of exactly those hits."""
    geom = synth.workload_geometry(2)
    geom.xX0[:] = 0.0
    ev = synth.make_events(geom, [300], workload=3, noise_frac=0.0, smear=False, scatter=False)
    o = oracle.find(geom, ev, keep=1)
    S = ev.seed_hits.shape[1]
    L = geom.n_layers
    n_ok = 0
    for s in range(S):
        th = ev.track_hits[:, ev.seed_track[s]]
        h = o["hit_idx"][0, :, s]
        reached = th >= 0
        if np.all(h[reached] == th[reached]):
            n_ok += 1
    assert n_ok >= S - 1
    # state of the rank-0 candidate == oracle fit of the same hits
    hits = np.full((L, 3, S), np.nan, np.float32)
    mask = np.zeros(S, np.uint32)
    for s in range(S):
        for l in range(L):
            j = o["hit_idx"][0, l, s]
            if j >= 0:
                hits[l, :, s] = ev.hits[:, j]
                mask[s] |= np.uint32(1 << l)
    f = oracle.fit(geom, hits, mask)
    full = (o["n_miss"][0] == 0) & (o["status"][0] == 0)
    np.testing.assert_allclose(o["state"][0][:, full], f["state"][:, full], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(o["chi2"][0][full], f["chi2"][full], rtol=1e-9, atol=1e-12)


def test_candidates_respect_rules(oracle_lib):
    """At most `keep` candidates, ranked by (hits desc, chi2 asc); a candidate stops at
    the max_miss-th missing layer; every accepted hit lies on its layer."""
    geom, ev = synth.find_workload(3, n_tracks=300)
    keep, max_miss = 6, 3
    o = oracle.find(geom, ev, keep=keep, max_miss=max_miss)
    S = ev.seed_hits.shape[1]
    L = geom.n_layers
    for s in range(S):
        nc = o["n_cand"][s]
        assert 1 <= nc <= keep
        keys = [(-o["n_hits"][k, s], o["chi2"][k, s]) for k in range(nc)]
        assert keys == sorted(keys)
        for k in range(nc):
            h = o["hit_idx"][k, :, s]
            assert np.sum(h == -1) == o["n_miss"][k, s] <= max_miss
            assert np.sum(h >= 0) == o["n_hits"][k, s]
            for l in range(L):
                if h[l] >= 0:
                    assert ev.hit_off[0, l] <= h[l] < ev.hit_off[0, l + 1]
            if o["n_miss"][k, s] == max_miss:
                last_miss = np.nonzero(h == -1)[0].max()
                assert np.all(h[last_miss + 1:] == -2)
