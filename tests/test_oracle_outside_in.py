"""Pins of the oracle's outside-in fit (no GPU): the backward filter of the reversed
particle, from the outermost hit inwards, against the forward filter and the smoother."""
import math

import numpy as np
import pytest

import oracle
import physics
import synth


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


def _diffuse_seeds(geom, ts, factor):
    n = ts.hits.shape[2]
    ss = np.zeros((6, n))
    sc = np.zeros((21, n))
    for i in range(n):
        st, cv = oracle.seed(geom, ts.hits[0, :, i].astype(float), ts.hits[1, :, i].astype(float),
                             ts.hits[2, :, i].astype(float))
        ss[:, i] = st
        sc[:, i] = [cv[a, b] * factor for a in range(6) for b in range(a + 1)]
    return ss, sc


def _outer_seeds(geom, ts, factor):
    """The helix through each track's three outermost hits (taken outermost first, so
    oriented inwards), reversed to the particle's own direction, with its prior
    inflated `factor` times."""
    n = ts.hits.shape[2]
    ss = np.zeros((6, n))
    sc = np.zeros((21, n))
    for i in range(n):
        m = int(ts.hit_mask[i]).bit_length() - 1
        st, cv = oracle.seed(geom, *(ts.hits[l, :, i].astype(float) for l in (m, m - 1, m - 2)))
        x, c = oracle.reverse_state(st[:, None], np.array([[cv[a, b] * factor] for a in range(6) for b in range(a + 1)]))
        ss[:, i] = x[:, 0]
        sc[:, i] = c[:, 0]
    return ss, sc


def _inflate(cov, factor):
    c = np.array(cov, np.float64)
    return c * factor


def test_reversal_is_an_involution_and_traces_the_same_helix(oracle_lib):
    """reverse_state twice is the identity; the reversed state's helix run forward by s
    reaches the point the original reaches at -s."""
    rng = np.random.default_rng(31)
    B = 3.8
    kB = 0.299792458e-2 * B
    for _ in range(50):
        x = np.array([rng.normal(0, 30), rng.normal(0, 30), rng.normal(0, 50), rng.uniform(-2, 2),
                      rng.uniform(-3, 3), rng.uniform(0.3, 2.8)])
        cv = rng.normal(size=21)
        xr, cr = oracle.reverse_state(x[:, None], cv[:, None])
        xx, cc = oracle.reverse_state(xr, cr)
        np.testing.assert_allclose(xx[:, 0], x, rtol=0, atol=1e-12)
        np.testing.assert_allclose(cc[:, 0], cv, rtol=0, atol=0)
        s = rng.uniform(1, 40)
        a = oracle.helix_at(xr[:, 0], s, B)
        b = oracle.helix_at(x, -s, B)
        np.testing.assert_allclose(a[:3], b[:3], rtol=0, atol=1e-9)


def test_outside_in_equals_forward_fit_on_straight_lines(oracle_lib):
    """B = 0, no material, small hit errors (the linear regime): both filters, from wide
    priors, fit the same straight line to the same hits, so the direction (phi, theta),
    its covariance and chi2 agree (the forward filter is pinned against linear weighted
    least squares)."""
    geom = synth.barrel(10, 5.0, 100.0, B=0.0, xX0=0.0, eta_max=1.0, sigma_rphi=1e-5, sigma_z=2e-5)
    n = 300
    ts = synth.simulate(geom, synth.rng_for(96), n, (1.0, 5.0), False, 1.0, scatter=False, hit_dtype=np.float64)
    # each filter starts from the generating state at its first layer with a prior wide
    # enough to weigh ~1e-4 of the hits (kappa is free at B = 0)
    ps = np.array([1e-3, 1e-3, 1e-3, 1.0, 1e-4, 1e-4])
    covs = np.array([[(ps[a] ** 2 if a == b else 0.0) for a in range(6) for b in range(a + 1)]] * n).T
    assert np.all(ts.hit_mask == (1 << geom.n_layers) - 1)
    f = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=ts.truth[0], seed_cov=covs)
    b = oracle.fit_outside_in(geom, ts.hits, ts.hit_mask, ts.truth[-1], covs)
    ok = (f["status"] == 0) & (b["status"] == 0)
    assert ok.mean() > 0.95
    Cf, Cb = oracle.unpack_cov(f["cov"]), oracle.unpack_cov(b["cov"])
    for p in (4, 5):
        d = f["state"][p] - b["state"][p]
        if p == 4:
            d = _wrap(d)
        sig = np.sqrt(Cf[p, p])
        assert np.max(np.abs(d[ok]) / sig[ok]) < 1e-3, p
        np.testing.assert_allclose(np.sqrt(Cb[p, p][ok]), sig[ok], rtol=1e-3)
    np.testing.assert_allclose(b["chi2"][ok], f["chi2"][ok], rtol=2e-3, atol=2e-3)
    np.testing.assert_array_equal(b["ndf"], f["ndf"])


def _pair(geom, n, workload):
    ts = synth.simulate(geom, synth.rng_for(workload), n, (0.5, 50.0), True, 1.5, keep_truth=True,
                        hit_dtype=np.float64)
    ss, sc = _diffuse_seeds(geom, ts, 1e3)
    f = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=ss, seed_cov=sc)
    sm = oracle.smooth(geom, ts.hits, ts.hit_mask, seed_state=ss, seed_cov=sc)
    # the outside-in fit seeded alike: the helix through the three outermost hits, its
    # prior inflated a thousand times (in the particle's own direction)
    bs, bc = _outer_seeds(geom, ts, 1e3)
    b = oracle.fit_outside_in(geom, ts.hits, ts.hit_mask, bs, bc)
    ok = (f["status"] == 0) & (b["status"] == 0) & (sm["lend"] >= 1)
    # projected onto the layer-0 surface along their own helices: a state keeps its
    # prior's variance along the track, which no measurement sees
    r0 = geom.radius[0]
    x_s, C_s = physics.project_to_surface(sm["state"][0], oracle.unpack_cov(sm["cov"][0]), r0, geom.k_B)
    x_b, C_b = physics.project_to_surface(b["state"], oracle.unpack_cov(b["cov"]), r0, geom.k_B)
    d = x_b - x_s
    d[4] = _wrap(d[4])
    sig_s = np.sqrt(np.einsum("iin->in", C_s))
    sig_b = np.sqrt(np.einsum("iin->in", C_b))
    return ts, ok, x_b, sig_b, np.abs(d) / sig_s, sig_b / sig_s


def test_outside_in_innermost_estimate_equals_smoother_in_the_linear_limit(oracle_lib):
    """B = 3.8 T, no material, hit errors a hundred times smaller (the linearisations of
    the two passes then coincide): the outside-in estimate at layer 0 equals the
    smoother's there, projected onto the layer-0 surface (state and errors)."""
    geom = synth.workload_geometry(2)
    geom.xX0[:] = 0.0
    geom.sigma_rphi *= 0.01
    geom.sigma_z *= 0.01
    _, ok, _, _, r, ratio = _pair(geom, 800, 98)
    assert ok.mean() > 0.9
    print("max |outside-in - smoother| / sigma per parameter", np.array2string(r[:, ok].max(axis=1), precision=1))
    assert r[:, ok].max() < 1e-2
    dev = np.abs(ratio[:, ok] - 1.0)
    print("median, max |sigma ratio - 1| per parameter", np.array2string(np.median(dev, axis=1), precision=1),
          np.array2string(dev.max(axis=1), precision=1))
    assert np.all(np.median(dev, axis=1) < 2e-3) and dev.max() < 0.05


def test_outside_in_innermost_estimate_against_smoother_and_truth(oracle_lib):
    """B = 3.8 T, x/X0 = 0.02 on every layer but the innermost, the workload's hit
    errors: the two estimates at layer 0 (same hits, same scattering) differ by the two
    passes' linearisations, a small fraction of a sigma (median; measured 0.03-0.08),
    carry the same errors, and both have unit pulls against the truth there."""
    geom = synth.workload_geometry(2)
    geom.xX0[0] = 0.0
    ts, ok, x_b, sig_b, r, ratio = _pair(geom, 1500, 97)
    assert ok.mean() > 0.9
    med = np.median(r[:, ok], axis=1)
    print("median |outside-in - smoother| / sigma per parameter", np.array2string(med, precision=3))
    assert np.all(med < 0.12)
    assert np.all(np.abs(np.median(ratio[:, ok], axis=1) - 1.0) < 0.02)
    tr = ts.truth[0]
    for p in range(6):
        d = x_b[p] - tr[p]
        if p == 4:
            d = _wrap(d)
        pull = d[ok] / sig_b[p, ok]
        assert abs(pull.mean()) < 0.08 and abs(pull.std() - 1.0) < 0.08, (p, pull.mean(), pull.std())
