"""Pins of the oracle's endcap model (no GPU): disk planes, bounded surfaces, eta regions.

A disk is the plane z = z_d, active between two radii; a bounded cylinder is active for
|z| <= Z.  A bounded surface that a track crosses outside its active area, or does not
reach, is passed over: no hit, no material, no miss.  The generator (synth) implements
the same detector independently, in numpy.
"""
import math

import numpy as np
import pytest

import oracle
import physics
import synth


def _wrap(a):
    return (a + math.pi) % (2 * math.pi) - math.pi


def test_plane_crossing_is_on_helix_and_plane(oracle_lib):
    """The crossing with z = z_d lies on the plane and on the helix at transverse arc
    s = (z_d - z) tan(theta); a plane behind the track, or beyond half a turn, has none."""
    rng = np.random.default_rng(21)
    B = 3.8
    kB = 0.299792458e-2 * B
    n_ok = 0
    for _ in range(200):
        th = rng.uniform(0.05, 0.8)
        x = np.array([rng.normal(0, 5), rng.normal(0, 5), rng.uniform(-20, 20), rng.uniform(-1, 1),
                      rng.uniform(-3, 3), th])
        zd = rng.uniform(60, 300)
        out, s = oracle.propagate_disk(x, zd, B)
        s_exp = (zd - x[2]) * math.tan(th)
        half_turn = abs(kB * x[3] * s_exp) >= math.pi
        if half_turn:
            assert out is None
            continue
        n_ok += 1
        assert s == pytest.approx(s_exp, rel=1e-14)
        assert out[2] == pytest.approx(zd, abs=1e-11)
        px, py, pz, ph = physics.helix_point(x, s_exp, kB)
        np.testing.assert_allclose(out[:2], [px, py], rtol=0, atol=1e-10)
        assert abs(_wrap(out[4] - ph)) < 1e-12
        assert out[3] == x[3] and out[5] == x[5]
        # the mirrored plane lies behind
        back, _ = oracle.propagate_disk(x, -zd, B)
        assert back is None
    assert n_ok > 100


def test_disk_measurement_matrix_is_tangent_projection(oracle_lib):
    """H of a disk = derivative of the local (z, rho0*dphi, rho) coordinates of the point
    where the state's 3-D tangent line meets the plane, for a state on the plane; the
    residual is (z_m - z_p, rho_p * dphi, rho_m - rho_p)."""
    rng = np.random.default_rng(22)
    for _ in range(60):
        c = np.array([rng.normal(0, 0.1), rng.normal(0, 0.1)])
        zd = rng.choice([-1, 1]) * rng.uniform(100, 300)
        rho0 = rng.uniform(20, 110)
        a = rng.uniform(-3, 3)
        th = rng.uniform(0.1, 0.9) if zd > 0 else rng.uniform(math.pi - 0.9, math.pi - 0.1)
        x = np.array([c[0] + rho0 * math.cos(a), c[1] + rho0 * math.sin(a), zd, rng.uniform(-2, 2),
                      a + rng.uniform(-1.0, 1.0), th])

        def local(xx):
            cot = 1 / math.tan(xx[5])
            mu = (zd - xx[2]) / cot
            qx = xx[0] + mu * math.cos(xx[4]) - c[0]
            qy = xx[1] + mu * math.sin(xx[4]) - c[1]
            dph = _wrap(math.atan2(qy, qx) - a)
            return np.array([zd, rho0 * dph, math.hypot(qx, qy)])

        Hn = np.zeros((3, 6))
        for j in range(6):
            h = 1e-6
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            Hn[:, j] = (local(xp) - local(xm)) / (2 * h)
        m = np.array([c[0] + (rho0 + 0.3) * math.cos(a + 0.01), c[1] + (rho0 + 0.3) * math.sin(a + 0.01), zd])
        H, r = oracle.measurement_disk(x, c, zd, m)
        np.testing.assert_allclose(H, Hn, rtol=1e-6, atol=2e-6)
        np.testing.assert_allclose(r, [0.0, rho0 * 0.01, 0.3], rtol=1e-9, atol=1e-9)


def test_disk_scattering_matches_generator_kicks(oracle_lib):
    """Q on a disk = covariance of the generator's kicks there (the path through the
    plane is x/X0 / |cos theta|: at eta 1.1 a unit path would be 27% short in variance)."""
    geom = synth.Geometry(radius=[4.0, 100.0], zhalf=[200.0, 200.0], xX0=[0.0, 0.03], disk_z=[0.0, 150.0],
                          disk_rmin=[0.0, 10.0], disk_rmax=[0.0, 140.0], cyl_zmax=[200.0, 0.0])
    n = 200_000
    for (pt, eta, phi, q) in [(0.8, 1.1, 0.4, 1.0), (3.0, 2.2, -2.0, -1.0)]:
        parts = (np.full(n, pt), np.full(n, phi), np.full(n, eta), np.full(n, q))
        pre = synth.simulate(geom, synth.rng_for(97), n, particles=parts, scatter=False, keep_truth=True)
        post = synth.simulate(geom, synth.rng_for(97), n, particles=parts, scatter=True, keep_truth=True)
        assert np.all(pre.hit_mask == 3)
        d = post.truth[1][[3, 4, 5]] - pre.truth[1][[3, 4, 5]]
        emp = np.cov(d)
        Q = oracle.scattering(geom, pre.truth[1][:, 0], (0.0, 0.0), 0.03, zd=150.0)[3:, 3:]
        for a in range(3):
            for b in range(3):
                scale = math.sqrt(Q[a, a] * Q[b, b])
                assert abs(emp[a, b] - Q[a, b]) < 0.02 * scale, (a, b, emp[a, b], Q[a, b])


def _truth_at_last(ts):
    n = ts.hits.shape[2]
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    return last, ts.truth[last, :, np.arange(n)].T


def test_noiseless_endcap_tracks_return_generating_helix(oracle_lib):
    """Noiseless hits, no material, |eta| < 2.5: the fit passes over the surfaces the
    track misses and ends on the generating helix at its last (cylinder or disk) hit."""
    geom = synth.barrel_endcap()
    n = 400
    ts = synth.simulate(geom, synth.rng_for(94), n, (0.5, 50.0), True, 2.5, smear=False, scatter=False,
                        hit_dtype=np.float64)
    last, tr = _truth_at_last(ts)
    assert np.mean(geom.is_disk[last]) > 0.3   # many tracks end on a disk
    o = oracle.fit(geom, ts.hits, ts.hit_mask)
    ok = o["status"] & oracle.ST_PROP_FAIL == 0
    assert ok.mean() > 0.95
    assert np.all(o["chi2"][ok] < 1e-12)
    d = o["state"] - tr
    d[4] = _wrap(d[4])
    assert np.max(np.abs(d[:3, ok])) < 1e-8
    assert np.max(np.abs(d[3, ok] / tr[3, ok])) < 1e-8
    assert np.max(np.abs(d[4:, ok])) < 1e-10
    nh = np.array([bin(int(m)).count("1") for m in ts.hit_mask])
    np.testing.assert_array_equal(o["ndf"][ok], 2 * nh[ok] - 5)


def _diffuse_seeds(geom, ts, factor):
    n = ts.hits.shape[2]
    ss = np.zeros((6, n), np.float32)
    sc = np.zeros((21, n), np.float32)
    for i in range(n):
        st, cv = oracle.seed(geom, ts.hits[0, :, i].astype(float), ts.hits[1, :, i].astype(float),
                             ts.hits[2, :, i].astype(float))
        ss[:, i] = st
        sc[:, i] = [cv[a, b] * factor for a in range(6) for b in range(a + 1)]
    return ss, sc


def test_endcap_pulls_and_chi2_unit_scale(oracle_lib):
    """Smeared, scattered barrel-and-endcap tracks (x/X0 = 0.02 per surface, 1/|cos theta|
    path on a disk): chi2/ndf = 1 and unit pulls of the state projected onto its last
    surface, separately for tracks ending on a cylinder and on a disk."""
    geom = synth.barrel_endcap(xX0=0.02)
    ts = synth.simulate(geom, synth.rng_for(95), 6000, (0.5, 50.0), True, 2.5, keep_truth=True)
    n = ts.hits.shape[2]
    last, tr = _truth_at_last(ts)
    ss, sc = _diffuse_seeds(geom, ts, 1e3)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=ss, seed_cov=sc)
    ok = o["status"] == 0
    assert ok.mean() > 0.9
    r = o["chi2"][ok] / o["ndf"][ok]
    assert abs(r.mean() - 1.0) < 0.03
    Cm = oracle.unpack_cov(o["cov"])
    disk = geom.is_disk[last]
    for sel, proj in ((~disk, "cyl"), (disk, "disk")):
        idx = np.nonzero(sel & ok)[0]
        assert idx.shape[0] > 1000, proj
        if proj == "cyl":
            xp, Cp = physics.project_to_surface(o["state"][:, idx], Cm[:, :, idx], geom.radius[last[idx]], geom.k_B)
        else:
            xp, Cp = physics.project_to_plane(o["state"][:, idx], Cm[:, :, idx], geom.disk_z[last[idx]], geom.k_B)
        for p, v in physics.pulls(xp, Cp, tr[:, idx], idx=(3, 4, 5)).items():
            assert abs(v.mean()) < 0.06, (proj, p, v.mean())
            assert abs(v.std() - 1.0) < 0.06, (proj, p, v.std())
        if proj == "disk":   # the transverse position on the plane
            for p, v in physics.pulls(xp, Cp, tr[:, idx], idx=(0, 1)).items():
                assert abs(v.std() - 1.0) < 0.06, (proj, p, v.std())


def test_passed_surfaces_leave_no_trace(oracle_lib):
    """A hitless bounded surface is passed over: fitting a track in the full geometry
    equals fitting it in the geometry of its hit surfaces alone, material included."""
    geom = synth.barrel_endcap(xX0=0.02)
    ts = synth.simulate(geom, synth.rng_for(96), 60, (0.5, 50.0), True, 2.5)
    o = oracle.fit(geom, ts.hits, ts.hit_mask)
    for i in range(60):
        keep = [l for l in range(geom.n_layers) if int(ts.hit_mask[i]) >> l & 1]
        sub = synth.Geometry(radius=geom.radius[keep], zhalf=geom.zhalf[keep], B=geom.B, xX0=geom.xX0[keep],
                             disk_z=geom.disk_z[keep], disk_rmin=geom.disk_rmin[keep],
                             disk_rmax=geom.disk_rmax[keep], cyl_zmax=geom.cyl_zmax[keep])
        h = np.ascontiguousarray(ts.hits[keep][:, :, i:i + 1])
        f = oracle.fit(sub, h, np.array([(1 << len(keep)) - 1], np.uint32))
        np.testing.assert_allclose(f["state"][:, 0], o["state"][:, i], rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(f["cov"][:, 0], o["cov"][:, i], rtol=1e-12, atol=1e-16)
        assert f["chi2"][0] == pytest.approx(o["chi2"][i], rel=1e-12, abs=1e-14)


def test_endcap_seeds_grouped_by_eta_region(oracle_lib):
    """Within an event, endcap seeds come in eta-region order: barrel, transition, endcap."""
    geom, ev = synth.endcap_find_workload(n_tracks=600)
    p2 = ev.seed_hits[2]
    eta = np.arcsinh(ev.hits[2, p2].astype(np.float64) / np.hypot(*ev.hits[:2, p2].astype(np.float64)))
    reg = synth.eta_region(eta)
    assert np.all(np.diff(reg) >= 0)
    assert set(np.unique(reg)) == {0, 1, 2}


def test_endcap_binned_search_equals_brute_force(oracle_lib):
    """On disks the bins run over phi and radius: scanning the bins that overlap each
    window gives exactly the brute-force result."""
    geom, ev = synth.endcap_find_workload(n_tracks=300)
    ob = oracle.find(geom, ev)
    oB = oracle.find(geom, ev, brute=True)
    for k in ob:
        np.testing.assert_array_equal(ob[k], oB[k], err_msg=k)
    # candidates end on disks, and pass over surfaces (-2 between hits)
    h = ob["hit_idx"][0]
    hit_disk = (h >= 0) & geom.is_disk[:, None]
    assert hit_disk.any(axis=0).mean() > 0.3
    passed_mid = [(np.nonzero(h[:, s] >= 0)[0].max() > np.nonzero(h[:, s] == -2)[0].min())
                  for s in range(h.shape[1]) if np.any(h[:, s] == -2)]
    assert np.mean(passed_mid) > 0.3


def test_noiseless_endcap_event_finds_the_truth(oracle_lib):
    """No smearing, scattering or noise, keep 1: the best candidate of (nearly) every
    seed holds exactly its track's hits, on cylinders and disks, and no misses."""
    geom = synth.barrel_endcap()
    ev = synth.make_events(geom, [300], workload=12, noise_frac=0.0, smear=False, scatter=False, eta_max=2.5)
    o = oracle.find(geom, ev, keep=1)
    S = ev.seed_hits.shape[1]
    n_ok = 0
    for s in range(S):
        th = ev.track_hits[:, ev.seed_track[s]]
        h = o["hit_idx"][0, :, s]
        if np.all(np.where(th >= 0, h == th, h < 0)):
            n_ok += 1
    assert n_ok >= S - 2
    assert np.mean(o["n_miss"][0] == 0) > 0.98
