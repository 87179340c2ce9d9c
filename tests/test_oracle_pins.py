"""Pins of the FP64 oracle against facts fixed by the mathematics (no GPU).

Each test checks the oracle against something other than itself: a textbook
identity, a closed form, an independent construction in this file, brute force,
or a Monte-Carlo invariant of the simulated data.
"""
import math

import numpy as np
import pytest

import oracle
import physics
import synth


def _spd(rng, n, scale=1.0):
    A = rng.normal(size=(n, n))
    return scale * (A @ A.T + n * np.eye(n))


# --------------------------------------------------------------------------------------
# Kalman algebra: sequential filter on a linear-Gaussian model = batch weighted LSQ
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("with_transition", [False, True])
def test_linear_filter_equals_batch_wls(oracle_lib, with_transition):
    """Gain, Joseph-form covariance and chi2 of the generic update: the filtered
    estimate after K updates equals the weighted least-squares solution with the prior
    as a pseudo-measurement, and the summed chi2 equals the minimum of its objective."""
    rng = np.random.default_rng(7)
    n, m, K = 6, 3, 9
    x0 = rng.normal(size=n)
    P0 = _spd(rng, n)
    F = np.eye(n) + 0.1 * rng.normal(size=(n, n)) if with_transition else np.eye(n)
    xt = rng.normal(size=n)
    Hs = [rng.normal(size=(m, n)) for _ in range(K)]
    Vs = [_spd(rng, m, 0.1) for _ in range(K)]
    # measurement k sees F^(k+1) x_true (transition applied before every update)
    Fk = [np.linalg.matrix_power(F, k + 1) for k in range(K)]
    ys = [H @ Fp @ xt + np.linalg.cholesky(V) @ rng.normal(size=m) for H, Fp, V in zip(Hs, Fk, Vs)]
    x, Cm, tot = x0.copy(), P0.copy(), 0.0
    for H, V, y in zip(Hs, Vs, ys):
        x, Cm = F @ x, F @ Cm @ F.T
        x, Cm, c = oracle.kalman_update(x, Cm, H, V, y - H @ x)
        tot += c
    P0i = np.linalg.inv(P0)
    W = P0i.copy()
    b = P0i @ x0
    for H, Fp, V, y in zip(Hs, Fk, Vs, ys):
        G = H @ Fp
        W += G.T @ np.linalg.solve(V, G)
        b += G.T @ np.linalg.solve(V, y)
    xb0 = np.linalg.solve(W, b)
    chi2b = (xb0 - x0) @ P0i @ (xb0 - x0)
    for H, Fp, V, y in zip(Hs, Fk, Vs, ys):
        res = y - H @ Fp @ xb0
        chi2b += res @ np.linalg.solve(V, res)
    FK = Fk[-1]
    np.testing.assert_allclose(x, FK @ xb0, rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(Cm, FK @ np.linalg.inv(W) @ FK.T, rtol=1e-9, atol=1e-12)
    assert abs(tot - chi2b) <= 1e-9 * chi2b


# --------------------------------------------------------------------------------------
# propagation
# --------------------------------------------------------------------------------------
def _random_states(rng, n, rmax=60.0):
    r = rng.uniform(0, rmax, n)
    a = rng.uniform(-math.pi, math.pi, n)
    pt = 0.5 * 100 ** rng.random(n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(-50, 50, n), q / pt,
                     rng.uniform(-math.pi, math.pi, n), rng.uniform(0.4, 2.7, n)])


def test_straight_line_limit(oracle_lib):
    """B = 0: the crossing is the line-circle root s = -a + sqrt(a^2 - c); at a tiny
    field it is continuous with it."""
    rng = np.random.default_rng(3)
    X = _random_states(rng, 300)
    for i in range(X.shape[1]):
        x = X[:, i]
        c = (rng.normal(0, 0.3), rng.normal(0, 0.3))
        r = 80.0
        ex, ey = x[0] - c[0], x[1] - c[1]
        a = ex * math.cos(x[4]) + ey * math.sin(x[4])
        s_ref = -a + math.sqrt(a * a - (ex * ex + ey * ey - r * r))
        out, s = oracle.propagate(x, c, r, 0.0)
        assert abs(s - s_ref) <= 1e-12 * r
        np.testing.assert_allclose(out[:3], [x[0] + s_ref * math.cos(x[4]), x[1] + s_ref * math.sin(x[4]),
                                             x[2] + s_ref / math.tan(x[5])], rtol=0, atol=1e-10)
        out2, s2 = oracle.propagate(x, c, r, 1e-9)
        assert abs(s2 - s_ref) <= 1e-8 * r


def test_origin_tracks_arc_closed_form(oracle_lib):
    """Tracks from the origin reach radius r after s = 2 R asin(r / 2R)."""
    rng = np.random.default_rng(4)
    kB = synth.K_B_PER_TESLA * 3.8
    for _ in range(300):
        pt = 0.6 * 80 ** rng.random()
        q = rng.choice([-1.0, 1.0])
        x = np.array([0.0, 0.0, 0.0, q / pt, rng.uniform(-3, 3), rng.uniform(0.5, 2.6)])
        R = pt / kB
        r = rng.uniform(1.0, min(110.0, 1.9 * R))
        _, s = oracle.propagate(x, (0.0, 0.0), r, 3.8)
        assert abs(s - 2 * R * math.asin(r / (2 * R))) <= 1e-11 * r


def test_crossing_matches_circle_intersection(oracle_lib):
    """Newton crossing of the oracle = the generator's circle-circle intersection (an
    independent construction), including displaced layer axes."""
    rng = np.random.default_rng(5)
    X = _random_states(rng, 500, rmax=40.0)
    kB = synth.K_B_PER_TESLA * 3.8
    cx, cy, r = 0.01, -0.02, 55.0
    s_g, qx, qy = synth.first_crossing(X[0], X[1], X[4], -kB * X[3], cx, cy, r)
    n_ok = 0
    for i in range(X.shape[1]):
        out, s = oracle.propagate(X[:, i], (cx, cy), r, 3.8)
        if not np.isfinite(s_g[i]):
            assert out is None
            continue
        n_ok += 1
        assert out is not None
        assert abs(s - s_g[i]) <= 1e-9 * r
        assert abs(out[0] - qx[i]) <= 1e-9 * r and abs(out[1] - qy[i]) <= 1e-9 * r
    assert n_ok > 400


@pytest.mark.parametrize("turn", [1, -1])
def test_grazing_crossings_are_found(oracle_lib, turn):
    """A helix whose circle overlaps the layer by 1e-5 .. 1e-3 of its radius crosses it
    over a short arc; one that falls short by as much does not.  Built from the circle
    geometry: centre at distance d from the axis, radius R, d + R = r (1 +/- eps), the
    track starting 0.3 rad before the circle's farthest point and moving towards it."""
    kB = synth.K_B_PER_TESLA * 3.8
    r, R, beta, delta = 103.375, 60.0, 0.9, 0.3
    for eps in (1e-5, 1e-4, 1e-3):
        for sign in (+1, -1):
            d = r * (1 + sign * eps) - R
            cc = d * np.array([math.cos(beta), math.sin(beta)])
            psi = beta - turn * delta                       # start, seen from the centre
            p0 = cc + R * np.array([math.cos(psi), math.sin(psi)])
            t = turn * np.array([-math.sin(psi), math.cos(psi)])   # direction of motion
            w = turn / R
            x = np.array([p0[0], p0[1], 0.0, -w / kB, math.atan2(t[1], t[0]), 1.2])
            out, s_arc = oracle.propagate(x, (0.0, 0.0), r, 3.8)
            if sign > 0:
                assert out is not None, eps
                assert abs(math.hypot(out[0], out[1]) - r) < 1e-9 * r
                # the crossing lies before the farthest point, reached after delta * R
                assert 0 < s_arc < delta * R
            else:
                assert out is None, eps


def test_transport_jacobian_central_differences(oracle_lib):
    """Fixed-arc transport Jacobian = central differences of the oracle's helix map."""
    rng = np.random.default_rng(6)
    X = _random_states(rng, 60)
    for i in range(X.shape[1]):
        x = X[:, i]
        s = rng.uniform(1, 40)
        J = oracle.transport_jacobian(x, s, 3.8)
        Jn = np.zeros((6, 6))
        for j in range(6):
            h = 1e-6 * max(1.0, abs(x[j]))
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            d = oracle.helix_at(xp, s, 3.8) - oracle.helix_at(xm, s, 3.8)
            d[4] = (d[4] + math.pi) % (2 * math.pi) - math.pi
            Jn[:, j] = d / (2 * h)
        np.testing.assert_allclose(J, Jn, rtol=1e-6, atol=1e-6 * (1 + s * s * 0.0114))


def test_measurement_matrix_is_tangent_projection(oracle_lib):
    """H = derivative of the local (rho, rho*phi, z) coordinates of the point where the
    state's 3-D tangent line meets the cylinder, for a state on the cylinder."""
    rng = np.random.default_rng(8)
    for _ in range(60):
        c = np.array([rng.normal(0, 0.1), rng.normal(0, 0.1)])
        r = rng.uniform(10, 100)
        a = rng.uniform(-3, 3)
        x = np.array([c[0] + r * math.cos(a), c[1] + r * math.sin(a), rng.uniform(-50, 50),
                      rng.uniform(-2, 2), a + rng.uniform(-1.0, 1.0), rng.uniform(0.5, 2.6)])
        rho0 = r
        phi0 = math.atan2(x[1] - c[1], x[0] - c[0])

        def local(xx):
            px, py = xx[0] - c[0], xx[1] - c[1]
            t = np.array([math.cos(xx[4]), math.sin(xx[4])])
            aa = px * t[0] + py * t[1]
            c0 = px * px + py * py - r * r
            lam = -c0 / (aa + math.copysign(math.sqrt(aa * aa - c0), aa))
            qx, qy = px + lam * t[0], py + lam * t[1]
            qz = xx[2] + lam / math.tan(xx[5])
            dph = (math.atan2(qy, qx) - phi0 + math.pi) % (2 * math.pi) - math.pi
            return np.array([math.hypot(qx, qy), rho0 * dph, qz])

        Hn = np.zeros((3, 6))
        for j in range(6):
            h = 1e-6
            xp, xm = x.copy(), x.copy()
            xp[j] += h
            xm[j] -= h
            Hn[:, j] = (local(xp) - local(xm)) / (2 * h)
        H, _ = oracle.measurement(x, c, x[:3])
        np.testing.assert_allclose(H, Hn, rtol=1e-6, atol=2e-6)


# --------------------------------------------------------------------------------------
# the fit on simulated tracks
# --------------------------------------------------------------------------------------
def test_seed_of_exact_points_is_generating_helix(oracle_lib):
    """The three-hit seed of three exact helix points is the helix at the first one."""
    geom = synth.workload_geometry(2)
    rng = synth.rng_for(91)
    ts = synth.simulate(geom, rng, 200, (0.5, 50.0), True, 1.5, smear=False, scatter=False,
                        hit_dtype=np.float64)
    for i in range(200):
        st, _ = oracle.seed(geom, ts.hits[0, :, i], ts.hits[1, :, i], ts.hits[2, :, i])
        tr = ts.truth[0, :, i]
        np.testing.assert_allclose(st[[0, 1, 2, 5]], tr[[0, 1, 2, 5]], rtol=1e-9, atol=1e-9)
        assert abs(st[3] - tr[3]) <= 1e-8 * abs(tr[3])
        assert abs((st[4] - tr[4] + math.pi) % (2 * math.pi) - math.pi) <= 1e-10


@pytest.mark.parametrize("k", [1, 2])
def test_noiseless_hits_return_generating_helix(oracle_lib, k):
    """Noiseless hits, no material: the fit ends on the generating helix (chi2 ~ 0)."""
    geom = synth.workload_geometry(k)
    geom.xX0[:] = 0.0
    ts = synth.simulate(geom, synth.rng_for(92), 300, (0.5, 50.0), True, 1.5, smear=False,
                        scatter=False, hit_dtype=np.float64)
    o = oracle.fit(geom, ts.hits, ts.hit_mask)
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    tr = ts.truth[last, :, np.arange(300)].T
    ok = o["status"] & oracle.ST_PROP_FAIL == 0
    assert ok.mean() > 0.95
    assert np.all(o["chi2"][ok] < 1e-12)
    d = o["state"] - tr
    d[4] = (d[4] + math.pi) % (2 * math.pi) - math.pi
    assert np.max(np.abs(d[:3, ok])) < 1e-8
    assert np.max(np.abs(d[3, ok] / tr[3, ok])) < 1e-8
    assert np.max(np.abs(d[4:, ok])) < 1e-10


def test_perturbed_seed_converges_to_helix(oracle_lib):
    """Noiseless hits, a wrong external seed (kept on the layer-0 surface, where the
    seed layer's update expects it) with a diffuse prior: the filter recovers the
    generating helix.  The seed is off by 1e-3 cm and 1e-4 rad; a wrong Jacobian, H
    or gain would leave an error of that order instead of ~1e-8."""
    geom = synth.workload_geometry(2)
    geom.xX0[:] = 0.0
    n = 300
    rng = np.random.default_rng(11)
    ts = synth.simulate(geom, synth.rng_for(93), n, (1.0, 50.0), True, 1.5, smear=False,
                        scatter=False, hit_dtype=np.float64)
    tr0 = ts.truth[0]
    r0 = geom.radius[0]
    scale = 1e-3
    seeds = np.zeros((6, n))
    covs = np.zeros((21, n))
    for i in range(n):
        g = rng.normal(size=6)
        a = math.atan2(tr0[1, i], tr0[0, i]) + scale * g[0] / r0
        seeds[:, i] = [r0 * math.cos(a), r0 * math.sin(a), tr0[2, i] + scale * g[2],
                       tr0[3, i] * (1 + scale * g[3]), tr0[4, i] + 0.1 * scale * g[4],
                       tr0[5, i] + 0.1 * scale * g[5]]
        w = np.array([1.0, 1.0, 1.0, abs(tr0[3, i]), 0.1, 0.1]) * scale * 1e4
        covs[:, i] = [(w[a_] ** 2 if a_ == b else 0.0) for a_ in range(6) for b in range(a_ + 1)]
    o = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=seeds, seed_cov=covs)
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    trl = ts.truth[last, :, np.arange(n)].T
    ok = o["status"] & oracle.ST_PROP_FAIL == 0
    assert ok.mean() > 0.95
    xp, Cp = physics.project_to_surface(o["state"], oracle.unpack_cov(o["cov"]), geom.radius[last], geom.k_B)
    d = xp - trl
    d[4] = (d[4] + math.pi) % (2 * math.pi) - math.pi
    assert np.max(np.abs(d[:3, ok])) < 1e-6
    assert np.max(np.abs(d[3, ok] / trl[3, ok])) < 1e-6
    assert np.max(np.abs(d[4:, ok])) < 1e-7
    assert np.max(o["chi2"][ok]) < 1e-5
    # the seed itself is off by the perturbation
    assert np.max(np.abs(seeds[4] - tr0[4])) > 1e-4


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


@pytest.mark.parametrize("k", [1, 2])
def test_pulls_and_chi2_unit_scale(oracle_lib, k):
    """Smeared, scattered tracks: with an uninformative seed chi2/ndf = 1 and the pulls
    of the state projected to the last surface have zero mean and unit width; with the
    ten-times-inflated three-hit seed (hits re-used) chi2/ndf is a few percent above 1."""
    geom, ts = synth.fit_workload(k, n=6000, keep_truth=True)
    n = ts.hits.shape[2]
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    tr = ts.truth[last, :, np.arange(n)].T
    ss, sc = _diffuse_seeds(geom, ts, 1e3)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=ss, seed_cov=sc)
    ok = o["status"] == 0
    assert ok.mean() > 0.9
    r = o["chi2"][ok] / o["ndf"][ok]
    assert abs(r.mean() - 1.0) < 0.03
    xp, Cp = physics.project_to_surface(o["state"], oracle.unpack_cov(o["cov"]), geom.radius[last], geom.k_B)
    for p, v in physics.pulls(xp, Cp, tr, idx=(2, 3, 4, 5)).items():
        assert abs(v[ok].mean()) < 0.05, (p, v[ok].mean())
        assert abs(v[ok].std() - 1.0) < 0.05, (p, v[ok].std())
    o10 = oracle.fit(geom, ts.hits, ts.hit_mask)
    ok10 = o10["status"] == 0
    r10 = (o10["chi2"][ok10] / o10["ndf"][ok10]).mean()
    assert 1.0 < r10 < 1.15


def test_covariances_stay_positive_definite(oracle_lib):
    """Every filtered covariance is symmetric (packed storage) and positive definite."""
    geom, ts = synth.fit_workload(2, n=1500)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, records=True)
    rec = o["records"]
    mins = []
    for i in range(rec.shape[0]):
        for l in range(rec.shape[1]):
            v = rec[i, l]
            if not np.isfinite(v[0]):
                continue
            Cm = oracle.unpack_cov(v[6:])
            np.linalg.cholesky(Cm)
            d = np.sqrt(np.diag(Cm))
            mins.append(np.linalg.eigvalsh(Cm / np.outer(d, d)).min())
    assert len(mins) > 1500 * 10
    assert min(mins) > 0


def test_scattering_matches_generator_kicks(oracle_lib):
    """Q at a state = covariance of the generator's random kicks in (kappa, phi, theta)."""
    geom = synth.Geometry(radius=[50.0], zhalf=[200.0], xX0=[0.03])
    n = 200_000
    for (pt, eta, phi, q) in [(0.8, 0.3, 0.4, 1.0), (3.0, -1.2, -2.0, -1.0)]:
        parts = (np.full(n, pt), np.full(n, phi), np.full(n, eta), np.full(n, q))
        pre = synth.simulate(geom, synth.rng_for(94), n, particles=parts, scatter=False)
        post = synth.simulate(geom, synth.rng_for(94), n, particles=parts, scatter=True)
        d = post.truth[0][[3, 4, 5]] - pre.truth[0][[3, 4, 5]]
        emp = np.cov(d)
        Q = oracle.scattering(geom, pre.truth[0][:, 0], (0.0, 0.0), 0.03)[3:, 3:]
        for a in range(3):
            for b in range(3):
                scale = math.sqrt(Q[a, a] * Q[b, b])
                assert abs(emp[a, b] - Q[a, b]) < 0.02 * scale, (a, b, emp[a, b], Q[a, b])


# --------------------------------------------------------------------------------------
# B = 0: the filter equals the weighted linear least-squares fit of the linearised model
# --------------------------------------------------------------------------------------
def test_straight_tracks_equal_linear_wls(oracle_lib):
    """B = 0, no material, tiny hit errors: the filtered direction and the final chi2
    equal the weighted linear least-squares solution of the straight-line crossing
    model linearised at the truth (built here by central differences of an independent
    line-cylinder intersection), with the seed prior as a pseudo-measurement."""
    geom = synth.barrel(10, 5.0, 100.0, B=0.0, xX0=0.0, eta_max=1.0, sigma_rphi=1e-5, sigma_z=2e-5)
    rng = np.random.default_rng(12)
    n = 40
    ts = synth.simulate(geom, synth.rng_for(95), n, (1.0, 5.0), False, 1.0, scatter=False,
                        hit_dtype=np.float64)
    L = geom.n_layers
    tr0 = ts.truth[0]
    ps = np.array([3e-4, 3e-4, 3e-4, 0.5, 3e-5, 3e-5])   # prior widths; kappa is decoupled at B = 0
    seeds = tr0 + ps[:, None] * rng.normal(size=(6, n))
    # the seed layer's update expects the seed on its surface: move it along the cylinder
    a0 = np.arctan2(tr0[1], tr0[0]) + ps[0] * rng.normal(size=n) / geom.radius[0]
    seeds[0] = geom.radius[0] * np.cos(a0)
    seeds[1] = geom.radius[0] * np.sin(a0)
    covs = np.array([[(ps[a] ** 2 if a == b else 0.0) for a in range(6) for b in range(a + 1)]] * n).T
    o = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=seeds, seed_cov=covs)
    Vi = np.diag([1 / geom.sigma_rphi ** 2, 1 / geom.sigma_z ** 2])
    idx5 = [0, 1, 2, 4, 5]
    for i in range(n):
        x_t = tr0[:, i]
        phi_ref = [math.atan2(y, x) for x, y in zip(ts.truth_hit[:, 0, i], ts.truth_hit[:, 1, i])]

        def y_model(p5):
            x0, y0, z0, ph, th = p5
            out = []
            for l in range(L):
                r = geom.radius[l]
                tx, ty = math.cos(ph), math.sin(ph)
                a = x0 * tx + y0 * ty
                c0 = x0 * x0 + y0 * y0 - r * r
                lam = -c0 / (a + math.copysign(math.sqrt(a * a - c0), a))
                qx, qy, qz = x0 + lam * tx, y0 + lam * ty, z0 + lam / math.tan(th)
                dph = (math.atan2(qy, qx) - phi_ref[l] + math.pi) % (2 * math.pi) - math.pi
                out += [r * dph, qz]
            return np.array(out)

        p_t = x_t[idx5]
        G = np.zeros((2 * L, 5))
        for j in range(5):
            h = 1e-7
            pp, pm = p_t.copy(), p_t.copy()
            pp[j] += h
            pm[j] -= h
            G[:, j] = (y_model(pp) - y_model(pm)) / (2 * h)
        meas = []
        for l in range(L):
            hx, hy, hz = ts.hits[l, :, i]
            dph = (math.atan2(hy, hx) - phi_ref[l] + math.pi) % (2 * math.pi) - math.pi
            meas += [geom.radius[l] * dph, hz]
        dy = np.array(meas) - y_model(p_t)
        P0i = np.diag(1 / ps[idx5] ** 2)
        W = P0i.copy()
        b = P0i @ (seeds[idx5, i] - p_t)
        for l in range(L):
            Gl = G[2 * l: 2 * l + 2]
            W += Gl.T @ Vi @ Gl
            b += Gl.T @ Vi @ dy[2 * l: 2 * l + 2]
        dp = np.linalg.solve(W, b)
        chi2_wls = (dp - (seeds[idx5, i] - p_t)) @ P0i @ (dp - (seeds[idx5, i] - p_t))
        for l in range(L):
            res = dy[2 * l: 2 * l + 2] - G[2 * l: 2 * l + 2] @ dp
            chi2_wls += res @ Vi @ res
        cov_wls = np.linalg.inv(W)
        # straight line: phi and theta do not change along the track
        for k5, k6 in ((3, 4), (4, 5)):
            est = o["state"][k6, i] - x_t[k6]
            sig = math.sqrt(cov_wls[k5, k5])
            assert abs(est - dp[k5]) < 1e-2 * sig, (i, k6, est, dp[k5], sig)
            assert abs(math.sqrt(oracle.unpack_cov(o["cov"][:, i])[k6, k6]) - sig) < 1e-3 * sig
        assert abs(o["chi2"][i] - chi2_wls) < 1e-3 * max(1.0, chi2_wls)


# --------------------------------------------------------------------------------------
# FP64-fallback trigger: the determinant of the equilibrated S
# --------------------------------------------------------------------------------------
def test_fallback_flag_at_known_correlation(oracle_lib):
    """An update whose S has measured rows of correlation rho (constructed so that the
    determinant of S scaled to unit diagonal is exactly 1 - rho^2) is flagged
    ill-conditioned exactly when 1 - rho^2 < 1e-2, on both sides of the threshold."""
    geom = synth.workload_geometry(2)
    hits, mask, st, cov = physics.correlated_seeds(geom, physics.FALLBACK_DETS)
    o = oracle.fit(geom, hits, mask, seed_state=st, seed_cov=cov)
    flagged = (o["status"] & oracle.ST_ILLCOND) != 0
    expect = np.array(physics.FALLBACK_DETS) < 1e-2
    np.testing.assert_array_equal(flagged, expect)
    assert o["status"][~expect].max() == 0   # nothing else is flagged
    # the construction: the S of the update has the intended correlation (the float32
    # prior moves each determinant by < 1e-4 of itself, far inside the 1% spacing)
    for i, d in enumerate(physics.FALLBACK_DETS):
        x, C = st[:, i].astype(np.float64), oracle.unpack_cov(cov[:, i].astype(np.float64))
        H, _ = oracle.measurement(x, (0.0, 0.0), hits[0, :, i].astype(np.float64))
        S = H @ C @ H.T + np.diag([geom.sigma_r ** 2, geom.sigma_rphi ** 2, geom.sigma_z ** 2])
        Dm = np.diag(1.0 / np.sqrt(np.diag(S)))
        assert abs(np.linalg.det(Dm @ S @ Dm) - d) < 1e-4 * d   # float32 rounding of the prior


# --------------------------------------------------------------------------------------
# gradient of the total chi2
# --------------------------------------------------------------------------------------
def _grad_case(n=24, at_truth=False):
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, n=n, align=a_true)
    align = a_true if at_truth else np.zeros_like(a_true)
    return geom, ts, align


@pytest.mark.parametrize("at_truth", [False, True])
def test_dual_gradient_matches_central_differences(oracle_lib, at_truth):
    geom, ts, align = _grad_case(at_truth=at_truth)
    xX0 = geom.xX0.copy()
    ga, gx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, xX0)
    h = 1e-6
    scale = max(np.abs(ga).max(), np.abs(gx).max())
    rng = np.random.default_rng(1)
    comps = [(l, k) for l in range(geom.n_layers) for k in range(5)]
    for (l, k) in [comps[j] for j in rng.choice(len(comps), 30, replace=False)]:
        ap, am = align.copy(), align.copy()
        xp, xm = xX0.copy(), xX0.copy()
        if k < 4:
            ap[l, k] += h
            am[l, k] -= h
            g = ga[l, k]
        else:
            xp[l] += h
            xm[l] -= h
            g = gx[l]
        fd = (oracle.total_chi2(geom, ts.hits, ts.hit_mask, ap, xp) -
              oracle.total_chi2(geom, ts.hits, ts.hit_mask, am, xm)) / (2 * h)
        assert abs(fd - g) <= 1e-6 * abs(g) + 2e-6 * scale, (l, k, fd, g)


def test_gradient_global_symmetries(oracle_lib):
    """A common shift of every layer (x, y, z) or a common rotation about the beam axis
    (at zero misalignment) moves hits and surfaces together and leaves the total chi2
    unchanged: the sums of the per-layer derivatives vanish."""
    geom, ts, align = _grad_case(n=40)
    ga, gx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0)
    for k in range(4):
        assert abs(ga[:, k].sum()) <= 1e-8 * np.abs(ga[:, k]).sum(), (k, ga[:, k].sum(), np.abs(ga[:, k]).sum())
    geom, ts, align = _grad_case(n=40, at_truth=True)
    ga, gx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0)
    for k in range(3):
        assert abs(ga[:, k].sum()) <= 1e-8 * np.abs(ga[:, k]).sum()



def _field_grad_case(at_truth):
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    ts = synth.simulate(geom, synth.rng_for(77), 24, (0.5, 50.0), True, 1.5, align=a_true, field=synth.FIELD_SOLENOID)
    return geom, ts, (a_true if at_truth else np.zeros_like(a_true))


@pytest.mark.parametrize("at_truth", [False, True])
def test_field_gradient_against_central_differences(oracle_lib, at_truth):
    """In the parameterised field (Sec. 3) each step takes the field at its start and the
    seed at its first hit; those points move with the alignment, and the dual numbers
    carry that.  The gradient is therefore the exact derivative of the total chi2: it
    meets the same central-difference bar as in the uniform field, while the gradient
    taken in the uniform field misses the central differences by percents of its scale."""
    geom, ts, align = _field_grad_case(at_truth)
    fld = synth.FIELD_SOLENOID
    xX0 = geom.xX0.copy()
    ga, gx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, xX0, field=fld)
    ua, ux = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, xX0)
    h = 1e-6
    scale = max(np.abs(ga).max(), np.abs(gx).max())
    worst_u = 0.0
    rng = np.random.default_rng(2)
    comps = [(l, k) for l in range(geom.n_layers) for k in range(5)]
    for (l, k) in [comps[j] for j in rng.choice(len(comps), 30, replace=False)]:
        ap, am = align.copy(), align.copy()
        xp, xm = xX0.copy(), xX0.copy()
        if k < 4:
            ap[l, k] += h
            am[l, k] -= h
            g, u = ga[l, k], ua[l, k]
        else:
            xp[l] += h
            xm[l] -= h
            g, u = gx[l], ux[l]
        fd = (oracle.total_chi2(geom, ts.hits, ts.hit_mask, ap, xp, field=fld) -
              oracle.total_chi2(geom, ts.hits, ts.hit_mask, am, xm, field=fld)) / (2 * h)
        assert abs(fd - g) <= 1e-6 * abs(g) + 2e-6 * scale, (l, k, fd, g)
        worst_u = max(worst_u, abs(fd - u) / scale)
    print(f"max |fd - g_uniform| / scale {worst_u:.2e}")
    assert worst_u > 2e-2


@pytest.mark.parametrize("part", ["z only", "r only"])
def test_field_gradient_symmetries(oracle_lib, part):
    """What the field leaves invariant pins the field's part of the gradient.  A field
    B (1 + c_z z^2) does not depend on x, y: a common shift of every hit and surface in
    x or y leaves the total chi2 unchanged (the per-layer derivatives sum to zero), a
    shift in z does not.  A field B (1 + c_r r^2) does not depend on z: the z sums
    vanish, the x and y sums do not.  Both fields are symmetric about the beam axis, so
    at zero misalignment a common rotation leaves the chi2 unchanged.  A gradient that
    omitted the field's change with the step's start point would make every shift sum
    vanish."""
    c_r, c_z = synth.FIELD_SOLENOID
    fld = (0.0, c_z) if part == "z only" else (c_r, 0.0)
    free, bound = ([0, 1], [2]) if part == "z only" else ([2], [0, 1])
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    for at_truth in (False, True):
        ts = synth.simulate(geom, synth.rng_for(77), 24, (0.5, 50.0), True, 1.5, align=a_true, field=fld)
        align = a_true if at_truth else np.zeros_like(a_true)
        ga, _ = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, field=fld)
        sums, mags = ga.sum(axis=0), np.abs(ga).sum(axis=0)
        print(f"[{part}, at truth {at_truth}] shift sums / magnitudes {np.round(sums / mags, 12)}")
        # rounding leaves ~1e-16 of the summed magnitudes; the field's part is >= 3e-8
        for k in free:
            assert abs(sums[k]) <= 1e-11 * mags[k], (k, sums[k], mags[k])
        for k in bound:
            assert abs(sums[k]) > 1e-9 * mags[k], (k, sums[k], mags[k])
        if not at_truth:
            assert abs(sums[3]) <= 1e-11 * mags[3]
