"""Pins of the oracle's material model (Sec. 3: x/X0 as a function of layer and z for
multiple scattering and energy loss), no GPU.

* A map whose every bin holds the layer's own x/X0, without energy loss, is the
  per-layer model: the fit is bit-identical to the plain one.
* One material step against the definitions written out here in numpy: the map is
  interpolated as the generator does it (synth.material_at, written separately from
  the oracle's lookup), kappa' = kappa p / p' with E' = E - eloss x_eff / beta^2, the
  other parameters unchanged, and the covariance A (C + Q) A^T with Q the oracle's
  scattering term at the interpolated x/X0 and A's kappa row taken by central
  differences of that closed form (the oracle takes it by dual numbers).
* Simulated tracks through the map with energy loss (the generator's own model):
  the fitted parameters' pulls have zero mean and unit width; leaving the energy loss
  out biases the curvature of low-momentum tracks by ~2 sigma, and replacing the map
  by one x/X0 per layer widens the pulls, so both parts of the model are seen.
* The parameterised field (Sec. 3): zero coefficients are the uniform field bit for
  bit; noiseless tracks stepped through a non-uniform field by the generator end on
  their generating state when fitted from it (every residual zero); smeared tracks
  give unit pulls with the model and wide, biased curvature pulls without it.
"""
import math

import numpy as np
import pytest

import oracle
import physics
import synth


def test_constant_map_without_loss_is_the_layer_model(oracle_lib):
    geom, ts = synth.fit_workload(2, n=3000)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask)
    for nz in (1, 8):
        xmap = np.repeat(geom.xX0[:, None], nz, axis=1)
        o = oracle.fit(geom, ts.hits, ts.hit_mask, material=(xmap, 0.0))
        for k in ("state", "cov", "chi2", "ndf", "status"):
            assert np.array_equal(o[k], ref[k]), (nz, k)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, material=(None, 0.0))
    assert np.array_equal(o["state"], ref["state"]) and np.array_equal(o["cov"], ref["cov"])


def _kappa_after_loss(kap, th, xe, eloss, mass):
    p = 1.0 / (abs(kap) * math.sin(th))
    e = math.sqrt(p * p + mass * mass)
    e1 = e - eloss * xe * (e * e) / (p * p)
    if e1 <= mass:
        return None
    return kap * p / math.sqrt(e1 * e1 - mass * mass)


def test_material_step_against_its_definition(oracle_lib):
    geom = synth.workload_geometry(2)
    xmap = synth.material_map(geom, 12)
    eloss = synth.ELOSS_SI_GEV_PER_X0
    rng = np.random.default_rng(5)
    align = np.array([0.01, -0.02, 0.3, 0.0])
    checked = 0
    for _ in range(200):
        l = int(rng.integers(1, geom.n_layers))
        r = geom.radius[l]
        a = rng.uniform(-math.pi, math.pi)
        z_loc = rng.uniform(-1.3, 1.3) * geom.zhalf[l]          # beyond the outer centres too
        x = np.array([align[0] + r * math.cos(a), align[1] + r * math.sin(a), z_loc + align[2],
                      rng.choice([-1, 1]) / (0.5 * 100 ** rng.random()),
                      a + rng.uniform(-0.8, 0.8), rng.uniform(0.5, math.pi - 0.5)])
        A0 = rng.standard_normal((6, 6))
        C0 = A0 @ A0.T * 1e-4 + np.eye(6) * 1e-5
        out = oracle.material_step(geom, l, x, C0, (xmap, eloss), align=align)
        xx = float(synth.material_at(geom, xmap, l, np.array([z_loc]))[0])
        cpsi = math.sin(x[5]) * abs(math.cos(x[4] - a))
        xe = xx / cpsi
        k1 = _kappa_after_loss(x[3], x[5], xe, eloss, geom.mass)
        assert out is not None and k1 is not None
        xs, Cs = out
        assert abs(xs[3] - k1) <= 1e-12 * abs(k1)
        assert np.array_equal(np.delete(xs, 3), np.delete(x, 3))
        # covariance: A (C + Q) A^T, A's kappa row by central differences
        Q = oracle.scattering(geom, x, align[:2], xx)
        hk, ht = 1e-6 * abs(x[3]), 1e-6
        dk = (_kappa_after_loss(x[3] + hk, x[5], xe, eloss, geom.mass) -
              _kappa_after_loss(x[3] - hk, x[5], xe, eloss, geom.mass)) / (2 * hk)
        dt = (_kappa_after_loss(x[3], x[5] + ht, xe, eloss, geom.mass) -
              _kappa_after_loss(x[3], x[5] - ht, xe, eloss, geom.mass)) / (2 * ht)
        A = np.eye(6)
        A[3, 3], A[3, 5] = dk, dt
        Cref = A @ (C0 + Q) @ A.T
        d = np.sqrt(np.diag(Cref))
        assert np.max(np.abs(Cs - Cref) / np.outer(d, d)) < 1e-8
        checked += 1
    assert checked == 200


def test_material_step_stops_a_particle_without_energy(oracle_lib):
    geom = synth.workload_geometry(2)
    l = 5
    r = geom.radius[l]
    x = np.array([r, 0.0, 0.0, 1.0 / 0.05, 0.0, math.pi / 2])        # pT = 50 MeV
    assert oracle.material_step(geom, l, x, np.eye(6) * 1e-4, (None, 10.0), xX0=0.02) is None
    assert oracle.material_step(geom, l, x, np.eye(6) * 1e-4, (None, 0.01), xX0=0.02) is not None


def _pulls(geom, ts, o):
    n = ts.hits.shape[2]
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    ok = (o["status"] & (oracle.ST_PROP_FAIL | oracle.ST_NEAR_TANGENT)) == 0
    tr = ts.truth[last, :, np.arange(n)].T
    xp, Cp = physics.project_to_surface(o["state"], oracle.unpack_cov(o["cov"]), geom.radius[last], geom.k_B)
    return physics.pulls(xp, Cp, tr), tr, ok


@pytest.mark.parametrize("part", ["full", "no_loss", "layer_xX0"])
def test_material_model_pulls(oracle_lib, part):
    geom, ts, mat = synth.material_workload(30000)
    m = {"full": mat, "no_loss": (mat[0], 0.0), "layer_xX0": (None, mat[1])}[part]
    o = oracle.fit(geom, ts.hits, ts.hit_mask, material=m)
    pl, tr, ok = _pulls(geom, ts, o)
    assert ok.mean() > 0.95
    low = ok & (ts.pt < 1.0)
    kq = pl[3][low] * np.sign(tr[3][low])
    widths = [pl[p][ok].std() for p in (3, 4, 5)]
    means = [pl[p][ok].mean() for p in (3, 4, 5)]
    print(f"[{part}] pull means {np.round(means, 3)} widths {np.round(widths, 3)}; "
          f"pT < 1 GeV signed kappa pull mean {kq.mean():+.3f} (n={low.sum()})")
    if part == "full":
        assert max(abs(v) for v in means) < 0.03
        assert max(abs(w - 1.0) for w in widths) < 0.03
        assert abs(kq.mean()) < 0.15
    elif part == "no_loss":
        assert kq.mean() < -1.0          # |kappa| underestimated where the momentum has dropped
    else:
        assert min(widths) > 1.08        # scattering underestimated where the map exceeds 0.02


# --------------------------------------------------------------------------------------
# the parameterised field
# --------------------------------------------------------------------------------------
def test_zero_field_coefficients_are_the_uniform_field(oracle_lib):
    geom, ts = synth.fit_workload(2, n=3000)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, field=(0.0, 0.0))
    for k in ("state", "cov", "chi2", "ndf", "status"):
        assert np.array_equal(o[k], ref[k]), k


def test_noiseless_tracks_in_the_field_return_the_generating_state(oracle_lib):
    """Noiseless hits in float64, no material, B_z falling by up to 16% along z, and the
    generating state at layer 0 as an external seed: with the field model every
    residual vanishes, so the fit ends on the generating trajectory (the generator
    steps with numpy's own helix code, each step in the field at its start); taking the
    field as uniform, or at the end of each step, misses by far more.  (A three-hit seed
    is not exact here: its hits span two steps in different fields.)"""
    geom = synth.workload_geometry(2)
    geom.xX0[:] = 0.0
    n = 300
    ts = synth.simulate(geom, synth.rng_for(94), n, (0.5, 50.0), True, 1.5, smear=False, scatter=False,
                        hit_dtype=np.float64, field=synth.FIELD_SOLENOID)
    last = np.array([int(m).bit_length() - 1 for m in ts.hit_mask])
    tr = ts.truth[last, :, np.arange(n)].T
    seed = np.ascontiguousarray(ts.truth[0])
    w = np.array([1e-2, 1e-2, 1e-1, 1e-2, 1e-3, 1e-3])
    cov = np.zeros((21, n))
    for i in range(6):
        cov[i * (i + 1) // 2 + i] = w[i] ** 2
    errs = {}
    for lab, fld in (("model", synth.FIELD_SOLENOID), ("uniform", None)):
        o = oracle.fit(geom, ts.hits, ts.hit_mask, seed_state=seed, seed_cov=cov, field=fld)
        ok = (o["status"] & oracle.ST_PROP_FAIL) == 0
        assert ok.mean() > 0.95
        d = o["state"] - tr
        d[4] = (d[4] + math.pi) % (2 * math.pi) - math.pi
        errs[lab] = (np.max(np.abs(d[:3, ok])), np.max(np.abs(d[3, ok] / tr[3, ok])), np.max(np.abs(d[4:, ok])),
                     o["chi2"][ok].max())
    print(errs)
    pos, kap, ang, chi2 = errs["model"]
    assert pos < 1e-9 and kap < 1e-9 and ang < 1e-11 and chi2 < 1e-15
    assert errs["uniform"][1] > 1e-3 and errs["uniform"][3] > 1.0


@pytest.mark.parametrize("model", [True, False])
def test_field_model_pulls(oracle_lib, model):
    """Tracks simulated in the field (smeared, scattered): the field model gives unit
    pulls; taking the field as uniform widens the curvature pull threefold and biases
    the curvature of tracks far along z by several sigma."""
    geom, ts, fld, _ = synth.field_workload(30000, material=False)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, field=fld if model else None)
    pl, tr, ok = _pulls(geom, ts, o)
    assert ok.mean() > 0.95
    far = ok & (np.abs(tr[2]) > 100)
    kq = (pl[3][far] * np.sign(tr[3][far])).mean()
    widths = [pl[p][ok].std() for p in (3, 4, 5)]
    means = [pl[p][ok].mean() for p in (3, 4, 5)]
    print(f"[field model {model}] pull means {np.round(means, 3)} widths {np.round(widths, 3)}; "
          f"|z| > 100 cm signed kappa pull mean {kq:+.3f} (n={far.sum()})")
    if model:
        assert max(abs(v) for v in means) < 0.03 and max(abs(w - 1.0) for w in widths) < 0.03
        assert abs(kq) < 0.1
    else:
        assert widths[0] > 2.0 and kq < -2.0


# --------------------------------------------------------------------------------------
# the material model's gradient (dual numbers through the map lookup and the loss)
# --------------------------------------------------------------------------------------
def test_loss_map_derivatives(oracle_lib):
    """kappa1 of the loss map from its definitions (numpy), and the closed-form
    dkappa1/dkappa, dkappa1/dtheta against central differences of kappa1."""
    geom = synth.workload_geometry(2)
    rng = np.random.default_rng(41)
    el = synth.ELOSS_SI_GEV_PER_X0
    m2 = geom.mass ** 2
    for _ in range(200):
        kap = rng.choice([-1, 1]) * rng.uniform(0.02, 2.0)
        th = rng.uniform(0.3, 2.8)
        xe = rng.uniform(0.01, 0.3)
        out = oracle.loss_map(geom, el, kap, th, xe)
        p = 1.0 / (abs(kap) * math.sin(th))
        E = math.sqrt(p * p + m2)
        E1 = E - el * xe * (p * p + m2) / (p * p)
        if E1 <= geom.mass:
            assert out is None
            continue
        k1 = kap * p / math.sqrt(E1 * E1 - m2)
        assert out[0] == pytest.approx(k1, rel=1e-13)
        for j, (dk, dt) in enumerate(((1e-7 * abs(kap), 0.0), (0.0, 1e-7))):
            up = oracle.loss_map(geom, el, kap + dk, th + dt, xe)[0]
            dn = oracle.loss_map(geom, el, kap - dk, th - dt, xe)[0]
            fd = (up - dn) / (2 * (dk + dt))
            assert out[1 + j] == pytest.approx(fd, rel=1e-6, abs=1e-8 * max(1.0, abs(k1) / (dk + dt) * 1e-7)), j


@pytest.mark.parametrize("part", ["map", "map + loss", "loss"])
def test_material_gradient_against_central_differences(oracle_lib, part):
    """The gradient of the total chi2 under the material model: with a map, the fifth
    component per layer is the derivative with respect to an additive offset of that
    layer's map row (x/X0 then comes from the map; the slope of the interpolation in z
    carries the alignment's effect on the crossing point); with the loss, kappa's
    change at each crossing and the covariance's linearisation are differentiated too.
    Both against central differences of the FP64 total chi2."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    xmap = synth.material_map(geom)
    el = synth.ELOSS_SI_GEV_PER_X0 if "loss" in part else 0.0
    use_map = "map" in part
    mat = (xmap if use_map else None, el)
    sim = mat if use_map else (geom.xX0[:, None], el)   # the generator takes the loss with a map
    ts = synth.simulate(geom, synth.rng_for(78), 20, (0.5, 50.0), True, 1.5, align=a_true, material=sim)
    align = np.zeros_like(a_true)
    xX0 = geom.xX0.copy()
    ga, gx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, xX0, material=mat)
    scale = max(np.abs(ga).max(), np.abs(gx).max())
    h = 1e-6
    rng = np.random.default_rng(3)
    comps = [(l, k) for l in range(geom.n_layers) for k in range(5)]
    for (l, k) in [comps[j] for j in rng.choice(len(comps), 30, replace=False)]:
        ap, am = align.copy(), align.copy()
        xp, xm = xX0.copy(), xX0.copy()
        mp, mm = xmap.copy(), xmap.copy()
        if k < 4:
            ap[l, k] += h
            am[l, k] -= h
            g = ga[l, k]
        else:
            if use_map:
                mp[l] += h
                mm[l] -= h
            else:
                xp[l] += h
                xm[l] -= h
            g = gx[l]
        fp = oracle.total_chi2(geom, ts.hits, ts.hit_mask, ap, xp, material=(mp if use_map else None, el))
        fm = oracle.total_chi2(geom, ts.hits, ts.hit_mask, am, xm, material=(mm if use_map else None, el))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g) <= 1e-6 * abs(g) + 2e-6 * scale, (l, k, fd, g)
