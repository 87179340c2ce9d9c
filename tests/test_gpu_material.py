"""GPU kf_fit with the detector model (kf_ctx_set_material: a map of x/X0 in (layer, z)
and the mean energy loss; kf_ctx_set_field: the field B_z(r, z)) against the FP64
oracle's fit with the same model.

Tolerances as for the plain fit: state 1e-4 (relative, floors 1 cm and 1 rad),
covariance 1e-4 (|dC_ij| / sqrt(C_ii C_jj)), chi2 0.05 + 1e-4 chi2, ndf and the
PROP_FAIL / BAD_INPUT bits exact; tracks with a near-tangent crossing are left out of
the state bar as there.  Cases: tracks simulated through the map with energy loss
(the model's own generator) on 17 layers, misaligned layers with gaps (the map
follows each layer's z shift), 20 000 tracks sampled from the 1e6-track call, a
loss large enough to stop slow particles, each part of the model alone, and a map of
constant rows without loss, which is the per-layer model; tracks stepped through the
parameterised field, alone and with the material model; and the finder (search and
refit) on events simulated with the whole model, under the finder's own parity rule
(tests/test_gpu_find.py)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import cov_err, mask_dev, need_gpu, rel_state_err, to_dev

pytestmark = pytest.mark.gpu

TOL_STATE = 1e-4
TOL_COV = 1e-4


def _fit(geom, ts, material, align=None, ctx=None, field=(0.0, 0.0)):
    need_gpu()
    from paper_1906_11744_amd import Context
    ctx = Context(geom) if ctx is None else ctx
    xmap, eloss = material
    ctx.set_material(None if xmap is None else to_dev(np.asarray(xmap, np.float32)), eloss)
    ctx.set_field(*field)
    a = None if align is None else to_dev(np.asarray(align, np.float32))
    out = ctx.fit(to_dev(ts.hits), mask_dev(ts.hit_mask), align=a, xX0=to_dev(geom.xX0.astype(np.float32)))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items() if torch.is_tensor(v)}


def _oracle_material(material):
    # the oracle reads the map the GPU reads: float32 values
    xmap, eloss = material
    return (None if xmap is None else np.asarray(xmap, np.float32).astype(np.float64), float(np.float32(eloss)))


def _compare(g, ref, label, idx=None, tol_cov=TOL_COV, state_sel=None):
    if idx is not None:
        g = {k: v[..., idx] for k, v in g.items()}
    st, cv, c2, ndf = g["state"], g["cov"], g["chi2"], g["ndf"]
    status = g["status"].view(np.uint32)
    pf = (status & oracle.ST_PROP_FAIL) != (ref["status"] & oracle.ST_PROP_FAIL)
    np.testing.assert_array_equal(status & oracle.ST_BAD_INPUT, ref["status"] & oracle.ST_BAD_INPUT)
    live = ((ref["status"] & oracle.ST_BAD_INPUT) == 0) & ~pf
    np.testing.assert_array_equal(ndf[live], ref["ndf"][live], err_msg=label)
    ok = live & ((ref["status"] & oracle.ST_NEAR_TANGENT) == 0)
    if state_sel is not None:
        print(f"[{label}] {int((ok & ~state_sel).sum())} tracks left out of the state and covariance bars")
        ok = ok & state_sel
    rel = rel_state_err(st, ref["state"])
    ce = cov_err(cv, ref["cov"])
    dchi = np.abs(c2.astype(np.float64) - ref["chi2"])
    print(f"[{label}] n={ok.sum()} max rel state err per param {np.array2string(rel[:, ok].max(axis=1), precision=2)};"
          f" max cov err {ce[ok].max():.2e}; max |dchi2| {dchi[ok].max():.2e}; PROP_FAIL differences {int(pf.sum())}"
          f" (oracle stops {int(((ref['status'] & oracle.ST_PROP_FAIL) != 0).sum())})")
    assert pf.mean() < 1e-3, label
    assert rel[:, ok].max() < TOL_STATE, label
    assert ce[ok].max() < tol_cov, label
    assert np.all(dchi[ok] < 0.05 + 1e-4 * ref["chi2"][ok]), label
    return ok


def test_material_map_with_energy_loss():
    geom, ts, mat = synth.material_workload(3000)
    g = _fit(geom, ts, mat)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask, material=_oracle_material(mat))
    _compare(g, ref, "map (16 bins) + energy loss, 17 layers")


def test_material_misaligned_with_gaps():
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    xmap = synth.material_map(geom, 24)
    mat = (xmap, synth.ELOSS_SI_GEV_PER_X0)
    ts = synth.simulate(geom, synth.rng_for(8), 3000, (0.5, 50.0), True, 1.5, align=a_true, material=mat)
    rng = np.random.default_rng(12)
    mask = ts.hit_mask.copy()
    for l in range(3, geom.n_layers):
        mask[rng.random(mask.size) < 0.15] &= ~np.uint32(1 << l)
    ts.hit_mask = mask
    g = _fit(geom, ts, mat, align=a_true)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask, align=a_true, material=_oracle_material(mat))
    # covariance bar 2e-4 as for the plain fit with gaps: after a three-layer gap right
    # after the seed the FP32 update leaves a few-ulp error in the kappa-kappa element
    # that later updates do not shrink (the plain fit's own gaps case measures 1.4e-4)
    _compare(g, ref, "map (24 bins) + loss, misaligned, 15% gaps", tol_cov=2e-4)


def test_material_1e6_tracks_sampled():
    """The benchmark's material configuration in one call; 20 000 tracks sampled."""
    geom, ts, mat = synth.material_workload(1_000_000)
    g = _fit(geom, ts, mat)
    idx = np.sort(np.random.default_rng(6).choice(ts.hits.shape[2], 20000, replace=False))
    ref = oracle.fit(geom, np.ascontiguousarray(ts.hits[:, :, idx]), ts.hit_mask[idx],
                     material=_oracle_material(mat))
    _compare(g, ref, "1e6 tracks with map + loss (sample)", idx=idx)


@pytest.mark.parametrize("part", ["map_only", "loss_only", "one_bin_map", "max_bins_map"])
def test_material_parts(part):
    geom, ts, mat = synth.material_workload(3000)
    m = {"map_only": (mat[0], 0.0), "loss_only": (None, mat[1]),
         "one_bin_map": (mat[0][:, :1].copy(), mat[1]),
         "max_bins_map": (synth.material_map(geom, 64), mat[1])}[part]   # KF_MAX_MAP_BINS
    g = _fit(geom, ts, m)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask, material=_oracle_material(m))
    _compare(g, ref, part)


def test_energy_loss_stops_slow_particles():
    """A loss 40 times silicon's: the slowest tracks range out inside the tracker; the
    layer where each stops (ndf) and the PROP_FAIL bit agree with the oracle.  The state
    bar applies to tracks whose |kappa| grows by less than 1.5 times over the fit:
    while a particle slows to p' << p, every step multiplies the relative error of its
    momentum by ~(p/p')^2, so FP32 cannot follow the last steps of a particle that
    nearly stops (5e-4 seen there)."""
    geom, ts, mat = synth.material_workload(3000)
    m = (mat[0], 40 * mat[1])
    g = _fit(geom, ts, m)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask, material=_oracle_material(m), records=True)
    stops = (ref["status"] & oracle.ST_PROP_FAIL) != 0
    assert stops.sum() > 50
    k0 = np.abs(ref["records"][:, 0, 3])
    gentle = np.abs(ref["state"][3]) < 1.5 * k0
    _compare(g, ref, "loss x 40: slow particles stop", state_sel=gentle)


def _oracle_field(field):
    return tuple(float(np.float32(c)) for c in field)


@pytest.mark.parametrize("with_material", [False, True])
def test_parameterised_field(with_material):
    geom, ts, fld, mat = synth.field_workload(3000, material=with_material)
    m = mat if with_material else (None, 0.0)
    g = _fit(geom, ts, m, field=fld)
    ref = oracle.fit(geom, ts.hits, ts.hit_mask, material=_oracle_material(m), field=_oracle_field(fld))
    _compare(g, ref, "field B_z(r, z)" + (" + map + loss" if with_material else ""))


def test_constant_map_without_loss_is_the_layer_model():
    geom, ts = synth.fit_workload(2, n=3000)
    need_gpu()
    from paper_1906_11744_amd import Context
    ctx = Context(geom)
    plain = ctx.fit(to_dev(ts.hits), mask_dev(ts.hit_mask), xX0=to_dev(geom.xX0.astype(np.float32)))
    plain = {k: v.cpu().numpy() for k, v in plain.items() if torch.is_tensor(v)}
    g = _fit(geom, ts, (np.repeat(geom.xX0[:, None], 8, axis=1), 0.0), ctx=ctx)
    ok = (plain["status"] & 3) == 0
    assert np.array_equal(g["status"], plain["status"]) and np.array_equal(g["ndf"], plain["ndf"])
    assert rel_state_err(g["state"], plain["state"].astype(np.float64))[:, ok].max() < 1e-6
    assert cov_err(g["cov"], plain["cov"].astype(np.float64))[ok].max() < 1e-6


def test_smoother_under_the_detector_model():
    """kf_smooth after a checkpointing fit, both under the whole model (map, loss,
    field), against the oracle's RTS pass over the GPU's own checkpoints (the step:
    1e-4 / 1e-4) and against the oracle's own fit and smoother (end to end: 2e-4 /
    5e-4, the bars of the plain smoother and for the same reasons)."""
    from gpu_common import cov_err as _ce
    need_gpu()
    from paper_1906_11744_amd import Context
    geom, ts, fld, mat = synth.field_workload(3000, material=True)
    ctx = Context(geom)
    ctx.set_material(to_dev(np.asarray(mat[0], np.float32)), mat[1])
    ctx.set_field(*fld)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    x = to_dev(geom.xX0.astype(np.float32))
    fwd = ctx.fit(hits, mask, xX0=x, ckpt=True)
    out = ctx.smooth(hits, mask, fwd, xX0=x)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if torch.is_tensor(v)}
    ck = fwd["ckpt"].cpu().numpy()
    m, f = _oracle_material(mat), _oracle_field(fld)
    r = oracle.smooth(geom, ts.hits, ts.hit_mask, material=m, field=f)
    s = oracle.smooth_filtered(geom, ck[:, :6], ck[:, 6:], g["last"], material=m, field=f)
    lend = r["lend"]
    ok = (r["status"] & (oracle.ST_NEAR_TANGENT | oracle.ST_PROP_FAIL)) == 0
    np.testing.assert_array_equal(g["last"][ok], lend[ok])
    assert np.all(g["first"][ok & (lend >= 0)] == 0)
    np.testing.assert_array_equal(s["first"][ok], g["first"][ok])
    wx = wc = ex = ec = 0.0
    for l in range(geom.n_layers):
        sel = ok & (lend >= l)
        if not sel.any():
            continue
        wx = max(wx, rel_state_err(g["state"][l][:, sel], s["state"][l][:, sel]).max())
        wc = max(wc, _ce(g["cov"][l][:, sel], s["cov"][l][:, sel]).max())
        ex = max(ex, rel_state_err(g["state"][l][:, sel], r["state"][l][:, sel]).max())
        ec = max(ec, _ce(g["cov"][l][:, sel], r["cov"][l][:, sel]).max())
    print(f"[smoother under the detector model] n={ok.sum()} step: state {wx:.2e} cov {wc:.2e}; "
          f"end to end: state {ex:.2e} cov {ec:.2e}")
    assert wx < 1e-4 and wc < 1e-4
    assert ex < 2e-4 and ec < 5e-4


def test_loss_without_map_in_the_adjoint_then_cleared():
    """The mean energy loss with one x/X0 per layer (no map): the adjoint accepts it and
    returns finite gradients that differ from the plain model's; clearing the model
    leaves the context usable for the finder."""
    need_gpu()
    from paper_1906_11744_amd import Context
    geom, ev = synth.find_workload(3, n_tracks=50)
    ctx = Context(geom)
    t = lambda a: to_dev(np.ascontiguousarray(a))
    _, ts = synth.fit_workload(2, n=100)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    xX0 = t(geom.xX0.astype(np.float32))
    w = torch.ones(100, device="cuda")
    fwd = ctx.fit(hits, mask, xX0=xX0, ckpt=True)
    ga0, gx0 = ctx.fit_backward(hits, mask, fwd, w, xX0=xX0)
    ctx.set_material(None, 0.0363)
    fwd = ctx.fit(hits, mask, xX0=xX0, ckpt=True)
    ga, gx = ctx.fit_backward(hits, mask, fwd, w, xX0=xX0)
    torch.cuda.synchronize()
    assert torch.isfinite(ga).all() and torch.isfinite(gx).all()
    assert not torch.equal(gx, gx0)
    ctx.set_material(None, 0.0)
    ctx.find(t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event))
    torch.cuda.synchronize()


@pytest.mark.parametrize("loss_scale", [1.0, 40.0])
def test_finder_with_the_detector_model(loss_scale):
    """One event of 2 000 tracks (20% noise) simulated through the map with energy loss
    in the field; kf_find with refit under the same model against the oracle's finder;
    with 40 times the loss, candidates whose particle stops end at that layer."""
    from test_gpu_find import compare, oracle_find
    need_gpu()
    from paper_1906_11744_amd import Context
    geom = synth.workload_geometry(2)
    xmap = synth.material_map(geom, 16)
    mat = (xmap, synth.ELOSS_SI_GEV_PER_X0 * loss_scale)
    fld = synth.FIELD_SOLENOID
    ev = synth.make_events(geom, [2000], workload=10, material=(xmap, synth.ELOSS_SI_GEV_PER_X0), field=fld)
    ctx = Context(geom)
    ctx.set_material(to_dev(xmap.astype(np.float32)), mat[1])
    ctx.set_field(*fld)
    t = lambda a: to_dev(np.ascontiguousarray(a))
    out = ctx.find(t(ev.hits), t(ev.hit_off), t(ev.seed_hits), t(ev.seed_event),
                   xX0=t(geom.xX0.astype(np.float32)), refit=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if torch.is_tensor(v)}
    r = oracle_find(geom, ev, refit=True, material=mat, field=fld)
    stats = compare(geom, ev, g, r, f"finder with map, loss x {loss_scale:g} and field", material=mat, field=fld)
    assert stats["exact"] + stats["reordered"] > 0.97 * ev.seed_hits.shape[1]
    stops = ((r["status"][0] & oracle.ST_PROP_FAIL) != 0).sum()
    print(f"oracle rank-0 candidates ending with PROP_FAIL: {stops}")
    # the refit of each seed's best candidate under the same model
    ok = (r["n_cand"] > 0) & ((r["rf_status"] & (oracle.ST_PROP_FAIL | oracle.ST_NEAR_TANGENT)) == 0)
    same = np.array([np.array_equal(g["hit_idx"][0, :, s], r["hit_idx"][0, :, s]) for s in range(ok.size)])
    sel = ok & same
    rel = rel_state_err(g["rf_state"][:, sel], r["rf_state"][:, sel])
    print(f"refit: n={sel.sum()} max rel state err {rel.max():.2e}")
    assert rel.max() < 1e-4
