"""GPU adjoint of the fit (kf_fit_backward, FP32) against the oracle's FP64 dual-number
gradient of the same total chi2.

Tolerance: ||g_gpu - g_ref|| / ||g_ref|| < 1e-3 over the 85 parameters (17 layers x
(dx, dy, dz, dphi, x/X0)), and per component |d| < 1e-3 ||g_ref||_inf + 1e-2 |g_ref|.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import mask_dev, need_gpu, to_dev

pytestmark = pytest.mark.gpu


def _case(n, at_truth):
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, n=n, align=a_true)
    align = a_true if at_truth else np.zeros_like(a_true)
    return geom, ts, align


def _gpu_grad(geom, ts, align, w, field=None, det_threshold=None, ckpt_every=1, static=False, material=None):
    need_gpu()
    from paper_1906_11744_amd import Context
    kf = Context(geom)
    if field is not None:
        kf.set_field(*field)
    keep = None
    if material is not None:   # (map [L][nz] float32 or None, eloss)
        keep = None if material[0] is None else to_dev(np.asarray(material[0], np.float32))
        kf.set_material(keep, material[1])
    if det_threshold is not None:
        kf.set_fallback_threshold(det_threshold)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    a = to_dev(np.asarray(align, np.float32))
    x = to_dev(geom.xX0.astype(np.float32))
    fwd = kf.fit(hits, mask, align=a, xX0=x, ckpt=True, ckpt_every=ckpt_every)
    back = kf.fit_backward_static if static else kf.fit_backward
    da, dx = back(hits, mask, fwd, to_dev(np.asarray(w, np.float32)), align=a, xX0=x)
    torch.cuda.synchronize()
    return da.cpu().numpy().astype(np.float64), dx.cpu().numpy().astype(np.float64), fwd


def _check(ga, gx, ra, rx, label):
    g = np.concatenate([ga.ravel(), gx])
    r = np.concatenate([ra.ravel(), rx])
    rel = np.linalg.norm(g - r) / np.linalg.norm(r)
    worst = np.max(np.abs(g - r) / (1e-3 * np.abs(r).max() + 1e-2 * np.abs(r)))
    print(f"[{label}] ||dg||/||g|| = {rel:.2e}; worst component / tolerance = {worst:.2f}")
    assert rel < 1e-3, label
    assert worst < 1.0, label


@pytest.mark.parametrize("at_truth", [False, True])
def test_gradient_matches_fp64_reference(at_truth):
    geom, ts, align = _case(2000, at_truth)
    w = np.random.default_rng(5).uniform(0.5, 1.5, ts.hits.shape[2])
    ga, gx, _ = _gpu_grad(geom, ts, align, w)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    _check(ga, gx, ra, rx, f"2000 tracks, align {'true' if at_truth else 'zero'}")


def test_gradient_full_size_1e5_tracks():
    """The differentiable-fit workload at full size (1e5 tracks, misaligned, x/X0 =
    0.02) in one launch.  The gradient is linear in the per-track weights, so weight 1
    on 2 000 sampled tracks and 0 elsewhere must give the oracle's gradient of those
    tracks alone."""
    geom, ts, align = _case(100_000, False)
    n = ts.hits.shape[2]
    idx = np.sort(np.random.default_rng(9).choice(n, 2000, replace=False))
    w = np.zeros(n)
    w[idx] = 1.0
    ga, gx, _ = _gpu_grad(geom, ts, align, w)
    ra, rx = oracle.fit_grad(geom, np.ascontiguousarray(ts.hits[:, :, idx]), ts.hit_mask[idx], align, geom.xX0)
    _check(ga, gx, ra, rx, "1e5 tracks, 2000 weighted")


@pytest.mark.parametrize("at_truth", [False, True])
def test_gradient_in_the_field_matches_fp64_reference(at_truth):
    """Tracks simulated in the parameterised field B (1 + c_r r^2 + c_z z^2), fitted and
    differentiated in it: the reverse sweep carries the field's change with each step's
    start point and the seed's first hit, and the reference is the oracle's exact
    dual-number gradient; the gradient taken in the uniform field differs from it by far
    more than the tolerance."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    fld = synth.FIELD_SOLENOID
    ts = synth.simulate(geom, synth.rng_for(78), 2000, (0.5, 50.0), True, 1.5, align=a_true, field=fld)
    align = a_true if at_truth else np.zeros_like(a_true)
    w = np.random.default_rng(6).uniform(0.5, 1.5, ts.hits.shape[2])
    ga, gx, _ = _gpu_grad(geom, ts, align, w, field=fld)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w, field=fld)
    _check(ga, gx, ra, rx, f"field, 2000 tracks, align {'true' if at_truth else 'zero'}")
    ua, ux = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    r, u = np.concatenate([ra.ravel(), rx]), np.concatenate([ua.ravel(), ux])
    assert np.linalg.norm(u - r) / np.linalg.norm(r) > 1e-2


def test_gradient_in_the_field_full_size_1e5_tracks():
    """The differentiable-fit workload's size under the parameterised field, in one
    launch as timed: weight 1 on 2 000 sampled tracks and 0 elsewhere gives the
    oracle's gradient of those tracks alone."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    fld = synth.FIELD_SOLENOID
    ts = synth.simulate(geom, synth.rng_for(79), 100_000, (0.5, 50.0), True, 1.5, align=a_true, field=fld)
    align = np.zeros_like(a_true)
    n = ts.hits.shape[2]
    idx = np.sort(np.random.default_rng(10).choice(n, 2000, replace=False))
    w = np.zeros(n)
    w[idx] = 1.0
    ga, gx, _ = _gpu_grad(geom, ts, align, w, field=fld)
    ra, rx = oracle.fit_grad(geom, np.ascontiguousarray(ts.hits[:, :, idx]), ts.hit_mask[idx], align, geom.xX0,
                             field=fld)
    _check(ga, gx, ra, rx, "field, 1e5 tracks, 2000 weighted")


@pytest.mark.parametrize("at_truth", [False, True])
def test_gradient_with_forced_fp64_inverse(at_truth):
    """A fallback threshold above 1 sends every update's S^-1 to FP64 in the forward fit;
    the reverse sweep then recomputes each S^-1 by the same FP64 path, and the gradient
    still equals the FP64 reference."""
    geom, ts, align = _case(2000, at_truth)
    w = np.random.default_rng(7).uniform(0.5, 1.5, ts.hits.shape[2])
    ga, gx, fwd = _gpu_grad(geom, ts, align, w, det_threshold=2.0)
    st = fwd["status"].cpu().numpy().view(np.uint32)
    fitted = (st & (oracle.ST_BAD_INPUT | oracle.ST_PROP_FAIL)) == 0
    assert np.all(st[fitted] & oracle.ST_ILLCOND)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    _check(ga, gx, ra, rx, f"forced FP64 S^-1, align {'true' if at_truth else 'zero'}")


def test_backward_is_deterministic():
    geom, ts, align = _case(20000, True)
    w = np.ones(ts.hits.shape[2])
    a1, x1, _ = _gpu_grad(geom, ts, align, w)
    a2, x2, _ = _gpu_grad(geom, ts, align, w)
    np.testing.assert_array_equal(a1, a2)
    np.testing.assert_array_equal(x1, x2)


def test_autograd_function():
    """torch.autograd through FitChi2: gradient of sum(w * chi2) equals kf_fit_backward
    with dchi2 = w, and the per-track chi2 equals the plain fit's."""
    need_gpu()
    from paper_1906_11744_amd import Context, fit_chi2
    geom, ts, align = _case(1500, True)
    kf = Context(geom)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    a = to_dev(align.astype(np.float32)).requires_grad_(True)
    x = to_dev(geom.xX0.astype(np.float32)).requires_grad_(True)
    w = to_dev(np.random.default_rng(2).uniform(0.5, 1.5, ts.hits.shape[2]).astype(np.float32))
    chi2 = fit_chi2(kf, hits, mask, a, x)
    (w * chi2).sum().backward()
    plain = kf.fit(hits, mask, align=a.detach(), xX0=x.detach())
    assert torch.equal(chi2.detach(), plain["chi2"])
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w.cpu().numpy().astype(np.float64))
    _check(a.grad.cpu().numpy().astype(np.float64), x.grad.cpu().numpy().astype(np.float64), ra, rx, "autograd")


@pytest.mark.parametrize("every", [2, 3, 5, 17])
def test_sparse_checkpoints_recompute_the_gradient(every):
    """Checkpoints on every k-th layer only (the fit stores ceil(17 / k) of them); the
    backward recomputes each run of layers between two from the lower one.  The
    gradient equals the dense-checkpoint one to float rounding (the recomputed states
    come from the adjoint's own forward step, not the fit kernel's bits) and meets the
    oracle's bar; the field's variant and the allocation-free entry point alike."""
    geom, ts, align = _case(3000, False)
    w = np.random.default_rng(6).uniform(0.5, 1.5, ts.hits.shape[2])
    ga1, gx1, _ = _gpu_grad(geom, ts, align, w)
    ga, gx, fwd = _gpu_grad(geom, ts, align, w, ckpt_every=every)
    assert fwd["ckpt"].shape[0] == -(-geom.n_layers // every)
    g1 = np.concatenate([ga1.ravel(), gx1])
    g = np.concatenate([ga.ravel(), gx])
    rel = np.linalg.norm(g - g1) / np.linalg.norm(g1)
    print(f"[every {every}] ||g_sparse - g_dense|| / ||g_dense|| = {rel:.2e}")
    assert rel < 1e-5
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    _check(ga, gx, ra, rx, f"checkpoints every {every}")
    gas, gxs, _ = _gpu_grad(geom, ts, align, w, ckpt_every=every, static=True)
    np.testing.assert_array_equal(gas, ga)
    np.testing.assert_array_equal(gxs, gx)
    if every == 3:
        field = (-1e-6, -4e-6)
        gaf1, gxf1, _ = _gpu_grad(geom, ts, align, w, field=field)
        gaf, gxf, _ = _gpu_grad(geom, ts, align, w, field=field, ckpt_every=every)
        gf1 = np.concatenate([gaf1.ravel(), gxf1])
        gf = np.concatenate([gaf.ravel(), gxf])
        assert np.linalg.norm(gf - gf1) / np.linalg.norm(gf1) < 1e-5


@pytest.mark.parametrize("part", ["map", "map + loss", "loss"])
def test_gradient_under_the_material_model(part):
    """The material model in the adjoint: the map's value at each crossing (its slope in
    z; with a map the fifth component is the derivative w.r.t. an additive offset of
    each layer's row) and the energy loss (kappa's change and its linearisation of the
    covariance), against the oracle's dual-number gradient on what the GPU reads (the
    map rounded to float32); and the same with checkpoints every third layer."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    xmap = synth.material_map(geom).astype(np.float32)
    el = synth.ELOSS_SI_GEV_PER_X0 if "loss" in part else 0.0
    use_map = "map" in part
    sim = (xmap, el) if use_map else (geom.xX0[:, None], el)
    ts = synth.simulate(geom, synth.rng_for(80), 2000, (0.5, 50.0), True, 1.5, align=a_true, material=sim)
    align = np.zeros_like(a_true)
    w = np.random.default_rng(11).uniform(0.5, 1.5, ts.hits.shape[2])
    mat = (xmap if use_map else None, float(np.float32(el)))
    ga, gx, _ = _gpu_grad(geom, ts, align, w, material=mat)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w,
                             material=(xmap.astype(np.float64) if use_map else None, mat[1]))
    _check(ga, gx, ra, rx, f"material model: {part}")
    ga3, gx3, _ = _gpu_grad(geom, ts, align, w, material=mat, ckpt_every=3)
    _check(ga3, gx3, ra, rx, f"material model: {part}, checkpoints every 3")
