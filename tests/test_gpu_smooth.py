"""GPU smoother (kf_smooth, FP32, through the C ABI) against the oracle's FP64 RTS
smoother, in two parts.

* The smoother step: the oracle's RTS pass run over the GPU fit's own checkpoints
  (the filtered estimates the kernel reads) must agree with the kernel at every layer
  first..last: state within 1e-4 (relative, floors as the fit), covariance within 1e-4
  (|dC_ij| / sqrt(C_ii C_jj)); first and last equal.
* End to end, against the oracle's forward fit plus RTS pass: the checkpoints carry
  the fit's own FP32 error, which the pass spreads over every layer it reaches.  The
  smoothed state at the inner layers follows the outer layers' direction, so an angle
  error of ~1e-6 rad turns into ~1e-4 cm over the ~100 cm lever arm (state: 2e-4); and
  the fit's covariance error, up to 1.4e-4 on tracks that cross three layers without a
  hit right after the seed (an FP32 property of the update there: the oracle's own
  update evaluated in float reaches 0.9-2.2e-4 on the same tracks), measured against
  C_f there, is measured against the smaller C_s here (4.1e-4 seen; covariance: 5e-4).

Tracks with a near-tangent crossing or a propagation failure in the oracle are left
out, as in the fit's tests; every other track has first = 0 and last = the oracle's
last updated layer, and zeros outside first..last."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import cov_err, mask_dev, need_gpu, rel_state_err, to_dev

pytestmark = pytest.mark.gpu

TOL_STATE = 1e-4
TOL_COV = 1e-4
TOL_E2E_STATE = 2e-4
TOL_E2E_COV = 5e-4


def _gpu_smooth(geom, ts, align=None, seeds=None):
    need_gpu()
    from paper_1906_11744_amd import Context
    ctx = Context(geom)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    a = None if align is None else to_dev(np.asarray(align, np.float32))
    x = to_dev(geom.xX0.astype(np.float32))
    kw = {} if seeds is None else dict(seed_state=to_dev(seeds[0]), seed_cov=to_dev(seeds[1]))
    fwd = ctx.fit(hits, mask, align=a, xX0=x, ckpt=True, **kw)
    out = ctx.smooth(hits, mask, fwd, align=a, xX0=x)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if torch.is_tensor(v)}
    g["ckpt"] = fwd["ckpt"].cpu().numpy()
    return g


def _per_layer(g, r, sel_of_l, L):
    rows, wx, wc = [], 0.0, 0.0
    for l in range(L):
        sel = sel_of_l(l)
        if not sel.any():
            continue
        rel = rel_state_err(g["state"][l][:, sel], r["state"][l][:, sel])
        ce = cov_err(g["cov"][l][:, sel], r["cov"][l][:, sel])
        rows.append((l, rel.max(axis=1), ce.max(), np.quantile(ce, 0.999)))
        wx, wc = max(wx, rel.max()), max(wc, ce.max())
    return rows, wx, wc


def _print(label, n, wx, wc, rows):
    print(f"[{label}] n={n}: max rel state err {wx:.2e}, max cov err {wc:.2e}")
    for l, rx, cm, cq in rows:
        print(f"   layer {l:2d}: state {np.array2string(rx, precision=1)} cov max {cm:.1e} p99.9 {cq:.1e}")


def _check(geom, g, r, label, align=None, idx=None):
    L = geom.n_layers
    if idx is not None:
        g = {k: v[..., idx] for k, v in g.items()}
    lend = r["lend"]
    ok = (r["status"] & (oracle.ST_NEAR_TANGENT | oracle.ST_PROP_FAIL)) == 0
    np.testing.assert_array_equal(g["last"][ok], lend[ok], err_msg=label)
    assert np.all(g["first"][ok & (lend >= 0)] == 0), label
    for l in range(L):
        out_ = ok & (lend < l)
        assert np.all(g["state"][l][:, out_] == 0) and np.all(g["cov"][l][:, out_] == 0), (label, l)
    # the step: the oracle's RTS pass over the kernel's own inputs
    ck = g["ckpt"]
    s = oracle.smooth_filtered(geom, ck[:, :6], ck[:, 6:], g["last"], align=align)
    np.testing.assert_array_equal(s["first"][ok], g["first"][ok], err_msg=label)
    rows, wx, wc = _per_layer(g, s, lambda l: ok & (lend >= l), L)
    _print(label + ", step on the GPU's checkpoints", int(ok.sum()), wx, wc, rows)
    # end to end
    rows_e, wxe, wce = _per_layer(g, r, lambda l: ok & (lend >= l), L)
    _print(label + ", end to end", int(ok.sum()), wxe, wce, rows_e)
    assert wx < TOL_STATE, label
    assert wc < TOL_COV, label
    assert wxe < TOL_E2E_STATE, label
    assert wce < TOL_E2E_COV, label


def test_smooth_17_layers_3000_tracks():
    geom, ts = synth.fit_workload(2, n=3000)
    g = _gpu_smooth(geom, ts)
    r = oracle.smooth(geom, ts.hits, ts.hit_mask)
    _check(geom, g, r, "17 layers, 3000 tracks")


def test_smooth_misaligned_and_gaps():
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, n=2000, align=a_true)
    rng = np.random.default_rng(9)
    mask = ts.hit_mask.copy()
    for l in range(3, geom.n_layers):
        mask[rng.random(mask.size) < 0.15] &= ~np.uint32(1 << l)
    ts.hit_mask = mask
    g = _gpu_smooth(geom, ts, align=a_true)
    r = oracle.smooth(geom, ts.hits, ts.hit_mask, align=a_true)
    _check(geom, g, r, "misaligned, masks with gaps", align=a_true)


def test_smooth_1e6_tracks_sampled():
    """The benchmark's workload in one call; 20 000 sampled tracks against the oracle."""
    geom, ts = synth.fit_workload(2)
    g = _gpu_smooth(geom, ts)
    idx = np.sort(np.random.default_rng(4).choice(ts.hits.shape[2], 20000, replace=False))
    r = oracle.smooth(geom, np.ascontiguousarray(ts.hits[:, :, idx]), ts.hit_mask[idx])
    _check(geom, g, r, "1e6 tracks (sample)", idx=idx)


def test_smooth_empty_and_requires_checkpoints():
    need_gpu()
    from paper_1906_11744_amd import Context
    geom, ts = synth.fit_workload(2, n=10)
    ctx = Context(geom)
    hits, mask = to_dev(ts.hits), mask_dev(ts.hit_mask)
    fwd = ctx.fit(hits, mask)
    with pytest.raises(ValueError):
        ctx.smooth(hits, mask, fwd)
