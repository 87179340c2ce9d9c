"""The library's smoother step (kf_smooth.h) instantiated on the host (no GPU) and run
over the FP64 oracle's filtered estimates rounded to float32, against the oracle's
RTS pass over the same rounded estimates:

* in double, the library's rearranged covariance form (3x3 reduction of the filtered
  term, offset-carried state) must reproduce the textbook RTS step to rounding;
* in float, what is measured is the step's own float arithmetic, on tracks with and
  without gaps in the hit pattern (gaps right after the seed leave C_f orders of
  magnitude above C_s, where a direct float evaluation cancels).
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from gpu_common import cov_err, rel_state_err

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_smooth(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("smooth") / "libsmooth_host.so")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                           os.path.join(HERE, "smooth_host.hip"), "-o", out], stderr=subprocess.DEVNULL)
    return C.CDLL(out)


def _case(kind):
    geom = synth.workload_geometry(2)
    if kind == "aligned":
        align = np.zeros((geom.n_layers, 4))
        _, ts = synth.fit_workload(2, n=3000)
        return geom, align, ts.hits, ts.hit_mask
    align = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, n=2000, align=align)
    rng = np.random.default_rng(9)
    mask = ts.hit_mask.copy()
    for l in range(3, geom.n_layers):
        mask[rng.random(mask.size) < 0.15] &= ~np.uint32(1 << l)
    return geom, align, ts.hits, mask


def _run(lib, fn, geom, align, rec, lend):
    L, n = geom.n_layers, lend.size
    xs, Cs = np.zeros((L, 6, n)), np.zeros((L, 21, n))
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    bad = getattr(lib, fn)(C.c_int(L), p(f64(geom.radius)), C.c_double(geom.B), C.c_double(geom.sigma_rphi),
                           C.c_double(geom.sigma_z), C.c_double(geom.sigma_r), C.c_double(geom.mass), p(f64(align)),
                           p(f64(geom.xX0)), C.c_long(n), p(rec), p(lend), p(xs), p(Cs))
    return bad, xs, Cs


@pytest.mark.parametrize("kind", ["aligned", "misaligned_gaps"])
def test_library_step_against_oracle_pass(host_smooth, kind):
    geom, align, hits, mask = _case(kind)
    sm = oracle.smooth(geom, hits, mask, align=align)
    o = oracle.fit(geom, hits, mask, align=align, records=True)
    lend = np.ascontiguousarray(sm["lend"], np.int32)
    rec = np.ascontiguousarray(o["records"].astype(np.float32).astype(np.float64))   # [n][L][27]
    recT = np.transpose(rec, (1, 2, 0))
    ref = oracle.smooth_filtered(geom, recT[:, :6], recT[:, 6:], lend, align=align)
    ok = ((sm["status"] & (oracle.ST_NEAR_TANGENT | oracle.ST_PROP_FAIL)) == 0) & (ref["first"] == 0)
    assert ok.mean() > 0.9
    worst = {}
    for fn in ("smooth_host_f64", "smooth_host_f32"):
        bad, xs, Cs = _run(host_smooth, fn, geom, align, rec, lend)
        assert bad == 0
        wx, wc = 0.0, 0.0
        for l in range(geom.n_layers):
            sel = ok & (lend >= l)
            if not sel.any():
                continue
            wx = max(wx, rel_state_err(xs[l][:, sel], ref["state"][l][:, sel]).max())
            wc = max(wc, cov_err(Cs[l][:, sel], ref["cov"][l][:, sel]).max())
        worst[fn] = (wx, wc)
        print(f"[{fn}, {kind}] max rel state err {wx:.2e}, max cov err {wc:.2e}")
    assert worst["smooth_host_f64"][0] < 1e-9 and worst["smooth_host_f64"][1] < 1e-7
    assert worst["smooth_host_f32"][0] < 1e-4 and worst["smooth_host_f32"][1] < 1e-4


def test_library_step_under_the_detector_model(host_smooth):
    """The same check under the detector model (16-bin material map, silicon's energy
    loss, the field B_z(r, z)): the oracle's pass takes each step's linearisation as
    A J with the loss's kappa row in A; the library's step maps the next layer's
    smoothed estimate back through A^-1 and applies the plain form."""
    geom, ts, fld, mat = synth.field_workload(3000, material=True)
    xmap32 = np.ascontiguousarray(mat[0], np.float32)
    m = (xmap32.astype(np.float64), float(np.float32(mat[1])))
    align = np.zeros((geom.n_layers, 4))
    sm = oracle.smooth(geom, ts.hits, ts.hit_mask, material=m, field=fld)
    o = oracle.fit(geom, ts.hits, ts.hit_mask, records=True, material=m, field=fld)
    lend = np.ascontiguousarray(sm["lend"], np.int32)
    rec = np.ascontiguousarray(o["records"].astype(np.float32).astype(np.float64))
    recT = np.transpose(rec, (1, 2, 0))
    ref = oracle.smooth_filtered(geom, recT[:, :6], recT[:, 6:], lend, material=m, field=fld)
    ok = ((sm["status"] & (oracle.ST_NEAR_TANGENT | oracle.ST_PROP_FAIL)) == 0) & (ref["first"] == 0)
    assert ok.mean() > 0.9
    L, n = geom.n_layers, lend.size
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    worst = {}
    for fn in ("smooth_host_model_f64", "smooth_host_model_f32"):
        xs, Cs = np.zeros((L, 6, n)), np.zeros((L, 21, n))
        bad = getattr(host_smooth, fn)(C.c_int(L), p(f64(geom.radius)), C.c_double(geom.B), C.c_double(geom.sigma_rphi),
                                       C.c_double(geom.sigma_z), C.c_double(geom.sigma_r), C.c_double(geom.mass),
                                       p(f64(align)), p(f64(geom.xX0)), C.c_long(n), p(rec), p(lend), p(xs), p(Cs),
                                       p(xmap32), C.c_int(xmap32.shape[1]), p(f64(geom.zhalf)), C.c_double(m[1]),
                                       C.c_double(fld[0]), C.c_double(fld[1]))
        assert bad == 0
        wx, wc = 0.0, 0.0
        for l in range(L):
            sel = ok & (lend >= l)
            if not sel.any():
                continue
            wx = max(wx, rel_state_err(xs[l][:, sel], ref["state"][l][:, sel]).max())
            wc = max(wc, cov_err(Cs[l][:, sel], ref["cov"][l][:, sel]).max())
        worst[fn] = (wx, wc)
        print(f"[{fn}] max rel state err {wx:.2e}, max cov err {wc:.2e}")
    assert worst["smooth_host_model_f64"][0] < 1e-9 and worst["smooth_host_model_f64"][1] < 1e-7
    assert worst["smooth_host_model_f32"][0] < 1e-4 and worst["smooth_host_model_f32"][1] < 1e-4


@pytest.mark.parametrize("kind", ["aligned", "misaligned_gaps"])
def test_float_block_with_condition_check(host_smooth, kind):
    """The step's C_p^-1 block in float, redone in double where its condition check
    fails (smallest equilibrated pivot, or smallest diagonal element of I - R Q3, below
    det_thr): at det_thr 1e-2 the float step meets the 1e-4 bar; with no fallback at all
    (det_thr 0) the covariance error is measured above it (1.2e-4 aligned, 2.3e-4 with
    misalignment and gaps, where the scattering dominates the filtered angles); det_thr
    above 1 redoes every step in double."""
    geom, align, hits, mask = _case(kind)
    sm = oracle.smooth(geom, hits, mask, align=align)
    o = oracle.fit(geom, hits, mask, align=align, records=True)
    lend = np.ascontiguousarray(sm["lend"], np.int32)
    rec = np.ascontiguousarray(o["records"].astype(np.float32).astype(np.float64))
    recT = np.transpose(rec, (1, 2, 0))
    ref = oracle.smooth_filtered(geom, recT[:, :6], recT[:, 6:], lend, align=align)
    ok = ((sm["status"] & (oracle.ST_NEAR_TANGENT | oracle.ST_PROP_FAIL)) == 0) & (ref["first"] == 0)
    L, n = geom.n_layers, lend.size
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    worst = {}
    for thr in (0.0, 1e-2, 2.0):
        xs, Cs = np.zeros((L, 6, n)), np.zeros((L, 21, n))
        bad = host_smooth.smooth_host_f32_check(
            C.c_int(L), p(f64(geom.radius)), C.c_double(geom.B), C.c_double(geom.sigma_rphi), C.c_double(geom.sigma_z),
            C.c_double(geom.sigma_r), C.c_double(geom.mass), p(f64(align)), p(f64(geom.xX0)), C.c_long(n), p(rec),
            p(lend), p(xs), p(Cs), C.c_double(thr))
        assert bad == 0
        wx = wc = 0.0
        for l in range(L):
            sel = ok & (lend >= l)
            if sel.any():
                wx = max(wx, rel_state_err(xs[l][:, sel], ref["state"][l][:, sel]).max())
                wc = max(wc, cov_err(Cs[l][:, sel], ref["cov"][l][:, sel]).max())
        worst[thr] = (wx, wc)
        print(f"[float block, det_thr {thr:g}, {kind}] max rel state err {wx:.2e}, max cov err {wc:.2e}")
    assert worst[1e-2][0] < 1e-4 and worst[1e-2][1] < 1e-4
    assert worst[2.0][1] < 2e-5
    assert worst[0.0][1] > worst[1e-2][1]
