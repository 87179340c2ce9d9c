"""The library's hand-written adjoint of the fit (kf_adjoint.h), instantiated in FP64
on the host, equals the oracle's forward-mode dual-number gradient of the same total
chi2 (no GPU).  Both differentiate the same filter with independent code, so they
agree to rounding."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def host_adjoint(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("adj") / "libadjoint_host.so")
    subprocess.check_call(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                           os.path.join(HERE, "adjoint_host.hip"), "-o", out],
                          stderr=subprocess.DEVNULL)
    lib = C.CDLL(out)
    return lib


def run_host(lib, geom, ts, align, xX0, w=None, field=(0.0, 0.0)):
    L = geom.n_layers
    n = ts.hits.shape[2]
    ga = np.zeros((L, 4))
    gx = np.zeros(L)
    hits = np.ascontiguousarray(ts.hits, np.float32)
    mask = np.ascontiguousarray(ts.hit_mask, np.uint32)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    rad, al, xx = f64(geom.radius), f64(align), f64(xX0)
    ww = None if w is None else f64(w)
    rc = lib.adjoint_host_fp64(C.c_int(L), p(rad), C.c_double(geom.B), C.c_double(geom.sigma_rphi),
                               C.c_double(geom.sigma_z), C.c_double(geom.sigma_r), C.c_double(geom.mass), p(al),
                               p(xx), C.c_long(n), p(hits), p(mask), None if ww is None else p(ww), p(ga), p(gx),
                               C.c_double(field[0]), C.c_double(field[1]))
    assert rc == 0
    return ga, gx


@pytest.mark.parametrize("at_truth", [False, True])
def test_host_adjoint_equals_dual_gradient(host_adjoint, at_truth):
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    _, ts = synth.fit_workload(4, n=60, align=a_true)
    align = a_true if at_truth else np.zeros_like(a_true)
    w = np.random.default_rng(3).uniform(0.5, 1.5, ts.hits.shape[2])
    ga, gx = run_host(host_adjoint, geom, ts, align, geom.xX0, w)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    scale = max(np.abs(ra).max(), np.abs(rx).max())
    np.testing.assert_allclose(ga, ra, rtol=1e-9, atol=1e-10 * scale)
    np.testing.assert_allclose(gx, rx, rtol=1e-9, atol=1e-10 * scale)


def test_host_adjoint_no_material(host_adjoint):
    geom = synth.workload_geometry(1)
    _, ts = synth.fit_workload(1, n=50)
    align = synth.misalignment(geom.n_layers) * 0.5
    ga, gx = run_host(host_adjoint, geom, ts, align, np.zeros(geom.n_layers))
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, np.zeros(geom.n_layers))
    scale = np.abs(ra).max()
    np.testing.assert_allclose(ga, ra, rtol=1e-9, atol=1e-10 * scale)


@pytest.mark.parametrize("at_truth", [False, True])
def test_host_adjoint_in_the_field_equals_dual_gradient(host_adjoint, at_truth):
    """Tracks simulated in the parameterised field, fitted in it: the reverse sweep,
    which carries the field's change with each step's start point and with the seed's
    first hit, equals the oracle's dual-number gradient (itself pinned to central
    differences of the total chi2).  Leaving that change out misses by ~1e-4 of the
    gradient's scale, five orders above this bar."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    fld = synth.FIELD_SOLENOID
    ts = synth.simulate(geom, synth.rng_for(77), 60, (0.5, 50.0), True, 1.5, align=a_true, field=fld)
    align = a_true if at_truth else np.zeros_like(a_true)
    w = np.random.default_rng(4).uniform(0.5, 1.5, ts.hits.shape[2])
    ga, gx = run_host(host_adjoint, geom, ts, align, geom.xX0, w, field=fld)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w, field=fld)
    ua, _ = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w)
    scale = max(np.abs(ra).max(), np.abs(rx).max())
    assert np.abs(ua - ra).max() > 1e-2 * scale          # the field matters at this size
    np.testing.assert_allclose(ga, ra, rtol=1e-9, atol=1e-10 * scale)
    np.testing.assert_allclose(gx, rx, rtol=1e-9, atol=1e-10 * scale)


@pytest.mark.parametrize("part", ["map", "map + loss", "loss"])
def test_host_adjoint_under_the_material_model_equals_dual_gradient(host_adjoint, part):
    """The material model (Sec. 3) in the reverse sweep: the map's value moves with the
    crossing's z (its interpolation's slope) and its row offset is the fifth component;
    the energy loss's change of kappa and its linearisation A of the covariance are
    differentiated through the loss's local Jacobian (forward-mode in the library).  In
    FP64 on the host it equals the oracle's dual-number gradient, which is pinned to
    central differences of the total chi2."""
    geom = synth.workload_geometry(2)
    a_true = synth.misalignment(geom.n_layers)
    xmap = synth.material_map(geom).astype(np.float32)
    el = synth.ELOSS_SI_GEV_PER_X0 if "loss" in part else 0.0
    use_map = "map" in part
    sim = (xmap, el) if use_map else (geom.xX0[:, None], el)
    ts = synth.simulate(geom, synth.rng_for(79), 60, (0.5, 50.0), True, 1.5, align=a_true, material=sim)
    align = np.zeros_like(a_true)
    w = np.random.default_rng(8).uniform(0.5, 1.5, ts.hits.shape[2])
    L, n = geom.n_layers, ts.hits.shape[2]
    ga, gx = np.zeros((L, 4)), np.zeros(L)
    f64 = lambda a: np.ascontiguousarray(a, np.float64)
    p = lambda a: a.ctypes.data_as(C.c_void_p)
    hits = np.ascontiguousarray(ts.hits, np.float32)
    mask = np.ascontiguousarray(ts.hit_mask, np.uint32)
    mp = np.ascontiguousarray(xmap) if use_map else None
    rc = host_adjoint.adjoint_host_model_fp64(
        C.c_int(L), p(f64(geom.radius)), p(f64(geom.zhalf)), C.c_double(geom.B), C.c_double(geom.sigma_rphi),
        C.c_double(geom.sigma_z), C.c_double(geom.sigma_r), C.c_double(geom.mass), p(f64(align)), p(f64(geom.xX0)),
        None if mp is None else p(mp), C.c_int(xmap.shape[1] if use_map else 0), C.c_double(el), C.c_long(n),
        p(hits), p(mask), p(f64(w)), p(ga), p(gx))
    assert rc == 0
    mat = (xmap.astype(np.float64) if use_map else None, el)
    ra, rx = oracle.fit_grad(geom, ts.hits, ts.hit_mask, align, geom.xX0, w, material=mat)
    scale = max(np.abs(ra).max(), np.abs(rx).max())
    print(f"[{part}] max |host - oracle| / scale: align {np.abs(ga - ra).max() / scale:.1e}, "
          f"x/X0 {np.abs(gx - rx).max() / scale:.1e}")
    np.testing.assert_allclose(ga, ra, rtol=1e-8, atol=1e-9 * scale)
    np.testing.assert_allclose(gx, rx, rtol=1e-8, atol=1e-9 * scale)
