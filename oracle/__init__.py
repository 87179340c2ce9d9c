"""Python access to the FP64 oracle (kf_oracle.cpp).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU-baseline leg of the
benchmark use it to check and time the GPU library.  The GPU library never
imports it.

build() compiles liboracle.so with g++ (-O2, OpenMP over tracks/seeds); load()
returns the ctypes handle, building on first use when the library is absent.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "kf_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

ST_PROP_FAIL = 1
ST_NEAR_TANGENT = 2
ST_ILLCOND = 4
ST_NONFINITE = 8
ST_BAD_INPUT = 16
ST_TERM_MISSES = 32


class OGeom(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("n_phi_bins", C.c_int32), ("n_z_bins", C.c_int32),
                ("pad", C.c_int32), ("B", C.c_double), ("sigma_rphi", C.c_double),
                ("sigma_z", C.c_double), ("sigma_r", C.c_double), ("mass", C.c_double),
                ("radius", C.c_double * 32), ("zhalf", C.c_double * 32),
                ("disk_z", C.c_double * 32), ("disk_rmin", C.c_double * 32), ("disk_rmax", C.c_double * 32),
                ("cyl_zmax", C.c_double * 32)]


class OModel(C.Structure):
    """The detector model of Sec. 3 (material map, energy loss, field)."""
    _fields_ = [("map", C.c_void_p), ("nz", C.c_int32), ("pad", C.c_int32), ("eloss", C.c_double),
                ("fr", C.c_double), ("fz", C.c_double)]


def _model(material, field):
    """(OModel or None, the float64 map it points to, kept alive by the caller)."""
    if material is None and field is None:
        return None, None
    material = (None, 0.0) if material is None else material
    field = (0.0, 0.0) if field is None else field
    xmap = None if material[0] is None else np.ascontiguousarray(material[0], np.float64)
    m = OModel(None if xmap is None else xmap.ctypes.data, 0 if xmap is None else int(xmap.shape[1]), 0,
               float(material[1]), float(field[0]), float(field[1]))
    return m, xmap


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _lib.oracle_total_chi2.restype = C.c_double
    return _lib


def num_threads() -> int:
    return int(load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (n < 1: all processors)."""
    load().oracle_set_num_threads(C.c_int(int(n)))


def ogeom(geom) -> OGeom:
    g = OGeom()
    g.n_layers = geom.n_layers
    g.n_phi_bins = geom.n_phi_bins
    g.n_z_bins = geom.n_z_bins
    g.B = geom.B
    g.sigma_rphi = geom.sigma_rphi
    g.sigma_z = geom.sigma_z
    g.sigma_r = geom.sigma_r
    g.mass = geom.mass
    for i in range(geom.n_layers):
        g.radius[i] = geom.radius[i]
        g.zhalf[i] = geom.zhalf[i]
        g.disk_z[i] = geom.disk_z[i]
        g.disk_rmin[i] = geom.disk_rmin[i]
        g.disk_rmax[i] = geom.disk_rmax[i]
        g.cyl_zmax[i] = geom.cyl_zmax[i]
    return g


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def propagate(state, center, r, B):
    out = np.zeros(6)
    s = C.c_double(0)
    st = np.ascontiguousarray(state, np.float64)
    ok = load().oracle_propagate(_p(st), C.c_double(center[0]), C.c_double(center[1]), C.c_double(r),
                                 C.c_double(B), _p(out), C.byref(s))
    return (out, s.value) if ok else (None, None)


def propagate_disk(state, zd, B):
    """Crossing with the plane z = zd: (state, arc) or (None, None)."""
    out = np.zeros(6)
    s = C.c_double(0)
    st = np.ascontiguousarray(state, np.float64)
    ok = load().oracle_propagate_disk(_p(st), C.c_double(zd), C.c_double(B), _p(out), C.byref(s))
    return (out, s.value) if ok else (None, None)


def measurement_disk(state, center, zd, m):
    """H (3x6) and residual on the disk plane z = zd centred at `center`."""
    H = np.zeros(18)
    r = np.zeros(3)
    st = np.ascontiguousarray(state, np.float64)
    mm = np.ascontiguousarray(m, np.float64)
    load().oracle_measurement_disk(_p(st), C.c_double(center[0]), C.c_double(center[1]), C.c_double(zd), _p(mm),
                                   _p(H), _p(r))
    return H.reshape(3, 6), r


def transport_jacobian(state, s, B):
    J = np.zeros(36)
    st = np.ascontiguousarray(state, np.float64)
    load().oracle_transport_jacobian(_p(st), C.c_double(s), C.c_double(B), _p(J))
    return J.reshape(6, 6)


def helix_at(state, s, B):
    out = np.zeros(6)
    st = np.ascontiguousarray(state, np.float64)
    load().oracle_helix_at(_p(st), C.c_double(s), C.c_double(B), _p(out))
    return out


def measurement(state, center, m):
    H = np.zeros(18)
    r = np.zeros(3)
    st = np.ascontiguousarray(state, np.float64)
    mm = np.ascontiguousarray(m, np.float64)
    load().oracle_measurement(_p(st), C.c_double(center[0]), C.c_double(center[1]), _p(mm), _p(H), _p(r))
    return H.reshape(3, 6), r


def scattering(geom, state, center, xX0, zd=0.0):
    """Q (6x6) at a state on a cylinder centred at `center`, or on the disk z = zd."""
    Q = np.zeros(36)
    g = ogeom(geom)
    st = np.ascontiguousarray(state, np.float64)
    load().oracle_scattering(C.byref(g), _p(st), C.c_double(center[0]), C.c_double(center[1]),
                             C.c_double(xX0), C.c_double(zd), _p(Q))
    return Q.reshape(6, 6)


def kalman_update(x, Cm, H, V, r):
    x = np.array(x, np.float64)
    Cm = np.array(Cm, np.float64)
    H = np.ascontiguousarray(H, np.float64)
    V = np.ascontiguousarray(V, np.float64)
    r = np.ascontiguousarray(r, np.float64)
    n, m = x.shape[0], r.shape[0]
    chi2 = C.c_double(0)
    ok = load().oracle_kalman_update(n, m, _p(x), _p(Cm), _p(H), _p(V), _p(r), C.byref(chi2))
    if not ok:
        raise ValueError("singular S")
    return x, Cm, chi2.value


def rts_step(xf, Cf, J, xp, Cp, xs1, Cs1, wrap_idx=-1):
    """One Rauch-Tung-Striebel step (dense, n <= 6): smoothed (x, C) at step l from the
    filtered one at l and the prediction and smoothed estimate at l + 1."""
    n = len(xf)
    a = [np.ascontiguousarray(v, np.float64) for v in (xf, Cf, J, xp, Cp, xs1, Cs1)]
    xs = np.zeros(n)
    Cs = np.zeros((n, n))
    ok = load().oracle_rts_step(n, *[_p(v) for v in a], _p(xs), _p(Cs), int(wrap_idx))
    if not ok:
        raise ValueError("singular predicted covariance")
    return xs, Cs


def smooth(geom, hits, mask, align=None, xX0=None, seed_state=None, seed_cov=None, material=None, field=None):
    """Forward fit plus RTS smoother of every track.  Returns state [L][6][n],
    cov [L][21][n] (layers 0..lend, zero beyond), lend [n] (last layer with an update,
    -1 if none) and the forward status [n].  material / field: the detector model as
    for fit() (each step's linearisation then includes the energy loss)."""
    dt = np.float64 if np.asarray(hits).dtype == np.float64 else np.float32
    hits = np.ascontiguousarray(hits, dt)
    mask = np.ascontiguousarray(mask, np.uint32)
    L, _, n = hits.shape
    from_hits = seed_state is None
    ss = None if from_hits else np.ascontiguousarray(seed_state, dt)
    sc = None if from_hits else np.ascontiguousarray(seed_cov, dt)
    out = dict(state=np.zeros((L, 6, n)), cov=np.zeros((L, 21, n)), lend=np.zeros(n, np.int32),
               status=np.zeros(n, np.uint32))
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    fn = load().oracle_smooth_f64 if dt == np.float64 else load().oracle_smooth
    model, _keep = _model(material, field)
    fn(C.byref(g), _p(_f64(align)), _p(_f64(xx)), None if model is None else C.byref(model), C.c_int64(n),
       _p(hits), _p(mask),
                         int(from_hits), _p(ss), _p(sc), _p(out["state"]), _p(out["cov"]), _p(out["lend"]),
                         _p(out["status"]))
    return out


def smooth_filtered(geom, state, cov, lend, align=None, xX0=None, material=None, field=None):
    """The RTS pass alone over given filtered estimates: state [L][6][n] and cov
    [L][21][n] after each layer (any float type; read as float64), lend [n] the last
    updated layer.  Returns state/cov as smooth() for layers first..lend (zero
    elsewhere) and first [n] (the lowest layer reached, -1 if lend < 0)."""
    state = np.ascontiguousarray(state, np.float64)
    cov = np.ascontiguousarray(cov, np.float64)
    lend = np.ascontiguousarray(lend, np.int32)
    L, _, n = state.shape
    out = dict(state=np.zeros((L, 6, n)), cov=np.zeros((L, 21, n)), first=np.zeros(n, np.int32))
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    model, _keep = _model(material, field)
    load().oracle_smooth_filtered(C.byref(g), _p(_f64(align)), _p(_f64(xx)), None if model is None else C.byref(model),
                                  C.c_int64(n), _p(lend), _p(state),
                                  _p(cov), _p(out["state"]), _p(out["cov"]), _p(out["first"]))
    return out


def material_step(geom, l, state, cov, material, xX0=0.0, align=None):
    """The material of layer l applied to a state at its crossing (Sec. 3): multiple
    scattering with the layer's x/X0 (the map's value at the crossing's z if
    material[0] is a map [L][nz], else xX0), then the mean ionisation loss
    material[1] * x_eff / beta^2.  Returns (state, cov) or None if the particle stops."""
    g = ogeom(geom)
    x = np.array(state, np.float64)
    Cm = np.array(cov, np.float64).reshape(36)
    xmap = None if material[0] is None else np.ascontiguousarray(material[0], np.float64)
    nz = 0 if xmap is None else int(xmap.shape[1])
    ok = load().oracle_material_step(C.byref(g), int(l), _p(_f64(align)), C.c_double(xX0), _p(xmap), C.c_int(nz),
                                     C.c_double(float(material[1])), _p(x), _p(Cm))
    return (x, Cm.reshape(6, 6)) if ok else None


def seed(geom, m0, m1, m2):
    st = np.zeros(6)
    cv = np.zeros(36)
    g = ogeom(geom)
    a, b, c = (np.ascontiguousarray(v, np.float64) for v in (m0, m1, m2))
    load().oracle_seed(C.byref(g), _p(a), _p(b), _p(c), _p(st), _p(cv))
    return st, cv.reshape(6, 6)


def fit(geom, hits, mask, align=None, xX0=None, seed_state=None, seed_cov=None, records=False, material=None,
        field=None):
    """Batched FP64 fit; seeds from hits 0-2 unless seed_state/seed_cov are given.

    hits [L][3][n] float32 (float64 hits select the float64-input entry), mask [n]
    uint32.  Returns a dict of float64 outputs; records=True adds records [n][L][27],
    the state and packed covariance after each processed layer (NaN beyond).
    material = (xX0_map [L][nz] or None, eloss GeV per X0): the material model of
    Sec. 3, see material_step.  field = (c_r, c_z): the field B_z(r, z) =
    B (1 + c_r r^2 + c_z z^2) (cm), each step the helix of the field at its start and the
    seed's curvature converted with the field at hit 0.
    """
    dt = np.float64 if np.asarray(hits).dtype == np.float64 else np.float32
    hits = np.ascontiguousarray(hits, dt)
    mask = np.ascontiguousarray(mask, np.uint32)
    L, _, n = hits.shape
    from_hits = seed_state is None
    ss = None if from_hits else np.ascontiguousarray(seed_state, dt)
    sc = None if from_hits else np.ascontiguousarray(seed_cov, dt)
    out = dict(state=np.zeros((6, n)), cov=np.zeros((21, n)), chi2=np.zeros(n),
               ndf=np.zeros(n, np.int32), status=np.zeros(n, np.uint32))
    rec = np.zeros((n, L, 27)) if records else None
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    if material is not None or field is not None:
        material = (None, 0.0) if material is None else material
        field = (0.0, 0.0) if field is None else field
        xmap = None if material[0] is None else np.ascontiguousarray(material[0], np.float64)
        nz = 0 if xmap is None else int(xmap.shape[1])
        fn = load().oracle_fit_model_f64 if dt == np.float64 else load().oracle_fit_model
        fn(C.byref(g), _p(_f64(align)), _p(_f64(xx)), _p(xmap), C.c_int(nz),
                                C.c_double(float(material[1])), C.c_double(float(field[0])),
                                C.c_double(float(field[1])), C.c_int64(n), _p(hits), _p(mask),
                                int(from_hits), _p(ss), _p(sc), _p(out["state"]), _p(out["cov"]),
                                _p(out["chi2"]), _p(out["ndf"]), _p(out["status"]), _p(rec))
    else:
        fn = load().oracle_fit_f64 if dt == np.float64 else load().oracle_fit
        fn(C.byref(g), _p(_f64(align)), _p(_f64(xx)), C.c_int64(n), _p(hits), _p(mask),
           int(from_hits), _p(ss), _p(sc), _p(out["state"]), _p(out["cov"]), _p(out["chi2"]),
           _p(out["ndf"]), _p(out["status"]), _p(rec))
    if records:
        out["records"] = rec
    return out


def reverse_state(state, cov=None):
    """The same particle run backwards: the path traced in the opposite direction is
    that of the opposite charge, so (x, y, z, kappa, phi, theta) -> (x, y, z, -kappa,
    phi + pi, pi - theta); the covariance follows with D = diag(1, 1, 1, -1, 1, -1).
    Its own inverse.  state [6][n], cov [21][n] packed."""
    x = np.array(state, np.float64)
    x[3] = -x[3]
    x[4] = (x[4] + 2 * np.pi) % (2 * np.pi) - np.pi   # phi + pi, wrapped to [-pi, pi)
    x[5] = np.pi - x[5]
    if cov is None:
        return x
    d = np.array([1.0, 1.0, 1.0, -1.0, 1.0, -1.0])
    c = np.array(cov, np.float64).copy()
    for i in range(6):
        for j in range(i + 1):
            c[i * (i + 1) // 2 + j] *= d[i] * d[j]
    return x, c


def fit_outside_in(geom, hits, mask, seed_state=None, seed_cov=None, align=None, xX0=None):
    """Outside-in fit (the backward propagation and final fit of Sec. 4.2 and Sec. 5):
    every track is filtered from its outermost hit layer inwards, seeded there from its
    three outermost hits as fit() seeds from the three innermost (these must be the
    three outermost layers the track reaches), or by seed_state [6][n] / seed_cov [21][n]
    (the particle's own direction; the position on that layer's surface), and the
    estimate at its innermost hit layer is returned as fit() returns the outermost one.  The backward pass is the forward filter of the
    reversed particle (reverse_state) through the layers in reverse order: each layer's
    scattering is added where the reversed particle reaches it, i.e. on the side of the
    layer nearer the beam, and the innermost layer's own material enters the result (its
    direction is the one before that layer)."""
    hits = np.asarray(hits)
    mask = np.ascontiguousarray(mask, np.uint32)
    L, _, n = hits.shape
    xx = np.asarray(geom.xX0 if xX0 is None else xX0, np.float64)
    al = np.zeros((L, 4)) if align is None else np.asarray(align, np.float64)
    rs, rc = (None, None) if seed_state is None else reverse_state(seed_state, seed_cov)
    out = dict(state=np.zeros((6, n)), cov=np.zeros((21, n)), chi2=np.zeros(n), ndf=np.zeros(n, np.int32),
               status=np.zeros(n, np.uint32))
    last = np.array([int(m).bit_length() - 1 for m in mask])
    for m in np.unique(last):
        if m < 0:
            continue
        sel = np.nonzero(last == m)[0]
        ls = np.arange(m, -1, -1)   # the layers, outermost first
        kw = {f: getattr(geom, f)[ls] for f in ("disk_z", "disk_rmin", "disk_rmax", "cyl_zmax")
              if getattr(geom, f, None) is not None}
        g = dataclasses.replace(geom, radius=geom.radius[ls], zhalf=geom.zhalf[ls], xX0=xx[ls], **kw)
        rmask = np.zeros(sel.size, np.uint32)
        for k, l in enumerate(ls):
            rmask |= ((mask[sel] >> np.uint32(l)) & np.uint32(1)) << np.uint32(k)
        o = fit(g, np.ascontiguousarray(hits[ls][:, :, sel]), rmask, align=np.ascontiguousarray(al[ls]),
                seed_state=None if rs is None else rs[:, sel], seed_cov=None if rc is None else rc[:, sel])
        st, cv = reverse_state(o["state"], o["cov"])
        out["state"][:, sel] = st
        out["cov"][:, sel] = cv
        for k in ("chi2", "ndf", "status"):
            out[k][sel] = o[k]
    return out


def total_chi2(geom, hits, mask, align, xX0, weight=None, field=None, material=None):
    """sum_i weight_i chi2_i of the FP64 fit (seeds from hits); field and material as
    for fit_grad()."""
    hits = np.ascontiguousarray(hits, np.float32)
    mask = np.ascontiguousarray(mask, np.uint32)
    g = ogeom(geom)
    fr, fz = (0.0, 0.0) if field is None else (float(field[0]), float(field[1]))
    xmap, eloss = (None, 0.0) if material is None else material
    xmap = None if xmap is None else np.ascontiguousarray(xmap, np.float64)
    nz = 0 if xmap is None else int(xmap.shape[1])
    return load().oracle_total_chi2(C.byref(g), _p(_f64(align)), _p(_f64(xX0)), C.c_int64(hits.shape[2]),
                                    _p(hits), _p(mask), _p(_f64(weight)), C.c_double(fr), C.c_double(fz), _p(xmap),
                                    C.c_int32(nz), C.c_double(float(eloss)))


def fit_grad(geom, hits, mask, align, xX0, weight=None, field=None, material=None):
    """FP64 gradient of sum_i weight_i chi2_i w.r.t. align [L][4] and xX0 [L] (dual
    numbers).  field = (c_r, c_z): the parameterised field; the derivative includes the
    field's change where a parameter moves a step's start point or the seed's first hit.
    material = (xX0_map [L][nz] or None, eloss): the material model as for fit(); with a
    map the second result is the derivative w.r.t. an additive offset of each layer's
    map row (xX0 is then not used)."""
    hits = np.ascontiguousarray(hits, np.float32)
    mask = np.ascontiguousarray(mask, np.uint32)
    L = hits.shape[0]
    ga = np.zeros((L, 4))
    gx = np.zeros(L)
    g = ogeom(geom)
    fr, fz = (0.0, 0.0) if field is None else (float(field[0]), float(field[1]))
    xmap, eloss = (None, 0.0) if material is None else material
    xmap = None if xmap is None else np.ascontiguousarray(xmap, np.float64)
    nz = 0 if xmap is None else int(xmap.shape[1])
    load().oracle_fit_grad(C.byref(g), _p(_f64(align)), _p(_f64(xX0)), C.c_int64(hits.shape[2]), _p(hits),
                           _p(mask), _p(_f64(weight)), _p(ga), _p(gx), C.c_double(fr), C.c_double(fz), _p(xmap),
                           C.c_int32(nz), C.c_double(float(eloss)))
    return ga, gx


def loss_map(geom, eloss, kappa, theta, xe):
    """(kappa1, dkappa1/dkappa, dkappa1/dtheta) of the mean energy loss over a path of
    xe radiation lengths, or None if the particle stops."""
    out = np.zeros(3)
    ok = load().oracle_loss_map(C.byref(ogeom(geom)), C.c_double(eloss), C.c_double(kappa), C.c_double(theta),
                                C.c_double(xe), _p(out))
    return out if ok else None


def find(geom, ev, chi2_cut=30.0, nsigma=3.0, keep=6, max_miss=3, brute=False, refit=False,
         align=None, xX0=None, tol_abs=0.05, tol_rel=1e-4, tol_win=5e-3, material=None, field=None):
    """FP64 combinatorial search of every seed of a synth.EventBatch; material and
    field as for fit() (the detector model in every prediction and in the refit).
    The result's "work" counts what the search did: predictions that reached their
    layer, hits inside a window (each given a chi2), updates of surviving hit branches,
    and seed refits (one per seed)."""
    L = geom.n_layers
    S = ev.seed_hits.shape[1]
    H = ev.hits.shape[1]
    hits = np.ascontiguousarray(ev.hits, np.float32)
    off = np.ascontiguousarray(ev.hit_off, np.int64)
    sev = np.ascontiguousarray(ev.seed_event, np.int32)
    sh = np.ascontiguousarray(ev.seed_hits, np.int32)
    o = dict(n_cand=np.zeros(S, np.int32), hit_idx=np.zeros((keep, L, S), np.int32),
             n_hits=np.zeros((keep, S), np.int32), n_miss=np.zeros((keep, S), np.int32),
             chi2=np.zeros((keep, S)), state=np.zeros((keep, 6, S)), cov=np.zeros((keep, 21, S)),
             status=np.zeros((keep, S), np.uint32), ambig=np.zeros(S, np.uint32), work=np.zeros(4, np.int64))
    if refit:
        o.update(rf_state=np.zeros((6, S)), rf_cov=np.zeros((21, S)), rf_chi2=np.zeros(S),
                 rf_ndf=np.zeros(S, np.int32), rf_status=np.zeros(S, np.uint32))
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    model, _keep = _model(material, field)
    load().oracle_find(C.byref(g), _p(_f64(align)), _p(_f64(xx)), None if model is None else C.byref(model),
                       C.c_int32(off.shape[0]), _p(off),
                       C.c_int64(H), _p(hits), C.c_int64(S), _p(sev), _p(sh), C.c_double(chi2_cut),
                       C.c_double(nsigma), C.c_int32(keep), C.c_int32(max_miss), C.c_int32(int(brute)),
                       C.c_double(tol_abs), C.c_double(tol_rel), C.c_double(tol_win),
                       _p(o["n_cand"]), _p(o["hit_idx"]), _p(o["n_hits"]), _p(o["n_miss"]), _p(o["chi2"]),
                       _p(o["state"]), _p(o["cov"]), _p(o["status"]), _p(o["ambig"]),
                       _p(o.get("rf_state")), _p(o.get("rf_cov")), _p(o.get("rf_chi2")),
                       _p(o.get("rf_ndf")), _p(o.get("rf_status")), _p(o["work"]))
    return o


def unpack_cov(c21):
    """[21, ...] packed lower triangle -> [6, 6, ...] symmetric."""
    c21 = np.asarray(c21)
    out = np.zeros((6, 6) + c21.shape[1:], dtype=c21.dtype)
    k = 0
    for i in range(6):
        for j in range(i + 1):
            out[i, j] = c21[k]
            out[j, i] = c21[k]
            k += 1
    return out


# Duplicate handling (Sec. 4.2).  The cuts are this project's readings (the paper
# gives none); both the oracle and the library take them as arguments.
SEED_CUTS = dict(psi_window=0.05, min_shared=2, min_shared_kin=1, kap_rel=0.1, kap_abs=0.15, theta=0.03,
                 phi=0.02, z=0.5)
TRACK_CUTS = dict(psi_window=0.05, shared_frac=0.5, kap_rel=0.1, kap_abs=0.01, theta=0.02)


def clean_seeds(geom, ev, cuts=None, align=None, xX0=None):
    """Seed cleaning of a synth.EventBatch's seeds: keep [S] (1 kept, 0 removed as the
    duplicate of a lower-index seed) and sens [S] (a decision within float rounding of
    a cut)."""
    c = dict(SEED_CUTS, **(cuts or {}))
    S = ev.seed_hits.shape[1]
    H = ev.hits.shape[1]
    keep = np.zeros(S, np.int32)
    sens = np.zeros(S, np.uint8)
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    off = np.ascontiguousarray(ev.hit_off, np.int64)
    load().oracle_clean_seeds(C.byref(g), _p(_f64(align)), _p(_f64(xx)), C.c_int32(off.shape[0]),
                              _p(np.ascontiguousarray(ev.hits, np.float32)), C.c_int64(H), _p(off), C.c_int64(S),
                              _p(np.ascontiguousarray(ev.seed_event, np.int32)),
                              _p(np.ascontiguousarray(ev.seed_hits, np.int32)), C.c_double(c["psi_window"]),
                              C.c_int32(c["min_shared"]), C.c_int32(c["min_shared_kin"]),
                              C.c_double(c["kap_rel"]), C.c_double(c["kap_abs"]),
                              C.c_double(c["theta"]), C.c_double(c["phi"]), C.c_double(c["z"]), _p(keep), _p(sens))
    return keep, sens.astype(bool)


def remove_duplicates(geom, hits, n_events, event, hit_idx, n_hits, chi2, state, cuts=None, align=None, xX0=None):
    """Duplicate removal over built tracks: event [n], hit_idx [L][n] global hit indices
    into hits [3][H] (< 0: none), n_hits [n], chi2 [n], state [6][n] (kappa and theta
    used).  Priority: more hits, lower chi2, lower index.  Returns keep [n], sens [n]."""
    c = dict(TRACK_CUTS, **(cuts or {}))
    n = int(np.asarray(event).shape[0])
    keep = np.zeros(n, np.int32)
    sens = np.zeros(n, np.uint8)
    g = ogeom(geom)
    xx = geom.xX0 if xX0 is None else xX0
    h = np.ascontiguousarray(hits, np.float32)
    load().oracle_remove_duplicates(C.byref(g), _p(_f64(align)), _p(_f64(xx)), C.c_int32(int(n_events)), _p(h),
                                    C.c_int64(h.shape[1]), C.c_int64(n), _p(np.ascontiguousarray(event, np.int32)),
                                    _p(np.ascontiguousarray(hit_idx, np.int32)),
                                    _p(np.ascontiguousarray(n_hits, np.int32)),
                                    _p(np.ascontiguousarray(chi2, np.float32)),
                                    _p(np.ascontiguousarray(state, np.float32)), C.c_double(c["psi_window"]),
                                    C.c_double(c["shared_frac"]), C.c_double(c["kap_rel"]), C.c_double(c["kap_abs"]),
                                    C.c_double(c["theta"]), _p(keep), _p(sens))
    return keep, sens.astype(bool)
