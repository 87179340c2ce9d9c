"""The C ABI without a GPU: the library loads, exports what include/kf.h declares, and
host-side validation returns the documented codes before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_1906_11744_amd import kf
    return kf, kf._lib()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "kf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char\*)\s+(kf_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_three_calls():
    names = declared_functions()
    for n in ("kf_fit", "kf_find", "kf_fit_backward", "kf_ctx_create", "kf_workspace_size", "kf_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    kf, lib = _lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(kf.exported_symbols()) == declared_functions()


def test_context_validation():
    kf, lib = _lib()
    geom = synth.workload_geometry(2)
    ctx = kf.Context(geom)
    assert ctx.n_layers == 17
    ctx.set_fallback_threshold(0.5)
    with pytest.raises(kf.KfError):
        ctx.set_fallback_threshold(-1.0)
    bad = synth.workload_geometry(2)
    bad.radius = bad.radius[::-1].copy()
    with pytest.raises(kf.KfError) as e:
        kf.Context(bad)
    assert e.value.code == -1
    g = kf.Geometry()
    g.n_layers = 40
    h = C.c_void_p()
    assert lib.kf_ctx_create(C.byref(g), C.byref(h)) == -1


def test_host_side_errors_before_launch():
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    fin = kf.FitIn(0, None, None, None, None, 1)
    fo = kf.FitOut()
    p = kf.LayerParams()
    # empty batch: nothing to do
    assert lib.kf_fit(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None) == 0
    # missing arrays
    fin = kf.FitIn(10, None, None, None, None, 1)
    assert lib.kf_fit(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None) == -1
    fin = kf.FitIn(-1, None, None, None, None, 1)
    assert lib.kf_fit(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None) == -1
    nb = C.c_size_t(1)
    assert lib.kf_workspace_size(ctx._h, kf.KF_OP_FIT, C.byref(fin), C.byref(nb)) == 0
    assert nb.value == 0   # the fit builds its layer table in LDS
    fin = kf.FitIn(10, None, None, None, None, 1)
    assert lib.kf_workspace_size(ctx._h, kf.KF_OP_FIT_BACKWARD, C.byref(fin), C.byref(nb)) == 0
    assert nb.value >= 256
    fin = kf.FindIn(1, None, 100, None, 10, None, None, 30.0, 3.0, 6, 3, 0)
    assert lib.kf_workspace_size(ctx._h, kf.KF_OP_FIND, C.byref(fin), C.byref(nb)) == 0
    assert nb.value >= 100 * 20
    assert lib.kf_workspace_size(ctx._h, 99, C.byref(fin), C.byref(nb)) == -2
    assert lib.kf_strerror(-3).decode().startswith("workspace")


def test_find_config_roundtrip_and_validation():
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(3))
    base = {"wide_window_bins": 16, "blocks_per_cu": 0, "use_graph": 0, "n_phi_bins": 0, "n_z_bins": 0,
            "lanes_per_seed": 0}
    assert ctx.find_config() == base
    ctx.set_find_config(wide_window_bins=0, blocks_per_cu=1, use_graph=1, n_phi_bins=512, n_z_bins=64,
                        lanes_per_seed=6)
    want = {"wide_window_bins": 0, "blocks_per_cu": 1, "use_graph": 1, "n_phi_bins": 512, "n_z_bins": 64,
            "lanes_per_seed": 6}
    assert ctx.find_config() == want
    with pytest.raises(kf.KfError):
        ctx.set_find_config(wide_window_bins=-1)
    with pytest.raises(kf.KfError):
        ctx.set_find_config(blocks_per_cu=-2)
    with pytest.raises(kf.KfError):
        ctx.set_find_config(use_graph=2)
    with pytest.raises(kf.KfError):        # 1024 x 64 bins: beyond KF_MAX_FIND_BINS
        ctx.set_find_config(n_phi_bins=1024)
    with pytest.raises(kf.KfError):
        ctx.set_find_config(n_z_bins=257)
    with pytest.raises(kf.KfError):        # 512 x 128 bins
        ctx.set_find_config(n_phi_bins=512, n_z_bins=128)
    for bad in (5, 7, 16, -1):
        with pytest.raises(kf.KfError):
            ctx.set_find_config(lanes_per_seed=bad)
    assert ctx.find_config() == want
    ctx.set_find_config(n_phi_bins=1024, n_z_bins=32)   # 32 768 bins: the limit
    assert ctx.find_config()["n_phi_bins"] == 1024


def test_launch_event_hook_validation():
    """kf_ctx_set_launch_events takes both events or neither (no device work here)."""
    import ctypes as C
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    assert lib.kf_ctx_set_launch_events(None, None, None) == -1   # KF_E_INVALID
    fake = C.c_void_p(0x1000)   # never dereferenced: only stored, and cleared again
    assert lib.kf_ctx_set_launch_events(ctx._h, fake, None) == -1
    assert lib.kf_ctx_set_launch_events(ctx._h, None, fake) == -1
    assert lib.kf_ctx_set_launch_events(ctx._h, fake, fake) == 0
    assert lib.kf_ctx_set_launch_events(ctx._h, None, None) == 0


def test_dedup_cuts_defaults_roundtrip_and_validation():
    """The library's default duplicate cuts are the oracle's; set/get round-trips; bad
    cuts are refused (host only)."""
    import oracle
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    c = ctx.dedup_cuts()
    s, t = oracle.SEED_CUTS, oracle.TRACK_CUTS
    assert c["psi_window"] == np.float32(s["psi_window"]) == np.float32(t["psi_window"])
    assert (c["min_shared"], c["min_shared_kin"]) == (s["min_shared"], s["min_shared_kin"])
    for k_lib, v in (("seed_kap_rel", s["kap_rel"]), ("seed_kap_abs", s["kap_abs"]), ("seed_theta", s["theta"]),
                     ("seed_phi", s["phi"]), ("seed_z", s["z"]), ("trk_shared_frac", t["shared_frac"]),
                     ("trk_kap_rel", t["kap_rel"]), ("trk_kap_abs", t["kap_abs"]), ("trk_theta", t["theta"])):
        assert c[k_lib] == np.float32(v), k_lib
    ctx.set_dedup_cuts(psi_window=0.1, min_shared=3)
    assert ctx.dedup_cuts()["psi_window"] == np.float32(0.1) and ctx.dedup_cuts()["min_shared"] == 3
    for bad in (dict(psi_window=0.0), dict(seed_theta=-1.0), dict(min_shared=0, min_shared_kin=1)):
        with pytest.raises(kf.KfError):
            ctx.set_dedup_cuts(**bad)
    assert ctx.dedup_cuts()["psi_window"] == np.float32(0.1)


def test_dedup_calls_reject_bad_arguments_before_launch():
    """kf_clean_seeds / kf_remove_duplicates: empty input is a no-op; NULL context,
    input or arrays and negative counts are refused before anything is launched."""
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    keep = C.c_void_p(0x1000)    # never dereferenced on these paths
    fin = kf.FindIn(1, None, 0, None, 0, None, None, 0.0, 0.0, 1, 1, 0)
    assert lib.kf_clean_seeds(ctx._h, None, C.byref(fin), None, None, 0, None) == 0     # n_seeds = 0
    fin = kf.FindIn(1, None, 0, None, 5, None, None, 0.0, 0.0, 1, 1, 0)
    assert lib.kf_clean_seeds(ctx._h, None, C.byref(fin), keep, None, 0, None) == -1    # missing arrays
    assert lib.kf_clean_seeds(None, None, C.byref(fin), keep, None, 0, None) == -1
    fin = kf.FindIn(-1, None, 0, None, 5, None, None, 0.0, 0.0, 1, 1, 0)
    assert lib.kf_clean_seeds(ctx._h, None, C.byref(fin), keep, None, 0, None) == -1    # n_events < 0
    tin = kf.TracksIn(1, 0, None, 0, None, None, None, None, None)
    assert lib.kf_remove_duplicates(ctx._h, None, C.byref(tin), None, None, 0, None) == 0
    tin = kf.TracksIn(1, 0, None, 3, None, None, None, None, None)
    assert lib.kf_remove_duplicates(ctx._h, None, C.byref(tin), keep, None, 0, None) == -1
    tin = kf.TracksIn(1, -2, None, 3, None, None, None, None, None)
    assert lib.kf_remove_duplicates(ctx._h, None, C.byref(tin), keep, None, 0, None) == -1
    assert lib.kf_remove_duplicates(ctx._h, None, None, keep, None, 0, None) == -1
    # workspace sizes grow with the items and the events
    nb = C.c_size_t(0)
    fin = kf.FindIn(64, None, 0, None, 1000, None, None, 0.0, 0.0, 1, 1, 0)
    assert lib.kf_workspace_size(ctx._h, kf.KF_OP_CLEAN_SEEDS, C.byref(fin), C.byref(nb)) == 0
    small = nb.value
    fin = kf.FindIn(64, None, 0, None, 100000, None, None, 0.0, 0.0, 1, 1, 0)
    assert lib.kf_workspace_size(ctx._h, kf.KF_OP_CLEAN_SEEDS, C.byref(fin), C.byref(nb)) == 0
    assert nb.value > small + 100000 * 40


def test_material_setting_validation_and_the_calls_it_excludes():
    """kf_ctx_set_material stores its arguments (no device work here); the finder, the
    smoother and the adjoint take the model and go on to their own checks (here: the
    missing workspace)."""
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    fake = C.c_void_p(0x1000)   # never dereferenced: no kf_fit is called here
    assert lib.kf_ctx_set_material(None, None, 0, C.c_float(0.0)) == -1
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(-1.0)) == -1
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(float("nan"))) == -1
    assert lib.kf_ctx_set_material(ctx._h, fake, 0, C.c_float(0.0)) == -1
    assert lib.kf_ctx_set_material(ctx._h, fake, 65, C.c_float(0.0)) == -1
    fin = kf.FindIn(1, fake, 100, fake, 10, fake, fake, 30.0, 3.0, 6, 3, 0)
    fo = kf.FindOut(*([fake] * 13))
    p = kf.LayerParams()
    fit_in = kf.FitIn(10, fake, fake, None, None, 1)
    fit_out = kf.FitOut(fake, fake, fake, fake, fake, fake)
    so = kf.SmoothOut(fake, fake, fake, fake)

    def codes():
        return (lib.kf_find(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None),
                lib.kf_smooth(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), C.byref(so), None, 0, None),
                lib.kf_fit_backward(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), fake, fake, fake,
                                    None, 0, None))
    # without a material setting each call stops at its missing workspace instead
    assert codes() == (-3, -3, -3)
    for args in ((fake, 1, 0.0), (fake, 64, 0.0363), (None, 0, 0.0363)):
        assert lib.kf_ctx_set_material(ctx._h, args[0], args[1], C.c_float(args[2])) == 0
        assert codes() == (-3, -3, -3), args
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(0.0)) == 0
    assert codes() == (-3, -3, -3)


def test_field_setting_validation_and_the_calls_it_excludes():
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    assert lib.kf_ctx_set_field(None, C.c_float(0.0), C.c_float(0.0)) == -1
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(float("inf")), C.c_float(0.0)) == -1
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(0.0), C.c_float(float("nan"))) == -1
    fake = C.c_void_p(0x1000)
    p = kf.LayerParams()
    fit_in = kf.FitIn(10, fake, fake, None, None, 1)
    fit_out = kf.FitOut(fake, fake, fake, fake, fake, fake)
    so = kf.SmoothOut(fake, fake, fake, fake)
    back = lambda: lib.kf_fit_backward(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), fake, fake, fake,
                                       None, 0, None)
    assert back() == -3
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(-1e-6), C.c_float(-4e-6)) == 0
    assert back() == -3           # the adjoint takes the field: it stops at the workspace
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(0.0363)) == 0
    assert back() == -3           # and the energy loss
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(0.0)) == 0
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(0.0), C.c_float(0.0)) == 0
    assert back() == -3
    g0 = synth.workload_geometry(2)
    g0.B = 0.0
    ctx0 = kf.Context(g0)
    assert lib.kf_ctx_set_field(ctx0._h, C.c_float(0.0), C.c_float(-4e-6)) == -2
    assert lib.kf_ctx_set_field(ctx0._h, C.c_float(0.0), C.c_float(0.0)) == 0


def test_static_backward_rejects_requests_beyond_its_scratch():
    """kf_fit_backward_static checks the size on the host and returns KF_E_SCRATCH
    before anything is launched (the pointers below are never dereferenced); a request
    that fits passes that check (and would launch: not run here)."""
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    assert lib.kf_static_scratch_bytes() == 16 << 20
    fake = C.c_void_p(256)
    ws = C.c_size_t()
    for n, fits in [(2_000_000, False), (1_500_000, True)]:
        fin = kf.FitIn(n, fake, fake, None, None, 1)
        assert lib.kf_workspace_size(ctx._h, kf.KF_OP_FIT_BACKWARD, C.byref(fin), C.byref(ws)) == 0
        assert (ws.value <= lib.kf_static_scratch_bytes()) == fits
    fin = kf.FitIn(2_000_000, fake, fake, None, None, 1)
    fo = kf.FitOut(fake, fake, fake, fake, fake, fake)
    p = kf.LayerParams(None, None)
    rc = lib.kf_fit_backward_static(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), fake, fake, fake, None)
    assert rc == -5 and b"static scratch" in lib.kf_strerror(rc)
    # argument errors come first, as for kf_fit_backward
    assert lib.kf_fit_backward_static(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), fake, None, fake, None) == -1


def test_endcap_geometry_validation_and_the_calls_it_excludes():
    """Disks and bounded cylinders: the seed layers must be cylinders, a disk needs
    0 <= rmin < rmax and no z bound, cylinder radii increase over the cylinders only;
    with bounded surfaces the material model, the field, the smoother and the adjoint
    refuse before launching, while kf_find goes on to its own checks."""
    kf, lib = _lib()
    geom = synth.barrel_endcap(xX0=0.02)
    ctx = kf.Context(geom)
    assert ctx.n_layers == 31
    for field, l, v in [("disk_z", 1, 50.0),          # a disk among the seed layers
                        ("disk_rmin", 20, 120.0),     # rmin above rmax
                        ("disk_rmin", 20, -1.0),
                        ("cyl_zmax", 20, 10.0),       # a z bound on a disk
                        ("disk_rmax", 3, 10.0),       # disk radii on a cylinder
                        ("cyl_zmax", 3, -5.0)]:
        bad = synth.barrel_endcap(xX0=0.02)
        getattr(bad, field)[l] = v
        with pytest.raises(kf.KfError) as e:
            kf.Context(bad)
        assert e.value.code == -1, (field, l)
    bad = synth.barrel_endcap(xX0=0.02)
    bad.radius[16] = bad.radius[15]       # two cylinders at one radius
    with pytest.raises(kf.KfError):
        kf.Context(bad)
    fake = C.c_void_p(0x1000)   # never dereferenced
    assert lib.kf_ctx_set_material(ctx._h, fake, 16, C.c_float(0.0)) == -2
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(0.0363)) == -2
    assert lib.kf_ctx_set_material(ctx._h, None, 0, C.c_float(0.0)) == 0
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(-1e-6), C.c_float(0.0)) == -2
    assert lib.kf_ctx_set_field(ctx._h, C.c_float(0.0), C.c_float(0.0)) == 0
    p = kf.LayerParams()
    fit_in = kf.FitIn(10, fake, fake, None, None, 1)
    fit_out = kf.FitOut(fake, fake, fake, fake, fake, fake)
    so = kf.SmoothOut(fake, fake, fake, fake)
    assert lib.kf_smooth(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), C.byref(so), None, 0, None) == -2
    assert lib.kf_fit_backward(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), fake, fake, fake,
                               None, 0, None) == -2
    assert lib.kf_fit_backward_static(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), fake, fake, fake,
                                      None) == -2
    fin = kf.FindIn(1, fake, 100, fake, 10, fake, fake, 30.0, 3.0, 6, 3, 0)
    fo = kf.FindOut(*([fake] * 13))
    assert lib.kf_find(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None) == -3


def test_sparse_checkpoint_arguments():
    """ckpt_every: 0..KF_MAX_LAYERS (0 and 1 keep every layer); the adjoint's workspace
    grows by the recomputed segment [k-1][27][n]; the smoother refuses k > 1; each error
    before anything is launched."""
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    fake = C.c_void_p(0x1000)
    fo = kf.FitOut(fake, fake, fake, fake, fake, fake)
    p = kf.LayerParams()
    for bad in (-1, 33):
        fin = kf.FitIn(10, fake, fake, None, None, 1, bad)
        assert lib.kf_fit(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), None, 0, None) == -1
        assert lib.kf_fit_backward(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), fake, fake, fake, None, 0,
                                   None) == -1
    ws = C.c_size_t()
    sizes = {}
    for k in (0, 1, 2, 4):
        fin = kf.FitIn(100_000, fake, fake, None, None, 1, k)
        assert lib.kf_workspace_size(ctx._h, kf.KF_OP_FIT_BACKWARD, C.byref(fin), C.byref(ws)) == 0
        sizes[k] = ws.value
    assert sizes[0] == sizes[1]
    seg = lambda k: -(-(k - 1) * 27 * 100_000 * 4 // 256) * 256
    assert sizes[2] - sizes[1] == seg(2) and sizes[4] - sizes[1] == seg(4)
    so = kf.SmoothOut(fake, fake, fake, fake)
    fin = kf.FitIn(10, fake, fake, None, None, 1, 2)
    assert lib.kf_smooth(ctx._h, C.byref(p), C.byref(fin), C.byref(fo), C.byref(so), None, 0, None) == -2


def test_smooth_rejects_batches_beyond_its_row_offsets():
    """kf_smooth addresses each [.][n] row by 32-bit byte offsets: n above 2^29 is
    KF_E_INVALID before anything else; n = 2^29 goes on to the workspace check."""
    kf, lib = _lib()
    ctx = kf.Context(synth.workload_geometry(2))
    fake = C.c_void_p(0x1000)   # never dereferenced: both calls return before any launch
    p = kf.LayerParams()
    fit_out = kf.FitOut(fake, fake, fake, fake, fake, fake)
    so = kf.SmoothOut(fake, fake, fake, fake)
    for n, code in (((1 << 29) + 1, -1), (1 << 29, -3)):
        fit_in = kf.FitIn(n, fake, fake, None, None, 1)
        assert lib.kf_smooth(ctx._h, C.byref(p), C.byref(fit_in), C.byref(fit_out), C.byref(so), None, 0,
                             None) == code, n
