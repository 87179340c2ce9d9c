"""Python binding of libkf.so (include/kf.h): argument marshalling only.

Every step of the fit, the finder and the adjoint runs in the library's HIP kernels;
torch supplies device memory and the current stream.  There is no fallback: if the
library is not built or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkf.so")

KF_MAX_LAYERS = 32
KF_MAX_KEEP = 8
KF_OP_FIT, KF_OP_FIND, KF_OP_FIT_BACKWARD, KF_OP_SMOOTH = 1, 2, 3, 4
KF_OP_CLEAN_SEEDS, KF_OP_REMOVE_DUPLICATES = 5, 6

ST_PROP_FAIL = 1
ST_NEAR_TANGENT = 2
ST_FP64_FALLBACK = 4
ST_NONFINITE = 8
ST_BAD_INPUT = 16
ST_TERM_MISSES = 32


class KfError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {code} ({_lib().kf_strerror(code).decode()})")
        self.code = code


class Geometry(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("B_tesla", C.c_float),
                ("radius_cm", C.c_float * KF_MAX_LAYERS), ("zhalf_cm", C.c_float * KF_MAX_LAYERS),
                ("sigma_rphi_cm", C.c_float), ("sigma_z_cm", C.c_float), ("sigma_r_cm", C.c_float),
                ("mass_gev", C.c_float), ("n_phi_bins", C.c_int32), ("n_z_bins", C.c_int32),
                ("disk_z_cm", C.c_float * KF_MAX_LAYERS), ("disk_rmin_cm", C.c_float * KF_MAX_LAYERS),
                ("disk_rmax_cm", C.c_float * KF_MAX_LAYERS), ("cyl_zmax_cm", C.c_float * KF_MAX_LAYERS)]


class LayerParams(C.Structure):
    _fields_ = [("align", C.c_void_p), ("xX0", C.c_void_p)]


class FitIn(C.Structure):
    _fields_ = [("n", C.c_int64), ("hits", C.c_void_p), ("hit_mask", C.c_void_p),
                ("seed_state", C.c_void_p), ("seed_cov", C.c_void_p), ("seed_from_hits", C.c_int32),
                ("ckpt_every", C.c_int32)]


class FitOut(C.Structure):
    _fields_ = [("state", C.c_void_p), ("cov", C.c_void_p), ("chi2", C.c_void_p), ("ndf", C.c_void_p),
                ("status", C.c_void_p), ("ckpt", C.c_void_p)]


class FindIn(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("hit_off", C.c_void_p), ("n_hits", C.c_int64),
                ("hits", C.c_void_p), ("n_seeds", C.c_int64), ("seed_event", C.c_void_p),
                ("seed_hits", C.c_void_p), ("chi2_cut", C.c_float), ("nsigma", C.c_float),
                ("keep", C.c_int32), ("max_miss", C.c_int32), ("refit", C.c_int32)]


class FindOut(C.Structure):
    _fields_ = [("n_cand", C.c_void_p), ("hit_idx", C.c_void_p), ("n_hits", C.c_void_p),
                ("n_miss", C.c_void_p), ("chi2", C.c_void_p), ("state", C.c_void_p), ("cov", C.c_void_p),
                ("status", C.c_void_p), ("rf_state", C.c_void_p), ("rf_cov", C.c_void_p),
                ("rf_chi2", C.c_void_p), ("rf_ndf", C.c_void_p), ("rf_status", C.c_void_p)]


class DedupCuts(C.Structure):
    _fields_ = [("psi_window", C.c_float), ("min_shared", C.c_int32), ("min_shared_kin", C.c_int32),
                ("seed_kap_rel", C.c_float), ("seed_kap_abs", C.c_float), ("seed_theta", C.c_float),
                ("seed_phi", C.c_float), ("seed_z", C.c_float), ("trk_shared_frac", C.c_float),
                ("trk_kap_rel", C.c_float), ("trk_kap_abs", C.c_float), ("trk_theta", C.c_float)]


class TracksIn(C.Structure):
    _fields_ = [("n_events", C.c_int32), ("n_hits", C.c_int64), ("hits", C.c_void_p), ("n", C.c_int64),
                ("event", C.c_void_p), ("hit_idx", C.c_void_p), ("n_hits_trk", C.c_void_p),
                ("chi2", C.c_void_p), ("state", C.c_void_p)]


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        lib = C.CDLL(LIB_PATH)
        lib.kf_strerror.restype = C.c_char_p
        lib.kf_ctx_create.argtypes = [C.POINTER(Geometry), C.POINTER(C.c_void_p)]
        lib.kf_ctx_destroy.argtypes = [C.c_void_p]
        lib.kf_ctx_set_fallback_threshold.argtypes = [C.c_void_p, C.c_float]
        lib.kf_ctx_set_launch_events.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        lib.kf_ctx_set_find_config.argtypes = [C.c_void_p, C.POINTER(FindConfig)]
        lib.kf_ctx_get_find_config.argtypes = [C.c_void_p, C.POINTER(FindConfig)]
        lib.kf_workspace_size.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.POINTER(C.c_size_t)]
        lib.kf_fit.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FitIn), C.POINTER(FitOut),
                               C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_find.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FindIn), C.POINTER(FindOut),
                                C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_find_autotune.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FindIn),
                                         C.POINTER(FindOut), C.c_void_p, C.c_size_t, C.c_void_p,
                                         C.POINTER(FindConfig)]
        lib.kf_ctx_set_dedup_cuts.argtypes = [C.c_void_p, C.POINTER(DedupCuts)]
        lib.kf_ctx_get_dedup_cuts.argtypes = [C.c_void_p, C.POINTER(DedupCuts)]
        lib.kf_clean_seeds.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FindIn), C.c_void_p,
                                       C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_remove_duplicates.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(TracksIn), C.c_void_p,
                                             C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_smooth.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FitIn), C.POINTER(FitOut),
                                  C.POINTER(SmoothOut), C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_fit_backward.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FitIn), C.POINTER(FitOut),
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        lib.kf_fit_backward_static.argtypes = [C.c_void_p, C.POINTER(LayerParams), C.POINTER(FitIn),
                                               C.POINTER(FitOut), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        lib.kf_static_scratch_bytes.restype = C.c_size_t
        lib.kf_static_scratch_bytes.argtypes = []
        _LIB = lib
    return _LIB


def _check(code, what):
    if code != 0:
        raise KfError(code, what)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev(t, dtype, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class SmoothOut(C.Structure):
    _fields_ = [("state", C.c_void_p), ("cov", C.c_void_p), ("first", C.c_void_p), ("last", C.c_void_p)]


class FindConfig(C.Structure):
    _fields_ = [("wide_window_bins", C.c_int32), ("blocks_per_cu", C.c_int32), ("use_graph", C.c_int32),
                ("n_phi_bins", C.c_int32), ("n_z_bins", C.c_int32), ("lanes_per_seed", C.c_int32)]


FIND_CONFIG_KEYS = ("wide_window_bins", "blocks_per_cu", "use_graph", "n_phi_bins", "n_z_bins", "lanes_per_seed")


class Context:
    """A kf_ctx for one detector geometry (anything with the attributes of
    synth.Geometry, or keyword arguments; disk_z, disk_rmin, disk_rmax and cyl_zmax
    describe endcap disks and bounded cylinders, all zero when absent)."""

    def __init__(self, geom=None, **kw):
        g = Geometry()
        src = dict(kw)
        if geom is not None:
            for k in ("radius", "zhalf", "B", "sigma_rphi", "sigma_z", "sigma_r", "mass", "n_phi_bins",
                      "n_z_bins"):
                src.setdefault(k, getattr(geom, k))
            for k in ("disk_z", "disk_rmin", "disk_rmax", "cyl_zmax"):
                if getattr(geom, k, None) is not None:
                    src.setdefault(k, getattr(geom, k))
        radius = [float(v) for v in src["radius"]]
        zhalf = [float(v) for v in src["zhalf"]]
        g.n_layers = len(radius)
        g.B_tesla = float(src["B"])
        for i, (r, z) in enumerate(zip(radius, zhalf)):
            g.radius_cm[i] = r
            g.zhalf_cm[i] = z
        g.sigma_rphi_cm = float(src.get("sigma_rphi", 0.01))
        g.sigma_z_cm = float(src.get("sigma_z", 0.1))
        g.sigma_r_cm = float(src.get("sigma_r", 0.001))
        g.mass_gev = float(src.get("mass", 0.13957039))
        g.n_phi_bins = int(src.get("n_phi_bins", 128))
        g.n_z_bins = int(src.get("n_z_bins", 32))
        for k in ("disk_z", "disk_rmin", "disk_rmax", "cyl_zmax"):
            for i, v in enumerate(src.get(k, ())):
                getattr(g, k + "_cm")[i] = float(v)
        self.geometry = g
        self.n_layers = g.n_layers
        h = C.c_void_p()
        _check(_lib().kf_ctx_create(C.byref(g), C.byref(h)), "kf_ctx_create")
        self._h = h
        self._ws = None
        self._material = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.kf_ctx_destroy(h)
            self._h = None

    def set_fallback_threshold(self, det_threshold: float):
        _check(_lib().kf_ctx_set_fallback_threshold(self._h, float(det_threshold)),
               "kf_ctx_set_fallback_threshold")

    def set_launch_events(self, start=None, stop=None):
        """kf_ctx_set_launch_events: hipEvent_t handles (ints or ctypes pointers) that the
        main kernel of each kf_fit / kf_smooth call records around its own execution;
        None, None turns the hook off."""
        _check(_lib().kf_ctx_set_launch_events(self._h, start, stop), "kf_ctx_set_launch_events")

    def set_material(self, xX0_map=None, eloss=0.0):
        """kf_ctx_set_material: xX0_map [L][nz] float32 CUDA tensor (x/X0 at the z-bin
        centres of each layer; None keeps the per-layer xX0) and the mean ionisation
        loss per radiation length in GeV (0: none).  The context keeps a reference to
        the map while it is set."""
        if xX0_map is None:
            _check(_lib().kf_ctx_set_material(self._h, None, 0, C.c_float(float(eloss))), "kf_ctx_set_material")
            self._material = None
            return
        _dev(xX0_map, torch.float32, None, "xX0_map")
        if xX0_map.dim() != 2 or xX0_map.shape[0] != self.n_layers:
            raise ValueError(f"xX0_map must be [{self.n_layers}][nz], got {tuple(xX0_map.shape)}")
        _check(_lib().kf_ctx_set_material(self._h, C.c_void_p(xX0_map.data_ptr()), int(xX0_map.shape[1]),
                                          C.c_float(float(eloss))), "kf_ctx_set_material")
        self._material = xX0_map

    def set_field(self, c_r=0.0, c_z=0.0):
        """kf_ctx_set_field: B_z(r, z) = B (1 + c_r r^2 + c_z z^2) (cm^-2); 0, 0 is the
        uniform field."""
        _check(_lib().kf_ctx_set_field(self._h, C.c_float(float(c_r)), C.c_float(float(c_z))), "kf_ctx_set_field")

    def set_find_config(self, **kw):
        """kf_ctx_set_find_config; keys of FIND_CONFIG_KEYS (wide_window_bins,
        blocks_per_cu, use_graph, n_phi_bins, n_z_bins, lanes_per_seed), others keep their value."""
        cfg = self.find_config()
        for k, v in kw.items():
            if k not in FIND_CONFIG_KEYS:
                raise TypeError(f"unknown find configuration field {k}")
            if v is not None:
                cfg[k] = int(v)
        c = FindConfig(*[cfg[k] for k in FIND_CONFIG_KEYS])
        _check(_lib().kf_ctx_set_find_config(self._h, C.byref(c)), "kf_ctx_set_find_config")

    def find_config(self):
        c = FindConfig()
        _check(_lib().kf_ctx_get_find_config(self._h, C.byref(c)), "kf_ctx_get_find_config")
        return {k: int(getattr(c, k)) for k in FIND_CONFIG_KEYS}

    def workspace(self, op, inp, device):
        nb = C.c_size_t(0)
        _check(_lib().kf_workspace_size(self._h, op, C.byref(inp), C.byref(nb)), "kf_workspace_size")
        need = max(int(nb.value), 256)
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    @staticmethod
    def _params(align, xX0):
        p = LayerParams()
        p.align = None if align is None else align.data_ptr()
        p.xX0 = None if xX0 is None else xX0.data_ptr()
        return p

    def fit(self, hits, hit_mask, align=None, xX0=None, seed_state=None, seed_cov=None, ckpt=False,
            out=None, stream=None, ckpt_every=1):
        """kf_fit.  hits [L][3][n] float32, hit_mask [n] int32/uint32 bits; seeds from
        hits 0-2 unless seed_state [6][n] / seed_cov [21][n] are given.  Returns a dict
        with state, cov, chi2, ndf, status (and, with ckpt, ckpt [ceil(L / k)][27][n]
        holding layers 0, k, 2k, ... for k = ckpt_every, and ckpt_every)."""
        L = self.n_layers
        n = hits.shape[2]
        dev = hits.device
        _dev(hits, torch.float32, (L, 3, n), "hits")
        if hit_mask.dtype not in (torch.int32, torch.uint32):
            raise TypeError("hit_mask must be int32 or uint32")
        _dev(hit_mask, hit_mask.dtype, (n,), "hit_mask")
        _dev(align, torch.float32, (L, 4), "align")
        _dev(xX0, torch.float32, (L,), "xX0")
        from_hits = seed_state is None
        if not from_hits:
            _dev(seed_state, torch.float32, (6, n), "seed_state")
            _dev(seed_cov, torch.float32, (21, n), "seed_cov")
        if out is None:
            out = dict(state=torch.empty((6, n), dtype=torch.float32, device=dev),
                       cov=torch.empty((21, n), dtype=torch.float32, device=dev),
                       chi2=torch.empty(n, dtype=torch.float32, device=dev),
                       ndf=torch.empty(n, dtype=torch.int32, device=dev),
                       status=torch.empty(n, dtype=torch.int32, device=dev))
            if ckpt:
                k = max(1, int(ckpt_every))
                out["ckpt"] = torch.empty(((L + k - 1) // k, 27, n), dtype=torch.float32, device=dev)
        if out.get("ckpt") is not None:
            out["ckpt_every"] = max(1, int(ckpt_every))
        fin = FitIn(n, hits.data_ptr(), hit_mask.data_ptr(), None if from_hits else seed_state.data_ptr(),
                    None if from_hits else seed_cov.data_ptr(), int(from_hits), int(ckpt_every))
        fo = FitOut(out["state"].data_ptr(), out["cov"].data_ptr(), out["chi2"].data_ptr(),
                    out["ndf"].data_ptr(), out["status"].data_ptr(),
                    out["ckpt"].data_ptr() if out.get("ckpt") is not None else None)
        ws = self.workspace(KF_OP_FIT, fin, dev)
        p = self._params(align, xX0)
        _check(_lib().kf_fit(self._h, C.byref(p), C.byref(fin), C.byref(fo), C.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream(stream)), "kf_fit")
        return out

    def find(self, hits, hit_off, seed_hits, seed_event, align=None, xX0=None, chi2_cut=30.0, nsigma=3.0,
             keep=6, max_miss=3, refit=False, out=None, stream=None, autotune=False):
        """kf_find.  hits [3][H] float32, hit_off [E][L+1] int64, seed_hits [3][S] int32,
        seed_event [S] int32.  Returns a dict of the kf_find_out arrays.  With
        autotune=True the call is kf_find_autotune (synchronising; the chosen
        configuration stays in the context and is in find_config())."""
        L = self.n_layers
        dev = hits.device
        H = hits.shape[1]
        E = hit_off.shape[0]
        S = seed_hits.shape[1]
        _dev(hits, torch.float32, (3, H), "hits")
        _dev(hit_off, torch.int64, (E, L + 1), "hit_off")
        _dev(seed_hits, torch.int32, (3, S), "seed_hits")
        _dev(seed_event, torch.int32, (S,), "seed_event")
        _dev(align, torch.float32, (L, 4), "align")
        _dev(xX0, torch.float32, (L,), "xX0")
        if out is None:
            f32 = dict(dtype=torch.float32, device=dev)
            i32 = dict(dtype=torch.int32, device=dev)
            out = dict(n_cand=torch.empty(S, **i32), hit_idx=torch.empty((keep, L, S), **i32),
                       n_hits=torch.empty((keep, S), **i32), n_miss=torch.empty((keep, S), **i32),
                       chi2=torch.empty((keep, S), **f32), state=torch.empty((keep, 6, S), **f32),
                       cov=torch.empty((keep, 21, S), **f32), status=torch.empty((keep, S), **i32))
            if refit:
                out.update(rf_state=torch.empty((6, S), **f32), rf_cov=torch.empty((21, S), **f32),
                           rf_chi2=torch.empty(S, **f32), rf_ndf=torch.empty(S, **i32),
                           rf_status=torch.empty(S, **i32))
        fin = FindIn(E, hit_off.data_ptr(), H, hits.data_ptr(), S, seed_event.data_ptr(), seed_hits.data_ptr(),
                     float(chi2_cut), float(nsigma), int(keep), int(max_miss), int(bool(refit)))
        g = out.get
        fo = FindOut(*[None if g(k) is None else g(k).data_ptr() for k in
                       ("n_cand", "hit_idx", "n_hits", "n_miss", "chi2", "state", "cov", "status",
                        "rf_state", "rf_cov", "rf_chi2", "rf_ndf", "rf_status")])
        ws = self.workspace(KF_OP_FIND, fin, dev)
        p = self._params(align, xX0)
        if autotune:
            _check(_lib().kf_find_autotune(self._h, C.byref(p), C.byref(fin), C.byref(fo), C.c_void_p(ws.data_ptr()),
                                           ws.numel(), _stream(stream), None), "kf_find_autotune")
        else:
            _check(_lib().kf_find(self._h, C.byref(p), C.byref(fin), C.byref(fo), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream(stream)), "kf_find")
        return out

    def dedup_cuts(self):
        """kf_ctx_get_dedup_cuts as a dict."""
        c = DedupCuts()
        _check(_lib().kf_ctx_get_dedup_cuts(self._h, C.byref(c)), "kf_ctx_get_dedup_cuts")
        return {f: getattr(c, f) for f, _ in DedupCuts._fields_}

    def set_dedup_cuts(self, **kw):
        """kf_ctx_set_dedup_cuts; fields not given keep their current value."""
        cur = self.dedup_cuts()
        unknown = set(kw) - set(cur)
        if unknown:
            raise TypeError(f"unknown cut(s) {sorted(unknown)}")
        cur.update(kw)
        _check(_lib().kf_ctx_set_dedup_cuts(self._h, C.byref(DedupCuts(**cur))), "kf_ctx_set_dedup_cuts")

    def clean_seeds(self, hits, hit_off, seed_hits, seed_event, align=None, xX0=None, out=None, stream=None):
        """kf_clean_seeds: keep [S] int32 (1 kept, 0 the duplicate of a lower-index seed)."""
        L = self.n_layers
        dev = seed_hits.device
        H = hits.shape[1]
        E = hit_off.shape[0]
        S = seed_hits.shape[1]
        _dev(hits, torch.float32, (3, H), "hits")
        _dev(hit_off, torch.int64, (E, L + 1), "hit_off")
        _dev(seed_hits, torch.int32, (3, S), "seed_hits")
        _dev(seed_event, torch.int32, (S,), "seed_event")
        _dev(align, torch.float32, (L, 4), "align")
        _dev(xX0, torch.float32, (L,), "xX0")
        if out is None:
            out = torch.empty(S, dtype=torch.int32, device=dev)
        _dev(out, torch.int32, (S,), "out")
        fin = FindIn(E, hit_off.data_ptr(), H, hits.data_ptr(), S, seed_event.data_ptr(), seed_hits.data_ptr(),
                     0.0, 0.0, 1, 1, 0)
        ws = self.workspace(KF_OP_CLEAN_SEEDS, fin, dev)
        p = self._params(align, xX0)
        _check(_lib().kf_clean_seeds(self._h, C.byref(p), C.byref(fin), C.c_void_p(out.data_ptr()),
                                     C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "kf_clean_seeds")
        return out

    def remove_duplicates(self, hits, n_events, event, hit_idx, n_hits, chi2, state, align=None, xX0=None,
                          out=None, stream=None):
        """kf_remove_duplicates over built tracks: event [n] int32, hit_idx [L][n] int32,
        n_hits [n] int32, chi2 [n] float32, state [6][n] float32 (kappa, theta compared).
        Returns keep [n] int32."""
        L = self.n_layers
        dev = event.device
        H = hits.shape[1]
        n = event.shape[0]
        _dev(hits, torch.float32, (3, H), "hits")
        _dev(event, torch.int32, (n,), "event")
        _dev(hit_idx, torch.int32, (L, n), "hit_idx")
        _dev(n_hits, torch.int32, (n,), "n_hits")
        _dev(chi2, torch.float32, (n,), "chi2")
        _dev(state, torch.float32, (6, n), "state")
        _dev(align, torch.float32, (L, 4), "align")
        _dev(xX0, torch.float32, (L,), "xX0")
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=dev)
        _dev(out, torch.int32, (n,), "out")
        tin = TracksIn(int(n_events), H, hits.data_ptr(), n, event.data_ptr(), hit_idx.data_ptr(),
                       n_hits.data_ptr(), chi2.data_ptr(), state.data_ptr())
        ws = self.workspace(KF_OP_REMOVE_DUPLICATES, tin, dev)
        p = self._params(align, xX0)
        _check(_lib().kf_remove_duplicates(self._h, C.byref(p), C.byref(tin), C.c_void_p(out.data_ptr()),
                                           C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)),
               "kf_remove_duplicates")
        return out

    def smooth(self, hits, hit_mask, fwd, align=None, xX0=None, out=None, stream=None):
        """kf_smooth: smoothed state [L][6][n] and cov [L][21][n] of every layer of a
        fitted batch (fwd from fit(..., ckpt=True) with the same align/xX0), and the
        per-track first/last smoothed layers."""
        L = self.n_layers
        n = hits.shape[2]
        dev = hits.device
        if fwd.get("ckpt") is None:
            raise ValueError("the forward fit must be run with ckpt=True")
        _dev(align, torch.float32, (L, 4), "align")
        _dev(xX0, torch.float32, (L,), "xX0")
        if out is None:
            out = dict(state=torch.empty((L, 6, n), dtype=torch.float32, device=dev),
                       cov=torch.empty((L, 21, n), dtype=torch.float32, device=dev),
                       first=torch.empty(n, dtype=torch.int32, device=dev),
                       last=torch.empty(n, dtype=torch.int32, device=dev))
        fin = FitIn(n, hits.data_ptr(), hit_mask.data_ptr(), None, None, 1, int(fwd.get("ckpt_every", 1)))
        fo = FitOut(fwd["state"].data_ptr(), fwd["cov"].data_ptr(), fwd["chi2"].data_ptr(),
                    fwd["ndf"].data_ptr(), fwd["status"].data_ptr(), fwd["ckpt"].data_ptr())
        so = SmoothOut(out["state"].data_ptr(), out["cov"].data_ptr(), out["first"].data_ptr(),
                       out["last"].data_ptr())
        ws = self.workspace(KF_OP_SMOOTH, fin, dev)
        p = self._params(align, xX0)
        _check(_lib().kf_smooth(self._h, C.byref(p), C.byref(fin), C.byref(fo), C.byref(so),
                                C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "kf_smooth")
        return out

    def fit_backward(self, hits, hit_mask, fwd, dchi2, align=None, xX0=None, stream=None):
        """kf_fit_backward: dLoss/dalign [L][4] and dLoss/dxX0 [L] given dLoss/dchi2 [n]
        and the forward outputs (with checkpoints) of a seed-from-hits fit."""
        L = self.n_layers
        n = hits.shape[2]
        dev = hits.device
        _dev(hits, torch.float32, (L, 3, n), "hits")
        _dev(dchi2, torch.float32, (n,), "dchi2")
        if fwd.get("ckpt") is None:
            raise ValueError("the forward fit must be run with ckpt=True")
        fin = FitIn(n, hits.data_ptr(), hit_mask.data_ptr(), None, None, 1, int(fwd.get("ckpt_every", 1)))
        fo = FitOut(fwd["state"].data_ptr(), fwd["cov"].data_ptr(), fwd["chi2"].data_ptr(),
                    fwd["ndf"].data_ptr(), fwd["status"].data_ptr(), fwd["ckpt"].data_ptr())
        da = torch.empty((L, 4), dtype=torch.float32, device=dev)
        dx = torch.empty(L, dtype=torch.float32, device=dev)
        ws = self.workspace(KF_OP_FIT_BACKWARD, fin, dev)
        p = self._params(align, xX0)
        _check(_lib().kf_fit_backward(self._h, C.byref(p), C.byref(fin), C.byref(fo), C.c_void_p(dchi2.data_ptr()),
                                      C.c_void_p(da.data_ptr()), C.c_void_p(dx.data_ptr()),
                                      C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)), "kf_fit_backward")
        return da, dx

    def fit_backward_static(self, hits, hit_mask, fwd, dchi2, align=None, xX0=None, out=None, stream=None):
        """kf_fit_backward_static: as fit_backward, with the library's static per-GPU
        scratch instead of a workspace.  out = (dalign [L][4], dxX0 [L]) float32 device
        tensors to write (allocated here if None; pass them to allocate nothing)."""
        L = self.n_layers
        n = hits.shape[2]
        dev = hits.device
        _dev(hits, torch.float32, (L, 3, n), "hits")
        _dev(dchi2, torch.float32, (n,), "dchi2")
        if fwd.get("ckpt") is None:
            raise ValueError("the forward fit must be run with ckpt=True")
        if out is None:
            out = (torch.empty((L, 4), dtype=torch.float32, device=dev), torch.empty(L, dtype=torch.float32, device=dev))
        da, dx = out
        _dev(da, torch.float32, (L, 4), "dalign")
        _dev(dx, torch.float32, (L,), "dxX0")
        fin = FitIn(n, hits.data_ptr(), hit_mask.data_ptr(), None, None, 1, int(fwd.get("ckpt_every", 1)))
        fo = FitOut(fwd["state"].data_ptr(), fwd["cov"].data_ptr(), fwd["chi2"].data_ptr(),
                    fwd["ndf"].data_ptr(), fwd["status"].data_ptr(), fwd["ckpt"].data_ptr())
        p = self._params(align, xX0)
        _check(_lib().kf_fit_backward_static(self._h, C.byref(p), C.byref(fin), C.byref(fo),
                                             C.c_void_p(dchi2.data_ptr()), C.c_void_p(da.data_ptr()),
                                             C.c_void_p(dx.data_ptr()), _stream(stream)), "kf_fit_backward_static")
        return da, dx


def static_scratch_bytes() -> int:
    """Per-GPU bytes of the scratch behind Context.fit_backward_static."""
    return int(_lib().kf_static_scratch_bytes())


def exported_symbols():
    """Names the header declares (for the load check)."""
    return ["kf_ctx_create", "kf_ctx_destroy", "kf_ctx_set_fallback_threshold", "kf_ctx_set_launch_events",
            "kf_ctx_set_material", "kf_ctx_set_field", "kf_ctx_set_find_config",
            "kf_ctx_get_find_config", "kf_workspace_size", "kf_fit", "kf_find", "kf_find_autotune",
            "kf_smooth", "kf_fit_backward", "kf_ctx_set_dedup_cuts", "kf_ctx_get_dedup_cuts", "kf_clean_seeds",
            "kf_remove_duplicates", "kf_strerror", "kf_fit_backward_static", "kf_static_scratch_bytes"]
