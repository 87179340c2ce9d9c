// C ABI of the library: argument validation, workspace layout and launches.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/kf.h"
#include "kf_internal.h"

struct kf_ctx {
  struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;
  };
  kf_geometry g;
  float det_thr;
  kf_find_config fcfg{16, 0, 0, 0, 0, 0};
  hipStream_t cap_stream = nullptr;  // capture stream of the graph path
  int cap_device = -1;
  uint64_t tick = 0;
  GraphEntry graphs[4];              // least recently used is replaced
  ~kf_ctx() {
    for (auto& g : graphs)
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  int grid_device = -1;   // device the occupancy figures below were taken on
  int grid_cus = 0;       // compute units
  int grid_per_cu[3][3] = {};  // find workgroups that fit on one compute unit ([variant][4, 6, 8 lanes])
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;  // timing hook (kf_ctx_set_launch_events)
  kf_dedup_cuts dcuts{0.05f, 2, 1, 0.1f, 0.15f, 0.03f, 0.02f, 0.5f, 0.5f, 0.1f, 0.01f, 0.02f};
  const float* mat_map = nullptr;  // material model (kf_ctx_set_material)
  int32_t mat_nz = 0;
  float eloss = 0.f;
  float fr = 0.f, fz = 0.f;        // parameterised field (kf_ctx_set_field)
  // the detector model beyond one x/X0 per layer and a uniform field: the fit only
  bool material() const { return mat_map != nullptr || eloss > 0.f || fr != 0.f || fz != 0.f; }
  bool bounded = false;            // the geometry has a disk or a bounded cylinder
  // the kernel variant of kf_find and the refit (kfi::Variant)
  int variant() const { return material() ? kfi::kModelV : (bounded ? kfi::kBoundedV : kfi::kPlain); }
  kfi::Surfaces surfaces() const {
    kfi::Surfaces s = {};
    for (int l = 0; l < g.n_layers; ++l) {
      s.disk_z[l] = g.disk_z_cm[l];
      s.rmin[l] = g.disk_rmin_cm[l];
      s.rmax[l] = g.disk_rmax_cm[l];
      s.zmax[l] = g.cyl_zmax_cm[l];
    }
    return s;
  }
};

namespace {

constexpr size_t kAlign = 256;

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

kfd::Model model_of(const kf_ctx* c) {
  kfd::Model m;
  m.kB = 0.299792458e-2f * c->g.B_tesla;
  m.v_r = c->g.sigma_r_cm * c->g.sigma_r_cm;
  m.v_rphi = c->g.sigma_rphi_cm * c->g.sigma_rphi_cm;
  m.v_z = c->g.sigma_z_cm * c->g.sigma_z_cm;
  m.mass2 = c->g.mass_gev * c->g.mass_gev;
  m.det_thr = c->det_thr;
  m.dr02 = c->g.radius_cm[2] - c->g.radius_cm[0];
  return m;
}

bool valid_geometry(const kf_geometry* g) {
  if (!g) return false;
  if (g->n_layers < 3 || g->n_layers > KF_MAX_LAYERS) return false;
  float last_r = 0.f;  // radius of the previous cylinder
  for (int l = 0; l < g->n_layers; ++l) {
    if (!(g->radius_cm[l] > 0.f) || !(g->zhalf_cm[l] > 0.f) || !isfinite(g->radius_cm[l]) ||
        !isfinite(g->zhalf_cm[l]))
      return false;
    const float zd = g->disk_z_cm[l], r0 = g->disk_rmin_cm[l], r1 = g->disk_rmax_cm[l], zm = g->cyl_zmax_cm[l];
    if (!isfinite(zd) || !isfinite(r0) || !isfinite(r1) || !(zm >= 0.f) || !isfinite(zm)) return false;
    if (zd != 0.f) {  // a disk: after the seed layers, 0 <= rmin < rmax, no z bound
      if (l < 3 || !(r0 >= 0.f) || !(r1 > r0) || zm != 0.f) return false;
    } else {          // a cylinder: no radii of a disk, radius above the previous cylinder's
      if (r0 != 0.f || r1 != 0.f || !(g->radius_cm[l] > last_r)) return false;
      last_r = g->radius_cm[l];
    }
  }
  if (!(g->sigma_rphi_cm > 0.f) || !(g->sigma_z_cm > 0.f) || !(g->sigma_r_cm > 0.f)) return false;
  if (!(g->mass_gev >= 0.f) || !isfinite(g->B_tesla)) return false;
  if (g->n_phi_bins < 1 || g->n_phi_bins > 1024 || g->n_z_bins < 1 || g->n_z_bins > 256) return false;
  return true;
}

// Workspace of a fit: the per-layer constants.
size_t fit_ws_bytes() { return round_up(sizeof(kfd::LayerK) * KF_MAX_LAYERS); }

// Checkpoint stride of a fit input (ckpt_every 0 and 1: every layer).
int ckpt_stride(const kf_fit_in* in) { return in->ckpt_every > 1 ? in->ckpt_every : 1; }

// Workspace of the adjoint: the layer table, then [L][5][blocks] FP64 partials, then
// with checkpoints every k > 1 layers the recomputed segment [k-1][27][n].
size_t backward_partials_bytes(const kf_ctx* ctx, int64_t n) {
  return round_up((size_t)ctx->g.n_layers * 5 * (size_t)kfi::adjoint_blocks(n > 0 ? n : 0) * sizeof(double));
}
size_t backward_ws_bytes(const kf_ctx* ctx, int64_t n, int every) {
  const size_t nn = (size_t)(n > 0 ? n : 0);
  return fit_ws_bytes() + backward_partials_bytes(ctx, n) + (every > 1 ? round_up((size_t)(every - 1) * 27 * nn * 4) : 0);
}

// Workspace of a find: layer constants | binned records [H] float4 | binned indices [H]
// | bin offsets [E][L][nbins + 1] | tile counter | backpointers of the persistent
// workgroups' current tiles.
struct FindWs {
  size_t layers, brec, hpos, bidx, boff, counter, bp, bpos, rpos, rmask, total;
};

int64_t find_tiles(const kf_find_in* in, int lanes_per_seed) {
  const int64_t t = kfi::find_tile_seeds(lanes_per_seed);
  return in->n_seeds > 0 ? (in->n_seeds + t - 1) / t : 0;
}

// Persistent find workgroups at most: as many as tiles of the largest grouping (8 lanes
// per seed, the fewest seeds per tile), and kMaxFindGrid.
int64_t find_grid_cap(const kf_find_in* in) {
  const int64_t t = find_tiles(in, 8);
  return t < kfi::kMaxFindGrid ? t : kfi::kMaxFindGrid;
}

// Lanes per seed of a find call: the configuration's, else the fewest of 4, 6, 8 that
// hold `keep` candidates; 0 if the configuration's is below keep.
int find_group(const kf_ctx* c, int keep) {
  if (c->fcfg.lanes_per_seed > 0) return c->fcfg.lanes_per_seed >= keep ? c->fcfg.lanes_per_seed : 0;
  return keep <= 4 ? 4 : (keep <= 6 ? 6 : 8);
}

int group_index(int lanes_per_seed) { return lanes_per_seed == 4 ? 0 : (lanes_per_seed == 6 ? 1 : 2); }

// The bin tiling kf_find walks: the configuration's, else the geometry's.
void find_bins(const kf_ctx* c, int* nphi, int* nz) {
  *nphi = c->fcfg.n_phi_bins > 0 ? c->fcfg.n_phi_bins : c->g.n_phi_bins;
  *nz = c->fcfg.n_z_bins > 0 ? c->fcfg.n_z_bins : c->g.n_z_bins;
}

FindWs find_ws(const kf_ctx* c, const kf_find_in* in) {
  FindWs w;
  const size_t H = (size_t)(in->n_hits > 0 ? in->n_hits : 0);
  // bin offsets for the largest tiling, so that one workspace serves every configuration
  const size_t nb = (size_t)KF_MAX_FIND_BINS + 1;
  const size_t E = (size_t)(in->n_events > 0 ? in->n_events : 0);
  w.layers = 0;
  w.brec = w.layers + fit_ws_bytes();
  w.hpos = w.brec + round_up(H * 16);
  w.bidx = w.hpos + round_up(H * 16);
  w.boff = w.bidx + round_up(H * 4);
  w.counter = w.boff + round_up(E * c->g.n_layers * nb * 4);
  w.bp = w.counter + kAlign;
  // with a refit: placed hits of the workgroups' tiles, of every seed's rank-0
  // candidate, and that candidate's layers
  const size_t S = (size_t)(in->n_seeds > 0 ? in->n_seeds : 0);
  const size_t L = (size_t)c->g.n_layers;
  const size_t grid = (size_t)find_grid_cap(in);
  w.bpos = w.bp + round_up(kfi::find_bp_bytes(c->g.n_layers, find_grid_cap(in)));
  w.rpos = w.bpos + (in->refit ? round_up(grid * L * 3 * 64 * sizeof(float)) : 0);
  w.rmask = w.rpos + (in->refit ? round_up(L * 3 * S * sizeof(float)) : 0);
  w.total = w.rmask + (in->refit ? round_up(S * sizeof(uint32_t)) : 0);
  return w;
}

// Persistent find grid: blocks_per_cu workgroups per compute unit, at most as many as
// fit at once.
// Workspace of duplicate handling: layer constants | par, spar [5][n] | sint [3][n] |
// skey, bin [n] | cnt, cur [E * nb] | off [E * nb + 1] | order [n].
struct DedupWs {
  size_t layers, par, spar, sint, skey, bin, cnt, cur, off, order, total;
  int64_t m;  // E * nb
};

DedupWs dedup_ws(const kf_ctx* c, int64_t n_items, int32_t n_events) {
  DedupWs w;
  const size_t n = (size_t)(n_items > 0 ? n_items : 0);
  const int64_t E = n_events > 0 ? n_events : 0;
  w.m = E * kfi::dedup_bins(c->dcuts.psi_window);
  w.layers = 0;
  w.par = w.layers + fit_ws_bytes();
  w.spar = w.par + round_up(5 * n * sizeof(float));
  w.sint = w.spar + round_up(5 * n * sizeof(float));
  w.skey = w.sint + round_up(3 * n * 4);
  w.bin = w.skey + round_up(n * 4);
  w.cnt = w.bin + round_up(n * 4);
  w.cur = w.cnt + round_up((size_t)w.m * 4);
  w.off = w.cur + round_up((size_t)w.m * 4);
  w.order = w.off + round_up(((size_t)w.m + 1) * 4);
  w.total = w.order + round_up(n * 4);
  return w;
}

int persistent_grid(kf_ctx* c, int nl, int lanes_per_seed, int* grid) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KF_E_HIP;
  if (c->grid_device != dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return KF_E_HIP;
    for (int m = 0; m < 3; ++m)
      for (int gi = 0; gi < 3; ++gi) {
        int per = 0;
        if (kfi::find_max_blocks(nl, m, gi == 0 ? 4 : (gi == 1 ? 6 : 8), &per) != hipSuccess) return KF_E_HIP;
        c->grid_per_cu[m][gi] = per > 0 ? per : 1;
      }
    if (kfi::prepare_bin(KF_MAX_FIND_BINS) != hipSuccess) return KF_E_HIP;
    c->grid_cus = cus;
    c->grid_device = dev;
  }
  const int have = c->grid_per_cu[c->variant()][group_index(lanes_per_seed)];
  const int want = c->fcfg.blocks_per_cu;
  *grid = c->grid_cus * (want > 0 && want < have ? want : have);
  return KF_OK;
}

int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return KF_OK;
  if (!ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) return KF_E_WORKSPACE;
  return KF_OK;
}

}  // namespace

extern "C" {

int kf_ctx_create(const kf_geometry* geom, kf_ctx** ctx) {
  if (!ctx) return KF_E_INVALID;
  *ctx = nullptr;
  if (!valid_geometry(geom)) return KF_E_INVALID;
  kf_ctx* c = new (std::nothrow) kf_ctx;
  if (!c) return KF_E_INVALID;
  c->g = *geom;
  c->det_thr = 1e-2f;
  for (int l = 0; l < geom->n_layers; ++l)
    if (geom->disk_z_cm[l] != 0.f || geom->cyl_zmax_cm[l] > 0.f) c->bounded = true;
  *ctx = c;
  return KF_OK;
}

int kf_ctx_destroy(kf_ctx* ctx) {
  delete ctx;
  return KF_OK;
}

int kf_ctx_set_fallback_threshold(kf_ctx* ctx, float det_threshold) {
  if (!ctx || !(det_threshold >= 0.f) || !isfinite(det_threshold)) return KF_E_INVALID;
  ctx->det_thr = det_threshold;
  return KF_OK;
}

int kf_ctx_set_launch_events(kf_ctx* ctx, void* start, void* stop) {
  if (!ctx || ((start == nullptr) != (stop == nullptr))) return KF_E_INVALID;
  ctx->ev_start = reinterpret_cast<hipEvent_t>(start);
  ctx->ev_stop = reinterpret_cast<hipEvent_t>(stop);
  return KF_OK;
}

int kf_ctx_set_material(kf_ctx* ctx, const float* xX0_map, int32_t nz, float eloss_gev_per_x0) {
  if (!ctx || !isfinite(eloss_gev_per_x0) || eloss_gev_per_x0 < 0.f) return KF_E_INVALID;
  if (ctx->bounded && (xX0_map || eloss_gev_per_x0 > 0.f)) return KF_E_UNSUPPORTED;
  if (xX0_map) {
    if (nz < 1 || nz > KF_MAX_MAP_BINS) return KF_E_INVALID;
    for (int l = 0; l < ctx->g.n_layers; ++l)
      if (!(ctx->g.zhalf_cm[l] > 0.f) || !isfinite(ctx->g.zhalf_cm[l])) return KF_E_INVALID;
  }
  ctx->mat_map = xX0_map;
  ctx->mat_nz = xX0_map ? nz : 0;
  ctx->eloss = eloss_gev_per_x0;
  return KF_OK;
}

int kf_ctx_set_field(kf_ctx* ctx, float c_r, float c_z) {
  if (!ctx || !isfinite(c_r) || !isfinite(c_z)) return KF_E_INVALID;
  if (!(ctx->g.B_tesla != 0.f) && (c_r != 0.f || c_z != 0.f)) return KF_E_UNSUPPORTED;
  if (ctx->bounded && (c_r != 0.f || c_z != 0.f)) return KF_E_UNSUPPORTED;
  ctx->fr = c_r;
  ctx->fz = c_z;
  return KF_OK;
}

int kf_ctx_set_find_config(kf_ctx* ctx, const kf_find_config* cfg) {
  if (!ctx || !cfg || cfg->wide_window_bins < 0 || cfg->blocks_per_cu < 0 || cfg->use_graph < 0 ||
      cfg->use_graph > 1 || cfg->n_phi_bins < 0 || cfg->n_phi_bins > 1024 || cfg->n_z_bins < 0 ||
      cfg->n_z_bins > 256 || !(cfg->lanes_per_seed == 0 || cfg->lanes_per_seed == 4 || cfg->lanes_per_seed == 6 ||
                               cfg->lanes_per_seed == 8))
    return KF_E_INVALID;
  const int nphi = cfg->n_phi_bins > 0 ? cfg->n_phi_bins : ctx->g.n_phi_bins;
  const int nz = cfg->n_z_bins > 0 ? cfg->n_z_bins : ctx->g.n_z_bins;
  if ((int64_t)nphi * nz > KF_MAX_FIND_BINS) return KF_E_INVALID;
  ctx->fcfg = *cfg;
  return KF_OK;
}

int kf_ctx_get_find_config(const kf_ctx* ctx, kf_find_config* cfg) {
  if (!ctx || !cfg) return KF_E_INVALID;
  *cfg = ctx->fcfg;
  return KF_OK;
}

int kf_ctx_set_dedup_cuts(kf_ctx* ctx, const kf_dedup_cuts* c) {
  if (!ctx || !c) return KF_E_INVALID;
  const float f[] = {c->seed_kap_rel, c->seed_kap_abs, c->seed_theta, c->seed_phi, c->seed_z,
                     c->trk_shared_frac, c->trk_kap_rel, c->trk_kap_abs, c->trk_theta};
  for (float v : f)
    if (!(v >= 0.f) || !isfinite(v)) return KF_E_INVALID;
  if (!(c->psi_window > 0.f) || !isfinite(c->psi_window) || c->min_shared < 0 || c->min_shared_kin < 0 ||
      c->min_shared_kin > c->min_shared)
    return KF_E_INVALID;
  ctx->dcuts = *c;
  return KF_OK;
}

int kf_ctx_get_dedup_cuts(const kf_ctx* ctx, kf_dedup_cuts* c) {
  if (!ctx || !c) return KF_E_INVALID;
  *c = ctx->dcuts;
  return KF_OK;
}

int kf_workspace_size(const kf_ctx* ctx, int op, const void* in, size_t* bytes) {
  if (!ctx || !in || !bytes) return KF_E_INVALID;
  switch (op) {
    case KF_OP_FIT:
      *bytes = 0;
      return KF_OK;
    case KF_OP_FIND:
      *bytes = find_ws(ctx, static_cast<const kf_find_in*>(in)).total;
      return KF_OK;
    case KF_OP_SMOOTH:
      *bytes = fit_ws_bytes();
      return KF_OK;
    case KF_OP_FIT_BACKWARD: {
      const kf_fit_in* f = static_cast<const kf_fit_in*>(in);
      *bytes = backward_ws_bytes(ctx, f->n, ckpt_stride(f));
      return KF_OK;
    }
    case KF_OP_CLEAN_SEEDS: {
      const kf_find_in* f = static_cast<const kf_find_in*>(in);
      *bytes = dedup_ws(ctx, f->n_seeds, f->n_events).total;
      return KF_OK;
    }
    case KF_OP_REMOVE_DUPLICATES: {
      const kf_tracks_in* t = static_cast<const kf_tracks_in*>(in);
      *bytes = dedup_ws(ctx, t->n, t->n_events).total;
      return KF_OK;
    }
    default:
      return KF_E_UNSUPPORTED;
  }
}

int kf_fit(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* out, void* ws,
           size_t ws_bytes, void* stream) {
  if (!ctx || !in || !out) return KF_E_INVALID;
  if (in->n < 0) return KF_E_INVALID;
  if (in->n == 0) return KF_OK;
  if (!in->hits || !in->hit_mask || !out->state || !out->cov || !out->chi2 || !out->ndf || !out->status)
    return KF_E_INVALID;
  if (!in->seed_from_hits && (!in->seed_state || !in->seed_cov)) return KF_E_INVALID;
  if (in->seed_from_hits && !(ctx->g.B_tesla != 0.f)) return KF_E_UNSUPPORTED;  // no curvature from hits at B = 0
  if (in->n > (int64_t)INT32_MAX * 256) return KF_E_INVALID;
  if (in->ckpt_every < 0 || in->ckpt_every > KF_MAX_LAYERS) return KF_E_INVALID;
  (void)ws;  // the fit needs no workspace
  (void)ws_bytes;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  kfi::FitArgs a;
  a.n = in->n;
  a.nl = ctx->g.n_layers;
  a.seed_from_hits = in->seed_from_hits ? 1 : 0;
  a.md = model_of(ctx);
  a.srphi = ctx->g.sigma_rphi_cm;
  a.sz = ctx->g.sigma_z_cm;
  a.hits = in->hits;
  a.mask = in->hit_mask;
  a.seed_state = in->seed_state;
  a.seed_cov = in->seed_cov;
  a.layers = nullptr;
  a.align = params ? params->align : nullptr;
  a.xX0 = params ? params->xX0 : nullptr;
  for (int l = 0; l < 32; ++l) a.radius[l] = l < ctx->g.n_layers ? ctx->g.radius_cm[l] : 0.f;
  a.mat_map = ctx->mat_map;
  a.mat_nz = ctx->mat_nz;
  a.eloss = ctx->eloss;
  a.fr = ctx->fr;
  a.fz = ctx->fz;
  for (int l = 0; l < 32; ++l) a.zhalf[l] = l < ctx->g.n_layers ? ctx->g.zhalf_cm[l] : 0.f;
  a.sf = ctx->surfaces();
  a.bounded = ctx->bounded ? 1 : 0;
  a.state = out->state;
  a.cov = out->cov;
  a.chi2 = out->chi2;
  a.ndf = out->ndf;
  a.status = out->status;
  a.ckpt = out->ckpt;
  a.ckpt_every = ckpt_stride(in);
  return kfi::launch_fit(a, st, ctx->ev_start, ctx->ev_stop) == hipSuccess ? KF_OK : KF_E_HIP;
}

}  // extern "C"

namespace {

int check_find(kf_ctx* ctx, const kf_find_in* in, const kf_find_out* out, void* ws, size_t ws_bytes) {
  if (!ctx || !in || !out) return KF_E_INVALID;
  if (in->n_events < 0 || in->n_seeds < 0 || in->n_hits < 0) return KF_E_INVALID;
  if (in->keep < 1 || in->keep > KF_MAX_KEEP || in->max_miss < 1) return KF_E_INVALID;
  if (find_group(ctx, in->keep) == 0) return KF_E_INVALID;  // configured lanes per seed below keep
  if (!(in->chi2_cut > 0.f) || !(in->nsigma > 0.f)) return KF_E_INVALID;
  if (in->n_seeds == 0) return KF_OK;
  if (in->n_events == 0 || !in->hit_off || !in->hits || !in->seed_event || !in->seed_hits) return KF_E_INVALID;
  if (!out->n_cand || !out->hit_idx || !out->n_hits || !out->n_miss || !out->chi2 || !out->state || !out->cov ||
      !out->status)
    return KF_E_INVALID;
  if (in->refit && (!out->rf_state || !out->rf_cov || !out->rf_chi2 || !out->rf_ndf || !out->rf_status))
    return KF_E_INVALID;
  // hit indices travel as (index + 2) << 3 in 32-bit backpointers
  if (in->n_hits >= (int64_t(1) << 28) - 2 || in->n_seeds >= (int64_t)INT32_MAX * 32) return KF_E_UNSUPPORTED;
  if (!(ctx->g.B_tesla != 0.f)) return KF_E_UNSUPPORTED;
  int nphi = 0, nz = 0;
  find_bins(ctx, &nphi, &nz);
  if ((int64_t)nphi * nz > KF_MAX_FIND_BINS) return KF_E_UNSUPPORTED;  // LDS of the bin kernel
  return check_ws(ws, ws_bytes, find_ws(ctx, in).total);
}

// The launches of one kf_find call (arguments already checked, n_seeds > 0); timed:
// the search kernel records the context's launch events (never inside a capture).
int enqueue_find(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out,
                 void* ws, hipStream_t st, bool timed) {
  const int group = find_group(ctx, in->keep);
  int grid = 0;  // (also readies the kernels' LDS limits before the first launch)
  if (persistent_grid(ctx, ctx->g.n_layers, group, &grid) != KF_OK) return KF_E_HIP;
  const FindWs w = find_ws(ctx, in);
  char* base = static_cast<char*>(ws);
  kfd::LayerK* layers = reinterpret_cast<kfd::LayerK*>(base + w.layers);
  const float* align = params ? params->align : nullptr;
  const float* xX0 = params ? params->xX0 : nullptr;
  kfi::BinArgs b;  // (the bin kernel also builds the layer table)
  b.nl = ctx->g.n_layers;
  find_bins(ctx, &b.nphi, &b.nz);
  b.n_events = in->n_events;
  b.H = in->n_hits;
  b.hit_off = in->hit_off;
  b.hits = in->hits;
  b.layers = layers;
  b.align = align;
  b.xX0 = xX0;
  b.mat_nz = ctx->mat_nz;
  b.sf = ctx->surfaces();
  for (int l = 0; l < 32; ++l) {
    b.radius[l] = l < ctx->g.n_layers ? ctx->g.radius_cm[l] : 0.f;
    b.zhalf[l] = l < ctx->g.n_layers ? ctx->g.zhalf_cm[l] : 1.f;
  }
  b.brec = reinterpret_cast<float4*>(base + w.brec);
  b.hpos = reinterpret_cast<float4*>(base + w.hpos);
  b.bidx = reinterpret_cast<int32_t*>(base + w.bidx);
  b.boff = reinterpret_cast<int32_t*>(base + w.boff);
  b.counter = reinterpret_cast<int32_t*>(base + w.counter);
  if (kfi::launch_bin(b, st) != hipSuccess) return KF_E_HIP;
  kfi::FindArgs f;
  f.nl = b.nl;
  f.nphi = b.nphi;
  f.nz = b.nz;
  f.keep = in->keep;
  f.max_miss = in->max_miss;
  f.n_events = in->n_events;
  f.wide_bins = ctx->fcfg.wide_window_bins;
  f.chi2_cut = in->chi2_cut;
  f.nsigma = in->nsigma;
  f.md = model_of(ctx);
  f.srphi = ctx->g.sigma_rphi_cm;
  f.sz = ctx->g.sigma_z_cm;
  f.n_seeds = in->n_seeds;
  f.H = in->n_hits;
  f.n_tiles = find_tiles(in, group);
  f.bp = reinterpret_cast<int32_t*>(base + w.bp);
  if (in->refit) {
    f.bpos = reinterpret_cast<float*>(base + w.bpos);
    f.rpos = reinterpret_cast<float*>(base + w.rpos);
    f.rmask = reinterpret_cast<uint32_t*>(base + w.rmask);
  }
  f.hits = in->hits;
  f.hit_off = in->hit_off;
  f.seed_event = in->seed_event;
  f.seed_hits = in->seed_hits;
  f.layers = layers;
  f.brec = b.brec;
  f.hpos = b.hpos;
  f.bidx = b.bidx;
  f.boff = b.boff;
  for (int l = 0; l < 32; ++l) f.zhalf[l] = b.zhalf[l];
  f.mat_map = ctx->mat_map;
  f.mat_nz = ctx->mat_nz;
  f.eloss = ctx->eloss;
  f.fr = ctx->fr;
  f.fz = ctx->fz;
  f.bounded = ctx->bounded ? 1 : 0;
  f.counter = b.counter;
  f.n_cand = out->n_cand;
  f.hit_idx = out->hit_idx;
  f.n_hits = out->n_hits;
  f.n_miss = out->n_miss;
  f.chi2 = out->chi2;
  f.state = out->state;
  f.cov = out->cov;
  f.status = out->status;
  if ((int64_t)grid > find_grid_cap(in)) grid = (int)find_grid_cap(in);
  if ((int64_t)grid > f.n_tiles) grid = (int)f.n_tiles;
  if (kfi::launch_find(f, group, grid, st, timed ? ctx->ev_start : nullptr, timed ? ctx->ev_stop : nullptr) !=
      hipSuccess)
    return KF_E_HIP;
  if (in->refit) {
    kfi::FitArgs a;
    a.n = in->n_seeds;
    a.nl = ctx->g.n_layers;
    a.seed_from_hits = 1;
    a.md = f.md;
    a.srphi = f.srphi;
    a.sz = f.sz;
    a.hits = nullptr;
    a.mask = nullptr;
    a.seed_state = nullptr;
    a.seed_cov = nullptr;
    a.layers = layers;
    a.state = out->rf_state;
    a.cov = out->rf_cov;
    a.chi2 = out->rf_chi2;
    a.ndf = out->rf_ndf;
    a.status = out->rf_status;
    a.ckpt = nullptr;
    a.mat_map = ctx->mat_map;
    a.mat_nz = ctx->mat_nz;
    a.eloss = ctx->eloss;
    a.fr = ctx->fr;
    a.fz = ctx->fz;
    a.bounded = ctx->bounded ? 1 : 0;  // (the surfaces are in the prepared layers)
    if (kfi::launch_refit(a, f.rpos, f.rmask, st) != hipSuccess) return KF_E_HIP;
  }
  return KF_OK;
}

// Everything a captured kf_find depends on, field by field (no struct padding).
std::vector<uint64_t> find_key(const kf_ctx* ctx, int dev, const kf_layer_params* params, const kf_find_in* in,
                               const kf_find_out* out, void* ws, size_t ws_bytes) {
  auto u = [](const void* p) { return (uint64_t)reinterpret_cast<uintptr_t>(p); };
  auto f = [](float v) {
    uint32_t b;
    memcpy(&b, &v, 4);
    return (uint64_t)b;
  };
  return {(uint64_t)dev,
          u(params ? params->align : nullptr),
          u(params ? params->xX0 : nullptr),
          (uint64_t)in->n_events,
          u(in->hit_off),
          (uint64_t)in->n_hits,
          u(in->hits),
          (uint64_t)in->n_seeds,
          u(in->seed_event),
          u(in->seed_hits),
          f(in->chi2_cut),
          f(in->nsigma),
          (uint64_t)in->keep,
          (uint64_t)in->max_miss,
          (uint64_t)(in->refit != 0),
          u(out->n_cand),
          u(out->hit_idx),
          u(out->n_hits),
          u(out->n_miss),
          u(out->chi2),
          u(out->state),
          u(out->cov),
          u(out->status),
          u(in->refit ? out->rf_state : nullptr),
          u(in->refit ? out->rf_cov : nullptr),
          u(in->refit ? out->rf_chi2 : nullptr),
          u(in->refit ? out->rf_ndf : nullptr),
          u(in->refit ? out->rf_status : nullptr),
          u(ws),
          (uint64_t)ws_bytes,
          u(ctx->mat_map),
          (uint64_t)ctx->mat_nz,
          f(ctx->eloss),
          f(ctx->fr),
          f(ctx->fz),
          (uint64_t)ctx->fcfg.wide_window_bins,
          (uint64_t)ctx->fcfg.blocks_per_cu,
          (uint64_t)ctx->fcfg.n_phi_bins,
          (uint64_t)ctx->fcfg.n_z_bins,
          (uint64_t)ctx->fcfg.lanes_per_seed,
          f(ctx->det_thr)};
}

// kf_find through a cached hipGraph: the call's launches are captured once on the
// context's own stream and the instantiated graph is replayed on the caller's stream
// for every later call with the same arguments.
int find_graph(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out, void* ws,
               size_t ws_bytes, hipStream_t st) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KF_E_HIP;
  const std::vector<uint64_t> key = find_key(ctx, dev, params, in, out, ws, ws_bytes);
  ++ctx->tick;
  kf_ctx::GraphEntry* hit = nullptr;
  for (auto& g : ctx->graphs)
    if (g.exec && g.key == key) hit = &g;
  if (!hit) {
    int grid = 0;  // sizes the grid (and sets the kernel's LDS limit) outside the capture
    if (persistent_grid(ctx, ctx->g.n_layers, find_group(ctx, in->keep), &grid) != KF_OK) return KF_E_HIP;
    if (ctx->cap_stream && ctx->cap_device != dev) {
      (void)hipStreamDestroy(ctx->cap_stream);
      ctx->cap_stream = nullptr;
    }
    if (!ctx->cap_stream) {
      if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        ctx->cap_stream = nullptr;
        return KF_E_HIP;
      }
      ctx->cap_device = dev;
    }
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return KF_E_HIP;
    const int rc = enqueue_find(ctx, params, in, out, ws, ctx->cap_stream, false);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (rc != KF_OK || ec != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != KF_OK ? rc : KF_E_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return KF_E_HIP;
    hit = &ctx->graphs[0];
    for (auto& g : ctx->graphs)
      if (!g.exec || g.used < hit->used) hit = &g;
    if (hit->exec) (void)hipGraphExecDestroy(hit->exec);
    hit->exec = exec;
    hit->key = key;
  }
  hit->used = ctx->tick;
  return hipGraphLaunch(hit->exec, st) == hipSuccess ? KF_OK : KF_E_HIP;
}

}  // namespace

extern "C" {

int kf_find(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out, void* ws,
            size_t ws_bytes, void* stream) {
  const int rc = check_find(ctx, in, out, ws, ws_bytes);
  if (rc != KF_OK || in->n_seeds == 0) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (ctx->fcfg.use_graph) return find_graph(ctx, params, in, out, ws, ws_bytes, st);
  return enqueue_find(ctx, params, in, out, ws, st, true);
}

}  // extern "C"

namespace {

// Argument checks of the adjoint (everything but the workspace).
int check_backward(const kf_ctx* ctx, const kf_fit_in* in, const kf_fit_out* fwd, const float* dchi2,
                   const float* dalign, const float* dxX0) {
  if (!ctx || !in || !fwd || !dalign || !dxX0) return KF_E_INVALID;
  if (in->n < 0 || in->ckpt_every < 0 || in->ckpt_every > KF_MAX_LAYERS) return KF_E_INVALID;
  if (!in->seed_from_hits) return KF_E_UNSUPPORTED;
  // the adjoint differentiates the material model (x/X0 per layer or the map, the energy
  // loss) and the field (with the points each step and the seed take it at)
  if (!(ctx->g.B_tesla != 0.f) || ctx->bounded) return KF_E_UNSUPPORTED;  // cylinders only
  if (in->n > 0 && (!in->hits || !in->hit_mask || !dchi2 || !fwd->ndf || !fwd->status || !fwd->ckpt))
    return KF_E_INVALID;
  return KF_OK;
}

// The adjoint's launches with its scratch at `base` (layer table, then the per-block
// FP64 partials; every byte is written before it is read, nothing needs clearing).
int enqueue_backward(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
                     const float* dchi2, float* dalign, float* dxX0, char* base, hipStream_t st) {
  kfd::LayerK* layers = reinterpret_cast<kfd::LayerK*>(base);
  const float* align = params ? params->align : nullptr;
  const float* xX0 = params ? params->xX0 : nullptr;
  if (kfi::launch_layer_prep(ctx->g.n_layers, ctx->g.radius_cm, align, xX0, layers, st, ctx->g.zhalf_cm,
                             ctx->mat_nz) != hipSuccess)
    return KF_E_HIP;
  const kfd::Model md = model_of(ctx);
  kfi::AdjArgs a;
  a.mat_map = ctx->mat_map;
  a.mat_nz = ctx->mat_nz;
  a.eloss = ctx->eloss;
  a.n = in->n;
  a.nl = ctx->g.n_layers;
  a.k.kB = md.kB;
  a.k.v_r = md.v_r;
  a.k.v_rphi = md.v_rphi;
  a.k.v_z = md.v_z;
  a.k.mass2 = md.mass2;
  a.k.det_thr = md.det_thr;
  a.srphi = ctx->g.sigma_rphi_cm;
  a.sz = ctx->g.sigma_z_cm;
  a.dr02 = md.dr02;
  a.fr = ctx->fr;
  a.fz = ctx->fz;
  a.hits = in->hits;
  a.mask = in->hit_mask;
  a.ndf = fwd->ndf;
  a.status = fwd->status;
  a.ckpt = fwd->ckpt;
  a.dchi2 = dchi2;
  a.layers = layers;
  a.n_blocks = kfi::adjoint_blocks(in->n);
  a.part = reinterpret_cast<double*>(base + fit_ws_bytes());
  a.every = ckpt_stride(in);
  a.seg = a.every > 1 ? reinterpret_cast<float*>(base + fit_ws_bytes() + backward_partials_bytes(ctx, in->n)) : nullptr;
  return kfi::launch_adjoint(a, dalign, dxX0, st) == hipSuccess ? KF_OK : KF_E_HIP;
}

// Scratch of kf_fit_backward_static: one copy per GPU in the code object's device
// memory, alive until the process ends.  Host code never passes `scratch` itself (its
// host-side name is not a device address): each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return KF_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KF_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KF_OK;
}

}  // namespace

extern "C" {

int kf_fit_backward(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
                    const float* dchi2, float* dalign, float* dxX0, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_backward(ctx, in, fwd, dchi2, dalign, dxX0);
  if (rc != KF_OK) return rc;
  rc = check_ws(ws, ws_bytes, backward_ws_bytes(ctx, in->n, ckpt_stride(in)));
  if (rc != KF_OK) return rc;
  return enqueue_backward(ctx, params, in, fwd, dchi2, dalign, dxX0, static_cast<char*>(ws),
                          reinterpret_cast<hipStream_t>(stream));
}

int kf_fit_backward_static(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
                           const float* dchi2, float* dalign, float* dxX0, void* stream) {
  int rc = check_backward(ctx, in, fwd, dchi2, dalign, dxX0);
  if (rc != KF_OK) return rc;
  if (backward_ws_bytes(ctx, in->n, ckpt_stride(in)) > kStaticScratchBytes) return KF_E_SCRATCH;
  void* base = nullptr;
  rc = static_scratch(&base);
  if (rc != KF_OK) return rc;
  return enqueue_backward(ctx, params, in, fwd, dchi2, dalign, dxX0, static_cast<char*>(base),
                          reinterpret_cast<hipStream_t>(stream));
}

size_t kf_static_scratch_bytes(void) { return kStaticScratchBytes; }

int kf_smooth(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
              const kf_smooth_out* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !in || !fwd || !out) return KF_E_INVALID;
  if (in->n < 0) return KF_E_INVALID;
  if (ctx->bounded) return KF_E_UNSUPPORTED;  // the smoother is for cylinders only
  if (in->ckpt_every > 1) return KF_E_UNSUPPORTED;  // it reads every layer's checkpoint
  if (in->n == 0) return KF_OK;
  if (!in->hit_mask || !fwd->ndf || !fwd->status || !fwd->ckpt || !out->state || !out->cov || !out->first ||
      !out->last)
    return KF_E_INVALID;
  if (in->n > ((int64_t)1 << 29)) return KF_E_INVALID;  // rows addressed by 32-bit byte offsets
  int rc = check_ws(ws, ws_bytes, fit_ws_bytes());
  if (rc != KF_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  kfd::LayerK* layers = reinterpret_cast<kfd::LayerK*>(ws);
  const float* align = params ? params->align : nullptr;
  const float* xX0 = params ? params->xX0 : nullptr;
  if (kfi::launch_layer_prep(ctx->g.n_layers, ctx->g.radius_cm, align, xX0, layers, st, ctx->g.zhalf_cm,
                             ctx->mat_nz) != hipSuccess)
    return KF_E_HIP;
  const kfd::Model md = model_of(ctx);
  kfi::SmoothArgs a;
  a.n = in->n;
  a.nl = ctx->g.n_layers;
  a.k.kB = md.kB;
  a.k.v_r = md.v_r;
  a.k.v_rphi = md.v_rphi;
  a.k.v_z = md.v_z;
  a.k.mass2 = md.mass2;
  a.mask = in->hit_mask;
  a.ndf = fwd->ndf;
  a.status = fwd->status;
  a.ckpt = fwd->ckpt;
  a.layers = layers;
  a.state = out->state;
  a.cov = out->cov;
  a.first = out->first;
  a.last = out->last;
  a.mat_map = ctx->mat_map;
  a.mat_nz = ctx->mat_nz;
  a.eloss = ctx->eloss;
  a.fr = ctx->fr;
  a.fz = ctx->fz;
  return kfi::launch_smooth(a, st, ctx->ev_start, ctx->ev_stop) == hipSuccess ? KF_OK : KF_E_HIP;
}

}  // extern "C"

namespace {

int run_dedup(kf_ctx* ctx, const kf_layer_params* params, kfi::DedupArgs& a, bool seeds, void* ws, size_t ws_bytes,
              void* stream) {
  const DedupWs w = dedup_ws(ctx, a.n, a.n_events);
  if (w.m >= (int64_t)INT32_MAX) return KF_E_INVALID;
  const int rc = check_ws(ws, ws_bytes, w.total);
  if (rc != KF_OK) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ws);
  kfd::LayerK* layers = reinterpret_cast<kfd::LayerK*>(base + w.layers);
  const float* align = params ? params->align : nullptr;
  const float* xX0 = params ? params->xX0 : nullptr;
  if (kfi::launch_layer_prep(ctx->g.n_layers, ctx->g.radius_cm, align, xX0, layers, st) != hipSuccess)
    return KF_E_HIP;
  const kf_dedup_cuts& c = ctx->dcuts;
  a.c = kfi::DedupCuts{c.psi_window, c.min_shared, c.min_shared_kin, c.seed_kap_rel, c.seed_kap_abs,
                       c.seed_theta, c.seed_phi, c.seed_z, c.trk_shared_frac, c.trk_kap_rel, c.trk_kap_abs,
                       c.trk_theta};
  a.nl = ctx->g.n_layers;
  a.nb = kfi::dedup_bins(c.psi_window);
  a.md = model_of(ctx);
  a.layers = layers;
  a.par = reinterpret_cast<float*>(base + w.par);
  a.spar = reinterpret_cast<float*>(base + w.spar);
  a.sint = reinterpret_cast<int32_t*>(base + w.sint);
  a.skey = reinterpret_cast<int32_t*>(base + w.skey);
  a.bin = reinterpret_cast<int32_t*>(base + w.bin);
  a.cnt = reinterpret_cast<int32_t*>(base + w.cnt);
  a.cur = reinterpret_cast<int32_t*>(base + w.cur);
  a.off = reinterpret_cast<int32_t*>(base + w.off);
  a.order = reinterpret_cast<int32_t*>(base + w.order);
  return kfi::launch_dedup(a, seeds, st) == hipSuccess ? KF_OK : KF_E_HIP;
}

}  // namespace

extern "C" {

int kf_clean_seeds(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, int32_t* keep, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!ctx || !in) return KF_E_INVALID;
  if (in->n_seeds < 0 || in->n_events < 0 || in->n_hits < 0) return KF_E_INVALID;
  if (in->n_seeds == 0) return KF_OK;
  if (!keep) return KF_E_INVALID;
  if (in->n_seeds > (int64_t)INT32_MAX - 1) return KF_E_INVALID;
  if (!in->seed_event || !in->seed_hits || (in->n_events > 0 && !in->hit_off) || (in->n_hits > 0 && !in->hits))
    return KF_E_INVALID;
  kfi::DedupArgs a{};
  a.n = in->n_seeds;
  a.n_events = in->n_events;
  a.hits = in->hits;
  a.H = in->n_hits;
  a.hit_off = in->hit_off;
  a.seed_event = in->seed_event;
  a.seed_hits = in->seed_hits;
  a.keep = keep;
  return run_dedup(ctx, params, a, true, ws, ws_bytes, stream);
}

int kf_remove_duplicates(kf_ctx* ctx, const kf_layer_params* params, const kf_tracks_in* in, int32_t* keep,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !in) return KF_E_INVALID;
  if (in->n < 0 || in->n_events < 0 || in->n_hits < 0) return KF_E_INVALID;
  if (in->n == 0) return KF_OK;
  if (!keep) return KF_E_INVALID;
  if (in->n > (int64_t)INT32_MAX - 1) return KF_E_INVALID;
  if (!in->event || !in->hit_idx || !in->n_hits_trk || !in->chi2 || !in->state || (in->n_hits > 0 && !in->hits))
    return KF_E_INVALID;
  kfi::DedupArgs a{};
  a.n = in->n;
  a.n_events = in->n_events;
  a.hits = in->hits;
  a.H = in->n_hits;
  a.event = in->event;
  a.hit_idx = in->hit_idx;
  a.n_hits = in->n_hits_trk;
  a.chi2 = in->chi2;
  a.state = in->state;
  a.keep = keep;
  return run_dedup(ctx, params, a, false, ws, ws_bytes, stream);
}

int kf_find_autotune(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out,
                     void* ws, size_t ws_bytes, void* stream, kf_find_config* best) {
  if (!ctx) return KF_E_INVALID;
  static const int kTiles[][2] = {{0, 0}, {256, 32}, {128, 64}, {256, 64}, {512, 32}, {512, 64}, {256, 128}, {1024, 32}};
  static const int kWideCoarse[] = {8, 32, 128};
  static const int kWideFine[] = {4, 16, 64};
  static const int kPer[] = {0, 12};
  static const int kLanes[] = {4, 6, 8};
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return KF_E_HIP;
  }
  const kf_find_config saved = ctx->fcfg;
  kf_find_config pick = saved;
  float best_ms = INFINITY;
  int rc = KF_OK;
  // the GPU's clock drops when it idles and takes tens of milliseconds of work to
  // return: the first configurations would be timed on a slow clock.  Run the call until
  // 100 ms of it have elapsed (at least 4 calls, at most 200) before timing anything.
  {
    float total = 0.f;
    for (int rep = 0; rep < 200 && rc == KF_OK && (rep < 4 || total < 100.f); ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = KF_E_HIP;
      if (rc == KF_OK) rc = kf_find(ctx, params, in, out, ws, ws_bytes, stream);
      if (rc == KF_OK && hipEventRecord(e1, st) != hipSuccess) rc = KF_E_HIP;
      if (rc == KF_OK && hipEventSynchronize(e1) != hipSuccess) rc = KF_E_HIP;
      float t = 0.f;
      if (rc == KF_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = KF_E_HIP;
      total += t;
    }
  }
  // times one configuration (one untimed call, then the fastest of three); configurations
  // the context rejects (a tiling beyond the bin limit for this geometry) are skipped
  auto trial = [&](kf_find_config cfg) {
    if (rc != KF_OK) return;
    if (kf_ctx_set_find_config(ctx, &cfg) != KF_OK) return;
    rc = kf_find(ctx, params, in, out, ws, ws_bytes, stream);
    float ms = INFINITY;
    for (int rep = 0; rep < 3 && rc == KF_OK; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = KF_E_HIP;
      if (rc == KF_OK) rc = kf_find(ctx, params, in, out, ws, ws_bytes, stream);
      if (rc == KF_OK && hipEventRecord(e1, st) != hipSuccess) rc = KF_E_HIP;
      if (rc == KF_OK && hipEventSynchronize(e1) != hipSuccess) rc = KF_E_HIP;
      float t = 0.f;
      if (rc == KF_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) rc = KF_E_HIP;
      if (rc == KF_OK && t < ms) ms = t;
    }
    if (rc == KF_OK && ms < best_ms) {
      best_ms = ms;
      pick = cfg;
    }
  };
  for (const auto& t : kTiles)
    for (int wide : kWideCoarse) trial(kf_find_config{wide, 0, saved.use_graph, t[0], t[1], 0});
  const kf_find_config stage1 = pick;
  for (int g : kLanes)
    if (in && g >= in->keep && g != find_group(ctx, in->keep))
      trial(kf_find_config{stage1.wide_window_bins, 0, saved.use_graph, stage1.n_phi_bins, stage1.n_z_bins, g});
  const kf_find_config stage2 = pick;
  for (int wide : kWideFine)
    trial(kf_find_config{wide, 0, saved.use_graph, stage2.n_phi_bins, stage2.n_z_bins, stage2.lanes_per_seed});
  const kf_find_config stage3 = pick;
  for (int per : kPer)
    if (per != stage3.blocks_per_cu) trial(kf_find_config{stage3.wide_window_bins, per, saved.use_graph,
                                                          stage3.n_phi_bins, stage3.n_z_bins,
                                                          stage3.lanes_per_seed});
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->fcfg = rc == KF_OK && best_ms < INFINITY ? pick : saved;
  if (rc == KF_OK && best_ms == INFINITY) rc = KF_E_INVALID;
  if (rc == KF_OK && best) *best = pick;
  return rc;
}

const char* kf_strerror(int code) {
  switch (code) {
    case KF_OK: return "ok";
    case KF_E_INVALID: return "invalid argument";
    case KF_E_UNSUPPORTED: return "unsupported request";
    case KF_E_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case KF_E_HIP: return "HIP runtime error at launch";
    case KF_E_SCRATCH: return "request exceeds the library's static scratch (kf_static_scratch_bytes)";
    default: return "unknown error code";
  }
}

}  // extern "C"
