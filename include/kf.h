/*
 * kf.h -- C ABI of the MI355X (gfx950) batched Kalman-filter track fit, combinatorial
 * track finder, adjoint of the fit, fixed-interval smoother and duplicate handling.
 *
 * The method: charged-particle tracks are fitted and built with the Kalman filter,
 * layer by layer, on symmetric 6x6 covariances, with search windows and candidate
 * scores for building and radiation lengths of every layer for multiple scattering
 * (paper, Sec. 2 and Sec. 3; window sizes and scores, Sec. 4.3); the chain ends with
 * duplicate removal and a backward pass (Sec. 4.2, Sec. 5).  Beyond one x/X0 per layer
 * and a uniform field, a context can carry the detector model of Sec. 3 (a material
 * map in (layer, z), energy loss, a parameterised field: kf_ctx_set_material,
 * kf_ctx_set_field).  The paper prints no formulas; the library implements the
 * readings stated with each call below.
 *
 * Conventions for every call
 *   - Array arguments are DEVICE pointers owned by the caller, float32 structure of
 *     arrays ("[A][B][n]" means element (a, b, i) is at (a * B + b) * n + i).
 *   - Track state (x, y, z, kappa = q/pT, phi, theta) in cm, 1/GeV, rad; the field is
 *     along +z, uniform unless kf_ctx_set_field parameterises it; omega =
 *     -0.299792458e-2 * B * kappa is the signed turning rate per unit transverse arc
 *     length.
 *   - Covariances are packed lower triangles: element (i >= j) at i * (i + 1) / 2 + j.
 *   - Layer L is an infinite cylinder of radius radius_cm[L] unless the geometry makes
 *     it a disk or bounds it (kf_geometry, endcap fields); its alignment
 *     align[L] = (dx, dy, dz, dphi) moves its axis to (dx, dy), shifts its hits (and a
 *     disk's plane) by dz and rotates them by dphi about the axis.  Hits are given in
 *     the nominal frame.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = default stream) and
 *     never synchronise (kf_find_autotune excepted).  The library allocates no device memory per call: scratch
 *     space is the caller's `ws` of at least kf_workspace_size() bytes, 256-byte
 *     aligned.  Host-detectable errors return a negative KF_E_* code before anything
 *     is launched; numerical outcomes are reported per track in `status` bits.
 *   - Outputs are bit-deterministic for given inputs.
 */
#ifndef KF_H_
#define KF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KF_MAX_LAYERS 32
#define KF_MAX_KEEP 8
#define KF_MAX_MAP_BINS 64
#define KF_MAX_FIND_BINS 32768 /* phi x z bins of kf_find's hit binning */

/* return codes */
#define KF_OK 0
#define KF_E_INVALID (-1)     /* bad argument (null pointer, size, range) */
#define KF_E_UNSUPPORTED (-2) /* valid request the library does not implement */
#define KF_E_WORKSPACE (-3)   /* workspace missing, too small or misaligned */
#define KF_E_HIP (-4)         /* the HIP runtime reported an error at launch */
#define KF_E_SCRATCH (-5)     /* request larger than the library's static scratch */

/* per-track status bits */
#define KF_ST_PROP_FAIL 1u     /* the helix does not reach a layer it must cross; the fit stops there */
#define KF_ST_NEAR_TANGENT 2u  /* some crossing had |cos alpha| < 0.3 (alpha: track vs layer normal) */
#define KF_ST_FP64_FALLBACK 4u /* S failed the FP32 condition check: S^-1 and chi2 were done in FP64 */
#define KF_ST_NONFINITE 8u     /* a non-finite value appeared */
#define KF_ST_BAD_INPUT 16u    /* hit mask lacks the seed layers */
#define KF_ST_TERM_MISSES 32u  /* finder: candidate stopped after max_miss missing layers */

/* operations for kf_workspace_size */
#define KF_OP_FIT 1
#define KF_OP_FIND 2
#define KF_OP_FIT_BACKWARD 3
#define KF_OP_SMOOTH 4
#define KF_OP_CLEAN_SEEDS 5
#define KF_OP_REMOVE_DUPLICATES 6

/* Detector and hit model, copied into the context at creation (host struct). */
typedef struct kf_geometry {
  int32_t n_layers;              /* 3 .. KF_MAX_LAYERS */
  float B_tesla;                 /* uniform field along +z; 0 allowed with external seeds */
  float radius_cm[KF_MAX_LAYERS];  /* > 0, strictly increasing over the cylinders */
  float zhalf_cm[KF_MAX_LAYERS];   /* z range [-Z, Z] of the finder's z bins (> 0) */
  float sigma_rphi_cm;           /* hit resolution along the layer (r*phi) */
  float sigma_z_cm;              /* hit resolution along z */
  float sigma_r_cm;              /* radial regulariser of the 3-D hit (its row of H is zero) */
  float mass_gev;                /* particle mass in the Highland beta */
  int32_t n_phi_bins;            /* finder bins in phi over [-pi, pi): 1 .. 1024 */
  int32_t n_z_bins;              /* finder bins in z over [-Z, Z]: 1 .. 256; kf_find needs */
                                 /* n_phi_bins * n_z_bins <= KF_MAX_FIND_BINS */
  /* Endcap disks and bounded barrel layers (Sec. 3: barrel and endcap regions); all
   * zero (as a zero-initialised struct has them) keeps every layer an infinite
   * cylinder.
   *   disk_z_cm[L] != 0: layer L is the disk in the plane z = disk_z_cm[L] (+ its
   *     alignment dz), active for disk_rmin_cm[L] <= rho <= disk_rmax_cm[L] about its
   *     axis (0 <= rmin < rmax).  Its hit is measured as (z, rho * phi, rho): the
   *     residual (z_m - z_p, rho_p * dphi, rho_m - rho_p) with variances (sigma_r^2,
   *     sigma_rphi^2, sigma_z^2), H the projection along the state's tangent onto the
   *     plane; its scattering path is x/X0 / |cos theta|.  radius_cm[L] and zhalf_cm[L]
   *     are not used (they must still be > 0); the finder bins it in phi and in rho
   *     over [rmin, rmax] (n_z_bins of them).
   *   cyl_zmax_cm[L] > 0 (cylinders only): layer L is active for |z - dz| <= zmax.
   * A disk or bounded cylinder (a bounded surface) is crossed where the track has a hit
   * on it and passed over where it has none: no propagation, no material, no miss.
   * The finder passes over a bounded surface that a candidate does not reach, or
   * reaches outside its active area.  Layers 0-2 (the seed layers) must be cylinders,
   * and cylinder radii must increase with L (disks may sit anywhere after layer 2).
   * kf_fit_backward, kf_smooth, the material model and the parameterised field return
   * KF_E_UNSUPPORTED for a geometry with bounded surfaces. */
  float disk_z_cm[KF_MAX_LAYERS];
  float disk_rmin_cm[KF_MAX_LAYERS];
  float disk_rmax_cm[KF_MAX_LAYERS];
  float cyl_zmax_cm[KF_MAX_LAYERS];
} kf_geometry;

typedef struct kf_ctx kf_ctx;

/* Per-layer parameters (device pointers, may be NULL = all zero): align [L][4], xX0 [L]
 * radiation lengths of one crossing at normal incidence. */
typedef struct kf_layer_params {
  const float* align;
  const float* xX0;
} kf_layer_params;

/* Fit input.  hits [L][3][n]; hit_mask [n] (bit L = a hit on layer L).
 * seed_from_hits != 0: each seed is the helix through the (aligned) hits on layers
 * 0, 1, 2 (needs mask bits 0-2) with a diagonal prior covariance inflated ten times
 * in variance.  Otherwise seed_state [6][n] and seed_cov [21][n] are used; the seed's
 * position must lie on layer 0's surface (the layer-0 update does not propagate).
 * ckpt_every = k (0 and 1: every layer; at most KF_MAX_LAYERS): the checkpoints are
 * kept for layers 0, k, 2k, ... only (kf_fit_out.ckpt), and kf_fit_backward recomputes
 * the layers between them: a memory/compute trade (checkpoint bytes / k, one more
 * forward step per layer between checkpoints, a [k-1][27][n] segment in its
 * workspace).  kf_smooth needs every layer (k <= 1). */
typedef struct kf_fit_in {
  int64_t n;
  const float* hits;
  const uint32_t* hit_mask;
  const float* seed_state;
  const float* seed_cov;
  int32_t seed_from_hits;
  int32_t ckpt_every;
} kf_fit_in;

/* Fit output: state [6][n], cov [21][n], chi2 [n], ndf [n] = 2 * n_hits - 5,
 * status [n]; ckpt (optional, required by kf_fit_backward) [ceil(L / k)][27][n] with
 * k = max(1, ckpt_every): slot s holds the state and covariance after layer s k (after
 * each processed layer for k = 1; a layer the track passes over, or beyond its last
 * hit, keeps the previous slot's values or is not written). */
typedef struct kf_fit_out {
  float* state;
  float* cov;
  float* chi2;
  int32_t* ndf;
  uint32_t* status;
  float* ckpt;
} kf_fit_out;

/* Finder input.  Events' hits in one array hits [3][H]; hit_off [n_events][L+1]:
 * hits of event e on layer L are hit_off[e][L] .. hit_off[e][L+1]-1.  Seeds are hit
 * triplets on layers 0, 1, 2: seed_hits [3][n_seeds] global hit indices, seed_event
 * [n_seeds].  Seeds of one event should be contiguous for locality (not required). */
typedef struct kf_find_in {  /* n_hits < 2^28 - 2 */
  int32_t n_events;
  const int64_t* hit_off;
  int64_t n_hits;
  const float* hits;
  int64_t n_seeds;
  const int32_t* seed_event;
  const int32_t* seed_hits;
  float chi2_cut;   /* a hit joins a candidate if its chi2 < chi2_cut */
  float nsigma;     /* window half widths: nsigma * sqrt(S) in r*phi and z */
  int32_t keep;     /* candidates kept per seed, 1 .. KF_MAX_KEEP */
  int32_t max_miss; /* a candidate stops at its max_miss-th missing layer, >= 1 */
  int32_t refit;    /* != 0: also fit the hits of each seed's best candidate (rf_*) */
} kf_find_in;

/* Finder output (slot k < keep, unused slots: hit_idx -2, counts 0, values 0):
 * n_cand [S]; hit_idx [keep][L][S] global hit index, -1 missing layer, -2 not reached
 * (or a bounded surface passed over);
 * n_hits, n_miss [keep][S]; chi2 [keep][S]; state [keep][6][S]; cov [keep][21][S];
 * status [keep][S]; rf_* (only with refit): the fit of the rank-0 candidate's hits,
 * seeded from its first three, as kf_fit_out.  A seed whose event is out of range, or
 * whose hit q is not in its event's slice of layer q, gets n_cand 0 and status[0][s] =
 * KF_ST_BAD_INPUT; hit_off slices are clamped to [0, n_hits]. */
typedef struct kf_find_out {
  int32_t* n_cand;
  int32_t* hit_idx;
  int32_t* n_hits;
  int32_t* n_miss;
  float* chi2;
  float* state;
  float* cov;
  uint32_t* status;
  float* rf_state;
  float* rf_cov;
  float* rf_chi2;
  int32_t* rf_ndf;
  uint32_t* rf_status;
} kf_find_out;

/* Create / destroy a context (host only, no device work).  Returns KF_OK or
 * KF_E_INVALID for an inconsistent geometry. */
int kf_ctx_create(const kf_geometry* geom, kf_ctx** ctx);
int kf_ctx_destroy(kf_ctx* ctx);

/* Threshold on the determinant of the equilibrated S (unit diagonal) below which S^-1
 * and chi2 are computed in FP64 (default 1e-2, i.e. condition numbers above ~300).
 * A threshold > 1 forces the FP64 path for every update. */
int kf_ctx_set_fallback_threshold(kf_ctx* ctx, float det_threshold);

/* Timing hook.  While start and stop (hipEvent_t, created by the caller) are both
 * non-NULL, the main kernel of every kf_fit and kf_smooth call, and the search kernel of
 * every kf_find call made without a graph (use_graph 0), is launched with
 * hipExtLaunchKernel so that the two events record the beginning and the end of that
 * kernel's own execution on the stream (the measure a kernel trace reports, without
 * the dispatch gaps between consecutive launches); hipEventElapsedTime(start, stop)
 * then gives the duration of the last such launch.  NULL, NULL (the default) turns it
 * off.  KF_E_INVALID for a NULL context or exactly one NULL event. */
int kf_ctx_set_launch_events(kf_ctx* ctx, void* start, void* stop);

/* Material model of kf_fit beyond one x/X0 per layer (Sec. 3): a table of x/X0 per
 * layer and z bin, looked up at each crossing, feeding both the scattering term and a
 * mean energy loss.
 *   xX0_map: DEVICE pointer, [n_layers][nz] float32, owned by the caller and read by
 *     every later kf_fit until the setting changes (keep it alive and unchanged while
 *     set).  Row l holds x/X0 at normal incidence at the centres of nz equal bins over
 *     the layer's [-zhalf_cm[l], zhalf_cm[l]] in its own (aligned) frame; the value at
 *     a crossing is interpolated linearly in z between the centres and held constant
 *     beyond the outer ones.  It replaces kf_layer_params.xX0.  NULL keeps the
 *     per-layer xX0.  1 <= nz <= KF_MAX_MAP_BINS.
 *   eloss_gev_per_x0: mean ionisation loss of a minimum-ionising particle per
 *     radiation length (GeV, >= 0; 0.0363 for silicon; 0 = no loss).  At each crossed
 *     layer after the seed layer, after the scattering term, the energy drops by
 *     eloss * x_eff / beta^2 (x_eff = x/X0 / (sin theta |cos alpha|), the scattering
 *     term's path length; beta at the incoming momentum) at fixed direction:
 *     kappa <- kappa p / p', and the covariance follows kappa' as a function of
 *     (kappa, theta).  A particle left without kinetic energy stops there
 *     (KF_ST_PROP_FAIL).  No straggling term.
 * kf_find (and kf_find_autotune) take the same model in every prediction of the
 * search and in the refit; a candidate whose particle stops ends there
 * (KF_ST_PROP_FAIL), holding its prediction transported to that layer.  kf_smooth
 * takes it in every step (the step's linearisation then includes the loss; the
 * batch must have been fitted under the same setting).  kf_fit_backward differentiates
 * both (with a map, its dLoss/dxX0 [l] is the derivative with respect to an additive
 * offset of map row l).  KF_E_INVALID for a NULL context, a negative or non-finite
 * loss, nz out of range with a map, or a geometry with a zhalf_cm that is not
 * positive. */
int kf_ctx_set_material(kf_ctx* ctx, const float* xX0_map, int32_t nz, float eloss_gev_per_x0);

/* Parameterised magnetic field of kf_fit (Sec. 3: a constant or parameterised field):
 * B_z(r, z) = B_tesla (1 + c_r r^2 + c_z z^2), r = sqrt(x^2 + y^2) and z in cm in the
 * global frame (coefficients in cm^-2).  Each step from one layer to the next is the
 * helix of the field at the step's starting point (the filtered position on the
 * previous layer): its crossing and its transport Jacobian use that field, which the
 * Jacobian treats as constant over the step.  A seed built from hits converts the
 * three-hit curvature into kappa with the field at hit 0.  0, 0 (the default) is the
 * uniform field.  kf_find and kf_smooth take the same field.  kf_fit_backward takes
 * it too, including the field's change where a parameter moves a step's start point
 * or the seed's first hit (the exact derivative of the fit's total chi2).
 * KF_E_INVALID for a NULL context or a non-finite coefficient; KF_E_UNSUPPORTED for a
 * nonzero coefficient when B_tesla is 0. */
int kf_ctx_set_field(kf_ctx* ctx, float c_r, float c_z);

/* Launch configuration of kf_find, held by the context.  Outputs do not depend on it
 * (same bits for every valid configuration); only the time does.
 *   n_phi_bins, n_z_bins: the tiling of each (event, layer)'s hits into bins over
 *     [-pi, pi) x [-Z, Z] that the search walks (0 = the geometry's n_phi_bins,
 *     n_z_bins).  Every window is covered by the bins it overlaps, and the hits tested
 *     inside it and their order of preference do not depend on the tiling, so finer
 *     bins change only how many hits outside the window are looked at.  1 .. 1024 and
 *     1 .. 256, product at most KF_MAX_FIND_BINS.
 *   lanes_per_seed: the lanes of a 64-lane wave that hold one seed's candidates (one
 *     candidate per lane): 4, 6 or 8, at least the call's keep (a call with keep above
 *     it returns KF_E_INVALID); 0 (the default) = the fewest of these that hold keep.
 *     A wave works on 64 / lanes_per_seed seeds at once, so the candidates per wave are
 *     that times keep: with keep = 6, 60 at 6 lanes per seed and 48 at 8.
 *   wide_window_bins: a candidate whose search window overlaps more than this many
 *     bins is scanned by all 64 lanes of its wave instead of its own lane (>= 0;
 *     default 16; 0 sends every window to the wave-wide scan).
 *   blocks_per_cu: persistent find workgroups per compute unit (0 = as many as fit;
 *     default 0).
 *   use_graph: 1 = kf_find captures its launches (layer constants, binning, search,
 *     refit) into a hipGraph on a stream of the context's own at the first call with
 *     a given set of arguments (pointers, sizes, options, configuration, device) and
 *     replays the instantiated graph on the caller's stream for every later call with
 *     the same arguments; the four most recently used graphs are kept until the
 *     context is destroyed.  Replays read the buffers' contents at replay time.  The
 *     graph holds no memset nodes.  0 = plain launches (default).  A context is not
 *     thread-safe. */
typedef struct kf_find_config {
  int32_t wide_window_bins;
  int32_t blocks_per_cu;
  int32_t use_graph;
  int32_t n_phi_bins;
  int32_t n_z_bins;
  int32_t lanes_per_seed;
} kf_find_config;

/* Set / read the context's kf_find configuration.  KF_E_INVALID for negative fields,
 * use_graph other than 0 or 1, or a bin tiling out of range. */
int kf_ctx_set_find_config(kf_ctx* ctx, const kf_find_config* cfg);
int kf_ctx_get_find_config(const kf_ctx* ctx, kf_find_config* cfg);

/* Workspace bytes needed by op (KF_OP_*) for the input `in` (a kf_fit_in or
 * kf_find_in; for KF_OP_FIT_BACKWARD and KF_OP_SMOOTH the kf_fit_in of the forward
 * call; for KF_OP_CLEAN_SEEDS a kf_find_in; for KF_OP_REMOVE_DUPLICATES a
 * kf_tracks_in; the last two also depend on the context's psi_window).  0 for
 * KF_OP_FIT (ws may then be NULL). */
int kf_workspace_size(const kf_ctx* ctx, int op, const void* in, size_t* bytes);

/* Batched Kalman fit, one track per GPU lane.  For every track: seed at layer 0,
 * update with hit 0, then for each later layer up to the last hit: propagate to the
 * first forward crossing of the helix with the layer, C <- J C J^T + Q (fixed-arc
 * transport Jacobian J, Highland multiple scattering Q of the layer's material at the
 * crossing angle), and where the layer has a hit: S = H C H^T + V in the local
 * cylindrical frame (H: the state's tangent line projected onto the layer), S^-1 by an
 * equilibrated inverse with the FP64 fallback above, chi2, gain K = C H^T S^-1 and
 * the Joseph-form update.  A bounded surface (disk, bounded cylinder) without a hit
 * is passed over; on a disk the crossing is that with its plane and the frame is the
 * plane's (kf_geometry).  Paper: Sec. 2 (Kalman filter on 6x6 covariances), Sec. 3
 * (geometry, material), Sec. 5 (the fitting step). */
int kf_fit(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* out,
           void* ws, size_t ws_bytes, void* stream);

/* Combinatorial track finding (paper Sec. 2: seeds processed in batches; Sec. 4.3:
 * search windows and candidate scores).  Hits are binned per event and layer into
 * n_phi_bins x n_z_bins; every seed is refitted over its three hits, then for each
 * layer 3 .. L-1 every live candidate is propagated, the hits inside its window
 * (|dphi| <= nsigma sqrt(S_rphi)/rho, |dz| <= nsigma sqrt(S_z)) get a chi2 with the
 * candidate's S^-1, hits with chi2 < chi2_cut and one missing-hit branch per
 * candidate compete, and the best `keep` branches per seed survive, ranked by (more
 * hits, smaller total chi2, parent rank, smaller hit index, missing-hit branch last).
 * Survivors with a hit are updated.  A candidate stops at its max_miss-th missing
 * layer or when propagation fails and is carried unchanged.  On a bounded surface a
 * candidate that does not reach it, or reaches it outside its active area, offers one
 * branch that passes it over (unchanged, no miss) instead of a missing-hit branch; on a
 * disk the window's second coordinate is rho (|drho| <= nsigma sqrt(S_rho)). */
int kf_find(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out,
            void* ws, size_t ws_bytes, void* stream);

/* Autotuner of kf_find's configuration for inputs like `in`: runs kf_find (arguments
 * as for kf_find; `out` receives the usual results) under candidate configurations:
 * after running the call until 100 ms of it have elapsed (the GPU's clock settles), it
 * times three calls of each with HIP events on `stream` (after one untimed call), keeps
 * the fastest in the context and copies it to *best (if not NULL).  The candidates:
 * the bin tiling (the geometry's, and phi x z = 256 x 32, 128 x 64, 256 x 64, 512 x 32,
 * 512 x 64, 256 x 128, 1024 x 32) crossed with wide_window_bins 8, 32, 128 (lanes per
 * seed 0); then, from the best, each other lanes_per_seed of 4, 6, 8 that holds keep;
 * then wide_window_bins 4, 16, 64; then blocks_per_cu 0, 12; use_graph as set.  Unlike every other call it SYNCHRONISES on `stream`.  On error the previous
 * configuration is kept and the error code returned. */
int kf_find_autotune(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, const kf_find_out* out,
                     void* ws, size_t ws_bytes, void* stream, kf_find_config* best);

/* Adjoint of kf_fit (seed_from_hits must be 1 and ckpt filled by the forward call, `in`
 * with that call's ckpt_every): given dchi2 [n] = dLoss/dchi2_i, accumulates
 * dLoss/dalign [L][4] and dLoss/dxX0 [L] (overwritten, float32) by a reverse sweep
 * over each track's layers that recomputes every step from its checkpoint (with sparse
 * checkpoints, each run of layers between two stored ones is first recomputed forward
 * from the lower one into the workspace).  The paper has no differentiation; this is the
 * vector-Jacobian product of the fit as implemented by kf_fit: every S^-1 is recomputed
 * as the forward formed it (equilibrated, in FP64 below the context's fallback
 * threshold).  Under a parameterised field (kf_ctx_set_field; the forward call must
 * have run under the same field) the field at each step's start and at the seed's
 * first hit is differentiated with those points.  Under the material model
 * (kf_ctx_set_material; the forward call under the same setting) the map's value at
 * each crossing moves with the crossing's z (its interpolation's slope), the energy
 * loss's change of kappa and its linearisation of the covariance are differentiated,
 * and with a map dxX0 [l] is the derivative with respect to an additive offset of the
 * map's row l (the per-layer xX0 is then not used). */
int kf_fit_backward(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
                    const float* dchi2, float* dalign, float* dxX0, void* ws, size_t ws_bytes, void* stream);

/* kf_fit_backward for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the same
 * reverse sweep and the same bits as kf_fit_backward, with its workspace (the layer
 * table, the per-block FP64 partials and, with checkpoints every k > 1 layers, the
 * recomputed segment: kf_workspace_size(KF_OP_FIT_BACKWARD, in) bytes) taken from a
 * scratch array that the library holds in every GPU's memory instead of from a
 * caller's `ws`.  The scratch is kf_static_scratch_bytes() = 16 MiB per GPU, held from
 * the first call on that GPU until the process ends (17 layers with every layer's
 * checkpoint: up to ~1.5e6 tracks; 32 layers: ~8e5; the segment takes (k - 1) x 108
 * bytes per track more).  A larger request returns KF_E_SCRATCH
 * before anything is launched; other errors as kf_fit_backward.  The call allocates
 * nothing.  Every call on one GPU shares that GPU's scratch, whatever the context or
 * stream: calls that may overlap on one GPU (different streams, threads) race and
 * must be serialised by the caller.  The scratch keeps the last call's contents;
 * nothing in it needs clearing (every byte is written before it is read). */
int kf_fit_backward_static(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
                           const float* dchi2, float* dalign, float* dxX0, void* stream);

/* Bytes of the static scratch of kf_fit_backward_static (per GPU). */
size_t kf_static_scratch_bytes(void);

/* Output of kf_smooth: state [L][6][n] and cov [L][21][n] (packed lower triangle) of
 * every layer first[i]..last[i] of track i, zero on the other layers; last [n] = the
 * last layer with an update (-1 for a track without one: all layers zero); first [n]
 * = the innermost layer smoothed (0, unless a step failed: see kf_smooth). */
typedef struct kf_smooth_out {
  float* state;
  float* cov;
  int32_t* first;
  int32_t* last;
} kf_smooth_out;

/* Fixed-interval (Rauch-Tung-Striebel) smoother over a fitted batch: the backward
 * pass over the built tracks that ends the paper's chain (Sec. 4.2, Sec. 5), on the
 * filter's own linearisation.  `in` and `params` are those of the forward kf_fit call
 * and `fwd` its output, which must hold the checkpoints (fwd->ckpt).  For every track,
 * from its last updated layer (smoothed = filtered there) down to layer 0: the step
 * to the next layer out is predicted from the checkpoint as the fit does it (x_p,
 * C_p = J C_f J^T + Q) and
 *   G = C_f J^T C_p^-1,  x_s = x_f + G (x_s' - x_p),  C_s = C_f + G (C_s' - C_p) G^T,
 * in float, except C_p's factorisation and the filtered-covariance term, which are
 * formed in double in a cancellation-free arrangement.  If a step fails (the next
 * layer is not reached from a checkpoint, or C_p is not positive definite) the
 * smoothing of that track stops and `first` records where.  A track whose fit ended
 * with BAD_INPUT has last = first = -1.  KF_E_INVALID for a NULL context, input or
 * output array, n < 0, n > 2^29 (far beyond what the checkpoints of one GPU's memory
 * hold: 1.8 KB per track at 17 layers), or fwd->ckpt NULL; KF_E_UNSUPPORTED for
 * in->ckpt_every > 1;
 * KF_E_WORKSPACE for a short or misaligned workspace.  Workspace:
 * kf_workspace_size(KF_OP_SMOOTH, in). */
int kf_smooth(kf_ctx* ctx, const kf_layer_params* params, const kf_fit_in* in, const kf_fit_out* fwd,
              const kf_smooth_out* out, void* ws, size_t ws_bytes, void* stream);

/* Duplicate handling (Sec. 4.2): seed cleaning before building and duplicate removal
 * after it.  The paper names the quantities compared (pT, eta and phi of seeds or
 * tracks, and shared hits) but no cuts; these are the context's (defaults below, set
 * with kf_ctx_set_dedup_cuts).  Both calls read the relation as pairwise within an
 * event with a priority order: an item is removed when an item of higher priority in
 * its event is its duplicate.  It is not made transitive (a removed item still removes
 * the items below it), so the result does not depend on evaluation order and is
 * bit-deterministic.  Every duplicate pair lies within psi_window in psi, the azimuth
 * of the item's first (placed) hit; the library bins each event's items in psi to
 * bound the search.  Differences use the azimuth wrapped to (-pi, pi]. */
typedef struct kf_dedup_cuts {
  float psi_window;     /* rad; default 0.05 */
  int32_t min_shared;   /* seeds: shared hits that alone make a duplicate; default 2 */
  int32_t min_shared_kin; /* seeds: shared hits needed for the kinematic test; default 1 */
  float seed_kap_rel, seed_kap_abs; /* |dkappa| <= rel * max|kappa| + abs; 0.1, 0.15 1/GeV */
  float seed_theta, seed_phi, seed_z; /* |dtheta|, |dphi| (rad), |dz| (cm); 0.03, 0.02, 0.5 */
  float trk_shared_frac; /* tracks: shared >= frac * min(n_hits); 0.5 */
  float trk_kap_rel, trk_kap_abs; /* tracks: |dkappa| cut as for seeds; 0.1, 0.01 1/GeV */
  float trk_theta;      /* tracks: |dtheta| (rad); 0.02 */
} kf_dedup_cuts;

/* Set / read the context's duplicate cuts.  KF_E_INVALID for a NULL argument, a
 * non-positive psi_window, negative cuts or min_shared_kin > min_shared. */
int kf_ctx_set_dedup_cuts(kf_ctx* ctx, const kf_dedup_cuts* cuts);
int kf_ctx_get_dedup_cuts(const kf_ctx* ctx, kf_dedup_cuts* cuts);

/* Seed cleaning.  Input: the events' hits and seeds of a kf_find_in (n_events,
 * hit_off, n_hits, hits, n_seeds, seed_event, seed_hits; the other fields unused).  A
 * seed takes part if its event is in range and each hit q lies in its event's slice of
 * layer q; others are kept.  A seed's kinematics are the three-hit helix at its first
 * placed hit (as kf_fit's seed): kappa, theta, phi, z.  Seeds i, j of one event are
 * duplicates when |dpsi| <= psi_window and either they share >= min_shared hits (the
 * same global index on the same layer), or they share >= min_shared_kin hits and
 * |dkappa| <= seed_kap_rel * max(|kappa_i|, |kappa_j|) + seed_kap_abs, |dtheta| <=
 * seed_theta, |dphi| <= seed_phi, |dz| <= seed_z.  Priority: the lower seed index.
 * Output keep [n_seeds] int32: 1 kept, 0 removed.  KF_E_INVALID for a NULL context,
 * input or array, negative counts; KF_E_WORKSPACE for a short workspace
 * (kf_workspace_size(KF_OP_CLEAN_SEEDS, in)). */
int kf_clean_seeds(kf_ctx* ctx, const kf_layer_params* params, const kf_find_in* in, int32_t* keep, void* ws,
                   size_t ws_bytes, void* stream);

/* Built tracks for kf_remove_duplicates, e.g. each seed's rank-0 finder candidate:
 * event [n]; hit_idx [L][n] global hit indices into hits [3][n_hits] (< 0: none);
 * n_hits_trk [n]; chi2 [n]; state [6][n] (kappa and theta are compared; e.g. the
 * refit's rf_state). */
typedef struct kf_tracks_in {
  int32_t n_events;
  int64_t n_hits;
  const float* hits;
  int64_t n;
  const int32_t* event;
  const int32_t* hit_idx;
  const int32_t* n_hits_trk;
  const float* chi2;
  const float* state;
} kf_tracks_in;

/* Duplicate removal over built tracks.  A track takes part if its event is in range,
 * n_hits_trk > 0 and it has a hit index in [0, n_hits); psi is the azimuth of the placed
 * hit on its lowest such layer.  Tracks i, j of one event are duplicates when |dpsi| <=
 * psi_window, they share at least trk_shared_frac * min(n_hits_trk) hits (the same hit
 * on the same layer), |dkappa| <= trk_kap_rel * max|kappa| + trk_kap_abs and |dtheta|
 * <= trk_theta.  Priority: more hits, then lower chi2, then the lower index.  Output
 * keep [n] int32.  Errors as kf_clean_seeds; workspace
 * kf_workspace_size(KF_OP_REMOVE_DUPLICATES, in). */
int kf_remove_duplicates(kf_ctx* ctx, const kf_layer_params* params, const kf_tracks_in* in, int32_t* keep,
                         void* ws, size_t ws_bytes, void* stream);

/* Static description of a return code. */
const char* kf_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* KF_H_ */
