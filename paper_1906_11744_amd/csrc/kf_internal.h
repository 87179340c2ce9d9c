// Internal launch interface between the C ABI (kf_api.hip) and the kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_adjoint.h"
#include "kf_device.h"

namespace kfi {

// Endcap surfaces per layer (kf_geometry's fields; all zero: every layer an infinite
// cylinder): a disk's plane z (0: a cylinder) and radii, a cylinder's |z| bound (0: none).
struct Surfaces {
  float disk_z[32], rmin[32], rmax[32], zmax[32];
};

// Constants of layer l: radius, alignment (centre shift, z shift, cos/sin of the
// rotation), material, endcap surface.  align / xX0 may be null (all zero); zhalf / nz
// place the bins of a material map (nz = 0: none); zd, rmin, rmax, zmax: the layer's
// Surfaces entries (all 0: an infinite cylinder).
__device__ __forceinline__ kfd::LayerK make_layer(int l, const float* radius, const float* __restrict__ align,
                                                  const float* __restrict__ xX0, const float* zhalf = nullptr,
                                                  int nz = 0, float zd = 0.f, float rmin = 0.f, float rmax = 0.f,
                                                  float zmax = 0.f) {
  kfd::LayerK k;
  k.zs = (nz > 1) ? (float)nz / (2.f * zhalf[l]) : 0.f;
  k.zo = 0.5f * (float)nz - 0.5f;
  k.r = radius[l];
  k.cx = align ? align[4 * l + 0] : 0.f;
  k.cy = align ? align[4 * l + 1] : 0.f;
  k.dz = align ? align[4 * l + 2] : 0.f;
  const float dphi = align ? align[4 * l + 3] : 0.f;
  sincosf(dphi, &k.sphi, &k.cphi);
  k.xX0 = xX0 ? xX0[l] : 0.f;
  k.moved = (k.cx != 0.f || k.cy != 0.f || k.dz != 0.f || dphi != 0.f) ? 1.f : 0.f;
  k.disk = zd != 0.f ? 1.f : 0.f;
  k.bounded = (zd != 0.f || zmax > 0.f) ? 1.f : 0.f;
  k.zp = zd != 0.f ? zd + k.dz : 0.f;
  k.lo = zd != 0.f ? rmin : 0.f;
  k.hi = zd != 0.f ? rmax : zmax;
  return k;
}

// Kernel variants: one x/X0 per layer and a uniform field; the detector model (material
// map, energy loss, parameterised field); bounded surfaces (disks, bounded cylinders)
// with one x/X0 per layer and a uniform field.
enum Variant : int { kPlain = 0, kModelV = 1, kBoundedV = 2 };

// Everything a fit launch needs, by value.
struct FitArgs {
  int64_t n;
  int32_t nl;
  int32_t seed_from_hits;
  kfd::Model md;
  float srphi, sz;
  const float* hits;
  const uint32_t* mask;
  const float* seed_state;
  const float* seed_cov;
  const kfd::LayerK* layers;  // [nl], prepared on the device (refit), or
  const float* align;         // computed by each fit workgroup from these (fit)
  const float* xX0;
  float radius[32];
  // detector model beyond one x/X0 per layer and a uniform field (fit only): map [nl][mat_nz] of x/X0 at
  // z-bin centres over [-zhalf, zhalf] (null: xX0), mean loss per radiation length
  const float* mat_map = nullptr;
  int32_t mat_nz = 0;
  float eloss = 0.f;
  float zhalf[32] = {};
  // parameterised field B_z(r, z) = B (1 + fr r^2 + fz z^2) (fit only; 0, 0: uniform)
  float fr = 0.f, fz = 0.f;
  // endcap surfaces (fit only: the refit reads them from the prepared layers)
  Surfaces sf = {};
  int32_t bounded = 0;  // the geometry has a disk or a bounded cylinder
  float* state;
  float* cov;
  float* chi2;
  int32_t* ndf;
  uint32_t* status;
  float* ckpt;
  int32_t ckpt_every = 1;  // checkpoint slot s holds layer s * ckpt_every
};

struct BinArgs {
  int32_t nl, nphi, nz, n_events;
  int64_t H;
  const int64_t* hit_off;  // [E][L+1]
  const float* hits;       // [3][H]
  // the layer table: each workgroup builds its layer's entry from these (as the fit
  // does), and those of event 0 store it in `layers` for the search and the refit
  kfd::LayerK* layers;
  float radius[32];
  const float* align;      // [L][4] or null
  const float* xX0;        // [L] or null
  int32_t mat_nz;
  Surfaces sf;
  float zhalf[32];
  float4* brec;            // [H] binned (x, y, z, phi) of placed hits
  float4* hpos;            // [H] the same records in the caller's hit order
  int32_t* bidx;           // [H] caller's index of each binned hit
  int32_t* boff;           // [E][L][nbins + 1] absolute start of every bin
  int32_t* counter;        // find tile queue, zeroed here
  // set by launch_bin: the number of hits staged in LDS per range, the LDS offset of
  // the per-hit bins (then places), and their size
  int32_t stage, stage_off, hold_bytes;
};

struct FindArgs {
  int32_t nl, nphi, nz, keep, max_miss, n_events;
  int32_t wide_bins;  // windows over more bins than this are scanned by the whole wave
  float chi2_cut, nsigma;
  kfd::Model md;
  float srphi, sz;
  int64_t n_seeds, H, n_tiles;
  const int64_t* hit_off;  // [E][L+1]
  const float* hits;
  const int32_t* seed_event;
  const int32_t* seed_hits;
  const kfd::LayerK* layers;
  const float4* brec;
  const float4* hpos;  // [H] placed (x, y, z, phi) of every hit in the caller's order
  const int32_t* bidx;
  const int32_t* boff;
  float zhalf[32];
  // detector model (as in FitArgs): material map [nl][mat_nz] or null, loss, field
  const float* mat_map = nullptr;
  int32_t mat_nz = 0;
  float eloss = 0.f;
  float fr = 0.f, fz = 0.f;
  int32_t bounded = 0;  // the geometry has a disk or a bounded cylinder
  int32_t* counter;
  int32_t* bp;       // [grid][nl][64] backpointers of each workgroup's current tile
  // with a refit: placed hit positions [grid][nl][3][64] of each workgroup's current tile
  // (per layer and lane, where the lane's candidate took a hit), and for every seed its
  // rank-0 candidate's placed hits rpos [nl][3][S] and their layers rmask [S]
  float* bpos = nullptr;
  float* rpos = nullptr;
  uint32_t* rmask = nullptr;
  int32_t* n_cand;
  int32_t* hit_idx;
  int32_t* n_hits;
  int32_t* n_miss;
  float* chi2;
  float* state;
  float* cov;
  uint32_t* status;
};

struct AdjArgs {
  int64_t n;
  int32_t nl;
  kfa::Consts<float> k;
  float srphi, sz, dr02;
  float fr = 0.f, fz = 0.f;  // parameterised field B_z(r, z) = B (1 + fr r^2 + fz z^2)
  const float* hits;
  const uint32_t* mask;
  const int32_t* ndf;
  const uint32_t* status;
  const float* ckpt;
  const float* dchi2;
  const kfd::LayerK* layers;
  int64_t n_blocks;  // adjoint_blocks(n)
  double* part;      // [L][5][n_blocks] per-block gradient sums
  int32_t every = 1;     // checkpoints every `every` layers (slot s = layer s * every)
  float* seg = nullptr;  // [every - 1][27][n]: the layers between two checkpoints, recomputed
  // the material model (as in FitArgs): map [nl][mat_nz] or null, mean loss per X0
  const float* mat_map = nullptr;
  int32_t mat_nz = 0;
  float eloss = 0.f;
};

// Blocks of the adjoint kernel for n tracks (one FP64 partial per block and parameter).
int64_t adjoint_blocks(int64_t n);

hipError_t launch_adjoint(const AdjArgs& a, float* dalign, float* dxX0, hipStream_t stream);

struct SmoothArgs {
  int64_t n;
  int32_t nl;
  kfa::Consts<float> k;
  const uint32_t* mask;
  const int32_t* ndf;
  const uint32_t* status;
  const float* ckpt;
  const kfd::LayerK* layers;
  float* state;    // [L][6][n]
  float* cov;      // [L][21][n]
  int32_t* first;  // [n]
  int32_t* last;   // [n]
  // detector model (as in FitArgs): material map [nl][mat_nz] or null, loss, field
  const float* mat_map = nullptr;
  int32_t mat_nz = 0;
  float eloss = 0.f;
  float fr = 0.f, fz = 0.f;
};

// Cuts of the duplicate relations (kf_dedup_cuts of kf.h, copied).
struct DedupCuts {
  float psi_window;
  int32_t min_shared, min_shared_kin;
  float seed_kap_rel, seed_kap_abs, seed_theta, seed_phi, seed_z;
  float trk_shared_frac, trk_kap_rel, trk_kap_abs, trk_theta;
};

struct DedupArgs {
  int64_t n;        // items (seeds or tracks)
  int32_t nl, n_events, nb;
  DedupCuts c;
  kfd::Model md;
  const kfd::LayerK* layers;
  const float* hits;  // [3][H]
  int64_t H;
  // seeds
  const int64_t* hit_off;
  const int32_t* seed_event;
  const int32_t* seed_hits;  // [3][n]
  // tracks
  const int32_t* event;
  const int32_t* hit_idx;  // [L][n]
  const int32_t* n_hits;
  const float* chi2;
  const float* state;  // [6][n]
  // workspace
  float* par;      // [5][n]
  float* spar;     // [5][n] par in sorted (bin) order
  int32_t* sint;   // [3][n] in sorted order: a seed's hits, or a track's hit count (row 0)
  int32_t* skey;   // [n] event * nb + bin of each sorted place
  int32_t* bin;    // [n], -1: takes no part
  int32_t* cnt;    // [n_events * nb]
  int32_t* off;    // [n_events * nb + 1]
  int32_t* cur;    // [n_events * nb]
  int32_t* order;  // [n]
  int32_t* keep;   // [n] output
};

int dedup_bins(float psi_window);
hipError_t launch_dedup(const DedupArgs& a, bool seeds, hipStream_t stream);

hipError_t launch_smooth(const SmoothArgs& a, hipStream_t stream, hipEvent_t ev_start = nullptr,
                         hipEvent_t ev_stop = nullptr);
hipError_t launch_bin(BinArgs a, hipStream_t stream);
hipError_t prepare_bin(int nbins);  // allows the bin kernel's LDS for nbins bins
size_t find_lds_bytes(int nl);
int find_tile_seeds(int lanes_per_seed);        // seeds per find tile (one workgroup)
constexpr int kMaxFindGrid = 4096;              // persistent find workgroups at most
size_t find_bp_bytes(int nl, int64_t grid);     // backpointer buffer of `grid` workgroups
// variant: a Variant (plain, detector model, bounded surfaces); lanes_per_seed: 4, 6 or
// 8 lanes hold one seed's candidates
hipError_t find_max_blocks(int nl, int variant, int lanes_per_seed, int* blocks_per_cu);
hipError_t launch_find(const FindArgs& a, int lanes_per_seed, int grid, hipStream_t stream,
                       hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

// Writes the per-layer constants (radius, alignment, its cos/sin, material; with
// zhalf_host and map_nz > 0 also the placement of the material map's z bins; with sf
// the endcap surfaces).
hipError_t launch_layer_prep(int nl, const float* radius_host, const float* align, const float* xX0,
                             kfd::LayerK* out, hipStream_t stream, const float* zhalf_host = nullptr,
                             int map_nz = 0, const Surfaces* sf = nullptr);
hipError_t launch_fit(const FitArgs& a, hipStream_t stream, hipEvent_t ev_start = nullptr,
                      hipEvent_t ev_stop = nullptr);
// Fit of each seed's rank-0 finder candidate from the placed hits the finder recorded:
// pos [L][3][n] (placed on their layers) on the layers of mask [n].
hipError_t launch_refit(const FitArgs& a, const float* pos, const uint32_t* mask, hipStream_t stream);

}  // namespace kfi
