// Batched Kalman fit: one track per lane, the whole layer loop in registers.
#include "kf_internal.h"

namespace kfi {

struct Radii {
  float r[32];
};

__global__ void layer_prep_kernel(int nl, Radii rad, Radii zh, int map_nz, const float* __restrict__ align,
                                  const float* __restrict__ xX0, kfd::LayerK* __restrict__ out, Surfaces sf) {
  const int l = threadIdx.x;
  if (l >= nl) return;
  out[l] = make_layer(l, rad.r, align, xX0, zh.r, map_nz, sf.disk_z[l], sf.rmin[l], sf.rmax[l], sf.zmax[l]);
}

hipError_t launch_layer_prep(int nl, const float* radius_host, const float* align, const float* xX0,
                             kfd::LayerK* out, hipStream_t stream, const float* zhalf_host, int map_nz,
                             const Surfaces* sf) {
  Radii rad, zh;
  for (int l = 0; l < 32; ++l) {
    rad.r[l] = l < nl ? radius_host[l] : 0.f;
    zh.r[l] = (zhalf_host && l < nl) ? zhalf_host[l] : 1.f;
  }
  if (!zhalf_host) map_nz = 0;
  const Surfaces none = {};
  hipLaunchKernelGGL(layer_prep_kernel, dim3(1), dim3(32), 0, stream, nl, rad, zh, map_nz, align, xX0, out,
                     sf ? *sf : none);
  return hipGetLastError();
}

__device__ __forceinline__ void store_ckpt(float* ck, int64_t n, int64_t i, int l, const kfd::Trk& k) {
  float* p = ck + (int64_t)l * 27 * n + i;
#pragma unroll
  for (int q = 0; q < 6; ++q) p[q * n] = q < 3 ? k.x[q] + k.xl[q] : (q == 4 ? kfd::wrap_pi(k.x[q]) : k.x[q]);
#pragma unroll
  for (int q = 0; q < 21; ++q) p[(6 + q) * n] = k.C[q];
}

// Hits of track i in the [L][3][n] layout, mask from the caller.
struct SoaHits {
  static constexpr bool kPlaced = false;
  const float* hits;
  const uint32_t* mask;
  __device__ void get(int64_t i, int64_t n, int l, float& hx, float& hy, float& hz) const {
    const float* h = hits + (int64_t)l * 3 * n + i;
    hx = h[0];
    hy = h[n];
    hz = h[2 * n];
  }
};

// Hits of seed i's rank-0 finder candidate, already placed on their layers by the
// finder: pos [L][3][n].
struct PlacedHits {
  static constexpr bool kPlaced = true;
  const float* pos;
  __device__ void get(int64_t i, int64_t n, int l, float& hx, float& hy, float& hz) const {
    const float* h = pos + (int64_t)l * 3 * n + i;
    hx = h[0];
    hy = h[n];
    hz = h[2 * n];
  }
};

// kVar: a Variant.  Bounded surfaces: a layer without a hit is passed over, a disk is
// reached on its plane and measured in its frame.
template <bool kCkpt, int kVar, class Src>
__device__ __forceinline__ void fit_one(const FitArgs& a, const kfd::LayerK* __restrict__ lays, int64_t i,
                                        uint32_t mask, const Src& src) {
  constexpr bool kModel = kVar == kModelV;
  constexpr bool kBounded = kVar == kBoundedV;
  const int64_t n = a.n;
  const uint32_t need = a.seed_from_hits ? 7u : 1u;
  uint32_t status = 0;
  kfd::Trk k;
  float chi2 = 0.f;
  int nh = 0;
  auto hit = [&](int l, float& mx, float& my, float& mz) {
    if constexpr (Src::kPlaced) {
      src.get(i, n, l, mx, my, mz);
    } else {
      float hx, hy, hz;
      src.get(i, n, l, hx, hy, hz);
      kfd::place(lays[l], hx, hy, hz, mx, my, mz);
    }
  };
  if ((mask & need) != need) {
    status = kfd::ST_BAD_INPUT;
#pragma unroll
    for (int q = 0; q < 6; ++q) k.x[q] = 0.f;
    k.xl[0] = k.xl[1] = k.xl[2] = 0.f;
#pragma unroll
    for (int q = 0; q < 21; ++q) k.C[q] = 0.f;
  } else {
    float m0x, m0y, m0z;
    hit(0, m0x, m0y, m0z);
    if (a.seed_from_hits) {
      float m1x, m1y, m1z, m2x, m2y, m2z;
      hit(1, m1x, m1y, m1z);
      hit(2, m2x, m2y, m2z);
      kfd::Model md0 = a.md;
      if (kModel) md0.kB = kfd::field_kB(a.md.kB, a.fr, a.fz, m0x, m0y, m0z);  // curvature to kappa at hit 0
      kfd::seed_from_three(k, md0, m0x, m0y, m0z, m1x, m1y, m2x, m2y, m2z, a.srphi, a.sz);
    } else {
#pragma unroll
      for (int q = 0; q < 6; ++q) k.x[q] = a.seed_state[q * n + i];
      k.xl[0] = k.xl[1] = k.xl[2] = 0.f;
#pragma unroll
      for (int q = 0; q < 21; ++q) k.C[q] = a.seed_cov[q * n + i];
    }
    kfd::init_trig(k);
    int last = 31 - __builtin_clz(mask);
    if (last > a.nl - 1) last = a.nl - 1;
    for (int l = 0; l <= last; ++l) {
      const kfd::LayerK ly = lays[l];
      // the layer's hit is loaded before the step, so that its latency hides behind it
      // (hits [L][3][n] is read in full; a layer without a hit ignores its values)
      float phx, phy, phz;
      src.get(i, n, l, phx, phy, phz);
      if (kBounded && ly.bounded != 0.f && !((mask >> l) & 1u)) {  // passed over
        if (kCkpt && l % a.ckpt_every == 0) store_ckpt(a.ckpt, n, i, l / a.ckpt_every, k);
        continue;
      }
      const bool disk = kBounded && ly.disk != 0.f;  // (layer 0 is a cylinder)
      if (l > 0) {
        // the step is the helix of the field at its starting point
        const float kB = kModel ? kfd::field_kB(a.md.kB, a.fr, a.fz, k.x[0] + k.xl[0], k.x[1] + k.xl[1], k.x[2])
                                : a.md.kB;
        kfd::Step st;
        if (!(disk ? kfd::plane_crossing(k, ly, kB, st) : kfd::crossing(k, ly, kB, st))) {
          status |= kfd::ST_PROP_FAIL;
          break;
        }
        kfd::transport(k, st, kB);
        if (disk) k.x[2] = ly.zp;  // on the plane exactly
      }
      const kfd::Frame f = kfd::frame_at(k, ly, disk);
      if (fabsf(f.cosa) < 0.3f) status |= kfd::ST_NEAR_TANGENT;
      if (kModel) {  // the material map at the crossing's z and the energy loss
        if (l > 0) {
          const float xx = a.mat_map ? kfd::map_xX0(a.mat_map + l * a.mat_nz, a.mat_nz, ly, k.x[2]) : ly.xX0;
          if (xx > 0.f) {
            kfd::add_scattering(k, f, xx, a.md.mass2);
            if (a.eloss > 0.f && !kfd::energy_loss(k, f, xx, a.eloss, a.md.mass2)) {
              status |= kfd::ST_PROP_FAIL;
              break;
            }
          }
        }
      } else if (l > 0 && ly.xX0 > 0.f) {
        kfd::add_scattering(k, f, ly.xX0, a.md.mass2);
      }
      if ((mask >> l) & 1u) {
        kfd::Pred p;
        kfd::prepare(k, f, a.md, p, disk);
        if (p.fp64) status |= kfd::ST_FP64;
        float mx = phx, my = phy, mz = phz;
        if constexpr (!Src::kPlaced) kfd::place(ly, phx, phy, phz, mx, my, mz);
        const kfd::Resid r = kfd::residual(k, f, ly, p, mx, my, mz, disk);
        kfd::apply_update(k, p, a.md, r.r1, r.r2, disk);
        chi2 += r.chi2;
        ++nh;
      }
      if (kCkpt && l % a.ckpt_every == 0) store_ckpt(a.ckpt, n, i, l / a.ckpt_every, k);
    }
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (!isfinite(k.x[q])) status |= kfd::ST_NONFINITE;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) a.state[q * n + i] = q < 3 ? k.x[q] + k.xl[q] : (q == 4 ? kfd::wrap_pi(k.x[q]) : k.x[q]);
#pragma unroll
  for (int q = 0; q < 21; ++q) a.cov[q * n + i] = k.C[q];
  a.chi2[i] = chi2;
  a.ndf[i] = 2 * nh - 5;
  a.status[i] = status;
}

// kCkpt: also store the state and covariance after every processed layer (a.ckpt; a
// layer passed over stores the state unchanged).  kVar: a Variant, the detector model
// (material map, energy loss, parameterised field) or bounded surfaces instead of
// infinite cylinders with one x/X0 per layer and a uniform field.
// The workgroup first builds the layer constants in LDS (one lane per layer), so that
// one kf_fit call is one kernel.  Five waves per SIMD (at most 96 VGPRs; the compiler
// spills two 8-byte values of the FP64-fallback path) hide more latency than the four
// that 112 VGPRs allow: 3% faster on the 1e6-track fit; six would spill ~30 registers.
// The bounded-surface variant carries both surface types' algebra and takes four.
template <bool kCkpt, int kVar>
__global__ __launch_bounds__(64, kVar == kBoundedV ? 4 : 5) void fit_kernel(FitArgs a) {
  __shared__ kfd::LayerK lays[32];
  const int t = threadIdx.x;
  if (t < a.nl) {
    if (kVar == kBoundedV)
      lays[t] = make_layer(t, a.radius, a.align, a.xX0, a.zhalf, 0, a.sf.disk_z[t], a.sf.rmin[t], a.sf.rmax[t],
                           a.sf.zmax[t]);
    else
      lays[t] = make_layer(t, a.radius, a.align, a.xX0, a.zhalf, kVar == kModelV ? a.mat_nz : 0);
  }
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  SoaHits src{a.hits, a.mask};
  fit_one<kCkpt, kVar>(a, lays, i, a.mask[i], src);
}

// Fit of each seed's best finder candidate from its own hits, which the finder left
// placed on their layers in pos [L][3][n] with their layers in mask [n]: one coalesced
// 4-byte load per coordinate instead of a gather from the event's hit arrays.
template <int kVar>
__global__ __launch_bounds__(256) void refit_kernel(FitArgs a, const float* __restrict__ pos,
                                                    const uint32_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  PlacedHits src{pos};
  fit_one<false, kVar>(a, a.layers, i, mask[i], src);
}

namespace {
// The variant of a launch (the API refuses the detector model with bounded surfaces).
int variant_of(const FitArgs& a) {
  if (a.mat_map != nullptr || a.eloss > 0.f || a.fr != 0.f || a.fz != 0.f) return kModelV;
  return a.bounded ? kBoundedV : kPlain;
}
}  // namespace

hipError_t launch_refit(const FitArgs& a, const float* pos, const uint32_t* mask, hipStream_t stream) {
  const int bs = 256;
  const dim3 g((unsigned)((a.n + bs - 1) / bs)), b(bs);
  switch (variant_of(a)) {
    case kModelV: hipLaunchKernelGGL(refit_kernel<kModelV>, g, b, 0, stream, a, pos, mask); break;
    case kBoundedV: hipLaunchKernelGGL(refit_kernel<kBoundedV>, g, b, 0, stream, a, pos, mask); break;
    default: hipLaunchKernelGGL(refit_kernel<kPlain>, g, b, 0, stream, a, pos, mask); break;
  }
  return hipGetLastError();
}

template <bool kCkpt, int kVar>
void launch_fit_variant(const FitArgs& a, unsigned nb, unsigned bs, hipStream_t stream, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
  if (ev_start && ev_stop)  // timing hook: the events bracket the kernel's own execution
    hipExtLaunchKernelGGL((fit_kernel<kCkpt, kVar>), dim3(nb), dim3(bs), 0, stream, ev_start, ev_stop, 0, a);
  else
    hipLaunchKernelGGL((fit_kernel<kCkpt, kVar>), dim3(nb), dim3(bs), 0, stream, a);
}

template <bool kCkpt>
void launch_fit_ckpt(const FitArgs& a, unsigned nb, unsigned bs, hipStream_t stream, hipEvent_t ev_start,
                     hipEvent_t ev_stop) {
  switch (variant_of(a)) {
    case kModelV: launch_fit_variant<kCkpt, kModelV>(a, nb, bs, stream, ev_start, ev_stop); break;
    case kBoundedV: launch_fit_variant<kCkpt, kBoundedV>(a, nb, bs, stream, ev_start, ev_stop); break;
    default: launch_fit_variant<kCkpt, kPlain>(a, nb, bs, stream, ev_start, ev_stop); break;
  }
}

hipError_t launch_fit(const FitArgs& a, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const unsigned bs = 64;  // one-wave workgroups pack the SIMDs slightly better than 256 lanes (0.7%)
  const unsigned nb = (unsigned)((a.n + bs - 1) / bs);
  if (a.ckpt) launch_fit_ckpt<true>(a, nb, bs, stream, ev_start, ev_stop);
  else launch_fit_ckpt<false>(a, nb, bs, stream, ev_start, ev_stop);
  return hipGetLastError();
}

}  // namespace kfi
