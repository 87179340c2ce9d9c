// Fixed-interval smoother over a fitted batch (kf_smooth): one track per lane, walked
// from its last updated layer inwards over the forward fit's checkpoint of each layer
// with the step of kf_smooth.h.
#include "kf_internal.h"
#include "kf_smooth.h"

namespace kfi {

// Word 3 of a raw buffer resource on gfx9-family parts: 32-bit data format, no swizzle.
constexpr int32_t kBufWord3 = 0x00020000;

// kModel: each step under the detector model (material map, energy loss, field).
// Three waves per SIMD (at most 168 VGPRs, no spills): the other waves hide each
// checkpoint load's latency, which beats holding a prefetched checkpoint (27 more live
// registers, two waves per SIMD): 0.89 against 0.97 ms on the 1e6-track batch.
template <bool kModel>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void smooth_kernel(SmoothArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  // Each row of n floats is read and written through a buffer resource of its own
  // (built in scalar registers) at this lane's 32-bit byte offset (n <= 2^29 on the
  // host), so that a load or store takes no vector address arithmetic.
  const uint32_t bo = (uint32_t)i * 4u;
  const int32_t row_bytes = (int32_t)(n * 4);
  auto ld = [bo, row_bytes](const float* row) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)row, 0, row_bytes, kBufWord3);
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, bo, 0, 0));
  };
  auto st4 = [bo, row_bytes](float* row, float v) __attribute__((always_inline)) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc((void*)row, 0, row_bytes, kBufWord3);
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, bo, 0, 0);
  };
  const int nl = a.nl;
  const kfa::Lay<float>* lays = reinterpret_cast<const kfa::Lay<float>*>(a.layers);
  const uint32_t st = a.status[i];
  const int nh = (a.ndf[i] + 5) / 2;
  int lend = (st & kfd::ST_BAD_INPUT) ? -1 : kfa::last_updated_layer(a.mask[i], nh, nl);
  if (lend > nl - 1) lend = nl - 1;
  // Every lane walks the same layer index, from the outermost layer in, so that each
  // load and store of a wave covers one contiguous run of its array (lanes whose last
  // updated layers differ would otherwise address different layers in one
  // instruction).  A lane writes zeros above its last updated layer and below a
  // failed step.  Carried inwards: the smoothed covariance and the smoothed state's
  // offset from the filtered one, with the filtered state of the layer outside.
  float xf1[6], ds[6], Cs[21];
#pragma unroll
  for (int q = 0; q < 6; ++q) xf1[q] = ds[q] = 0.f;
#pragma unroll
  for (int q = 0; q < 21; ++q) Cs[q] = 0.f;
  int first = lend;
  bool live = false;
  for (int l = nl - 1; l >= 0; --l) {
    float xf[6], Cf[21], xs[6];
    const float* c = a.ckpt + (int64_t)l * 27 * n;  // the filtered estimates at layer l
#pragma unroll
    for (int q = 0; q < 6; ++q) xf[q] = ld(c + q * n);
#pragma unroll
    for (int q = 0; q < 21; ++q) Cf[q] = ld(c + (6 + q) * n);
    if (l == lend) {
      live = true;
#pragma unroll
      for (int q = 0; q < 21; ++q) Cs[q] = Cf[q];
    } else if (live) {
      kfs::StepModel<float> sm{a.mat_map ? a.mat_map + (l + 1) * a.mat_nz : nullptr, a.mat_nz, a.eloss, a.fr, a.fz};
      if (kfs::rts_step<float>(xf, Cf, xf1, lays[l + 1], a.k, ds, Cs, kModel ? &sm : nullptr))
        first = l;
      else
        live = false;
    }
    kfs::smoothed_state<float>(xf, ds, xs);  // ds = 0 at l == lend
#pragma unroll
    for (int q = 0; q < 6; ++q) st4(a.state + ((int64_t)l * 6 + q) * n, live ? xs[q] : 0.f);
#pragma unroll
    for (int q = 0; q < 21; ++q) st4(a.cov + ((int64_t)l * 21 + q) * n, live ? Cs[q] : 0.f);
#pragma unroll
    for (int q = 0; q < 6; ++q) xf1[q] = xf[q];
  }
  a.first[i] = lend < 0 ? -1 : first;
  a.last[i] = lend;
}

template <bool kModel>
void launch_smooth_variant(const SmoothArgs& a, unsigned nb, hipStream_t stream, hipEvent_t ev_start,
                           hipEvent_t ev_stop) {
  if (ev_start && ev_stop)  // timing hook: the events bracket the kernel's own execution
    hipExtLaunchKernelGGL((smooth_kernel<kModel>), dim3(nb), dim3(64), 0, stream, ev_start, ev_stop, 0, a);
  else
    hipLaunchKernelGGL((smooth_kernel<kModel>), dim3(nb), dim3(64), 0, stream, a);
}

hipError_t launch_smooth(const SmoothArgs& a, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const unsigned nb = (unsigned)((a.n + 63) / 64);
  if (a.mat_map != nullptr || a.eloss > 0.f || a.fr != 0.f || a.fz != 0.f)
    launch_smooth_variant<true>(a, nb, stream, ev_start, ev_stop);
  else
    launch_smooth_variant<false>(a, nb, stream, ev_start, ev_stop);
  return hipGetLastError();
}

}  // namespace kfi
