// Adjoint of the batched fit (kf_fit_backward): one track per lane runs the reverse
// sweep of kf_adjoint.h from the forward's checkpoints and writes its per-layer
// gradient contributions; a second kernel sums them over tracks in a fixed order in
// FP64, so the result is bit-reproducible.
#include "kf_adjoint.h"
#include "kf_internal.h"

namespace kfi {

static_assert(sizeof(kfa::Lay<float>) == sizeof(kfd::LayerK), "layer table layouts must agree");

__global__ __launch_bounds__(256) void fit_adjoint_kernel(AdjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t n = a.n;
  const int nl = a.nl;
  const kfa::Lay<float>* lays = reinterpret_cast<const kfa::Lay<float>*>(a.layers);
  const uint32_t mask = a.mask[i];
  const uint32_t st = a.status[i];
  const int nh = (a.ndf[i] + 5) / 2;
  int lstart = (st & kfd::ST_BAD_INPUT) ? -1 : kfa::last_updated_layer(mask, nh, nl);
  if (lstart > nl - 1) lstart = nl - 1;
  float acc[3][5];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 5; ++q) acc[l][q] = 0.f;
  float* part = a.part;
  for (int l = nl - 1; l >= 3; --l)
    if (l > lstart)
#pragma unroll
      for (int q = 0; q < 5; ++q) part[((int64_t)l * 5 + q) * n + i] = 0.f;
  if (lstart >= 2) {
    float Cs[21];
    kfa::seed_cov(a.srphi, a.sz, a.dr02, a.k.kB, Cs);
    const float w = a.dchi2[i];
    auto hit = [&](int l, float h[3]) {
      const float* p = a.hits + (int64_t)l * 3 * n + i;
      h[0] = p[0];
      h[1] = p[n];
      h[2] = p[2 * n];
    };
    auto ckpt = [&](int l, float x[6], float C[21]) {
      const float* p = a.ckpt + (int64_t)l * 27 * n + i;
#pragma unroll
      for (int q = 0; q < 6; ++q) x[q] = p[q * n];
#pragma unroll
      for (int q = 0; q < 21; ++q) C[q] = p[(6 + q) * n];
    };
    auto emit = [&](int l, const float g[5]) {
      if (l < 3) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          if (l == 0) acc[0][q] += g[q];
          if (l == 1) acc[1][q] += g[q];
          if (l == 2) acc[2][q] += g[q];
        }
      } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) part[((int64_t)l * 5 + q) * n + i] = g[q];
      }
    };
    if (!kfa::track_adjoint<float>(lstart, mask, lays, a.k, Cs, w, hit, ckpt, emit)) {
      for (int l = 3; l <= lstart; ++l)
#pragma unroll
        for (int q = 0; q < 5; ++q) part[((int64_t)l * 5 + q) * n + i] = 0.f;
#pragma unroll
      for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int q = 0; q < 5; ++q) acc[l][q] = 0.f;
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int q = 0; q < 5; ++q) part[((int64_t)l * 5 + q) * n + i] = acc[l][q];
}

// Sum of part[o][0..n) for o = (layer, parameter), fixed order, FP64.
__global__ __launch_bounds__(256) void reduce_grad_kernel(const float* __restrict__ part, int64_t n,
                                                          float* __restrict__ dalign, float* __restrict__ dxX0) {
  __shared__ double red[256];
  const int o = blockIdx.x;
  const int tid = threadIdx.x;
  const float* p = part + (int64_t)o * n;
  double s = 0.0;
  for (int64_t i = tid; i < n; i += 256) s += (double)p[i];
  red[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const int l = o / 5, q = o % 5;
    if (q < 4) dalign[4 * l + q] = (float)red[0];
    else dxX0[l] = (float)red[0];
  }
}

hipError_t launch_adjoint(const AdjArgs& a, float* dalign, float* dxX0, hipStream_t stream) {
  const int bs = 256;
  const int64_t nb = (a.n + bs - 1) / bs;
  hipLaunchKernelGGL(fit_adjoint_kernel, dim3((unsigned)nb), dim3(bs), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(reduce_grad_kernel, dim3((unsigned)(a.nl * 5)), dim3(256), 0, stream, a.part, a.n, dalign,
                     dxX0);
  return hipGetLastError();
}

}  // namespace kfi
