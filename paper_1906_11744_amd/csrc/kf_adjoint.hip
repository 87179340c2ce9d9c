// Adjoint of the batched fit (kf_fit_backward): one track per lane runs the reverse
// sweep of kf_adjoint.h from the forward's checkpoints; each block sums its tracks'
// per-layer gradient contributions in FP64 and a second kernel sums the blocks, both
// in a fixed order, so the result is bit-reproducible.
#include "kf_adjoint.h"
#include "kf_internal.h"

namespace kfi {

static_assert(sizeof(kfa::Lay<float>) == sizeof(kfd::LayerK), "layer table layouts must agree");

// One wave per block.  Every lane owns a row of R = 5 * nl floats in LDS (padded to an odd
// stride so that the lanes' rows start in different banks) holding its track's gradient
// contribution per (layer, parameter); after the sweep the block sums the 64 rows in lane
// order in FP64 and writes one partial per (layer, parameter).
constexpr int kAdjBlock = 64;

__host__ __device__ inline int adj_row_stride(int nl) { return 5 * nl + ((5 * nl) % 2 == 0 ? 1 : 0); }

// kField: the parameterised field; kMat: the material map and/or the energy loss.
template <bool kField, bool kMat>
__global__ __launch_bounds__(kAdjBlock) void fit_adjoint_kernel(AdjArgs a) {
  extern __shared__ float red[];
  const int R = 5 * a.nl;
  const int Rp = adj_row_stride(a.nl);
  float* my = red + threadIdx.x * Rp;
  for (int o = 0; o < R; ++o) my[o] = 0.f;
  const int64_t i = (int64_t)blockIdx.x * kAdjBlock + threadIdx.x;
  if (i < a.n) {
    const int64_t n = a.n;
    const int nl = a.nl;
    const kfa::Lay<float>* lays = reinterpret_cast<const kfa::Lay<float>*>(a.layers);
    const uint32_t mask = a.mask[i];
    const uint32_t st = a.status[i];
    const int nh = (a.ndf[i] + 5) / 2;
    int lstart = (st & kfd::ST_BAD_INPUT) ? -1 : kfa::last_updated_layer(mask, nh, nl);
    if (lstart > nl - 1) lstart = nl - 1;
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
      auto load = [&](const float* p, float x[6], float C[21]) {
#pragma unroll
        for (int q = 0; q < 6; ++q) x[q] = p[q * n];
#pragma unroll
        for (int q = 0; q < 21; ++q) C[q] = p[(6 + q) * n];
      };
      const kfa::FieldK<float> fk{a.fr, a.fz, a.srphi, a.sz, a.dr02};
      const kfa::MatK<float> mk{a.mat_map, a.mat_nz, a.eloss};
      // The filtered estimate after layer l.  With checkpoints every k > 1 layers the
      // sweep (which asks for l = lstart - 1, lstart - 2, ..., 0) meets each run of
      // layers c + 1 .. c + k - 1 from its top: the run is then recomputed forward from
      // checkpoint c into the segment buffer, and read from it until the sweep reaches c.
      const int every = a.every;
      int seg_base = -1;
      auto ckpt = [&](int l, float x[6], float C[21]) {
        const int c = l - l % every;
        if (l == c) {
          load(a.ckpt + (int64_t)(c / every) * 27 * n + i, x, C);
          return;
        }
        if (seg_base != c) {
          float xr[6], Cr[21];
          load(a.ckpt + (int64_t)(c / every) * 27 * n + i, xr, Cr);
          const int top = min(c + every - 1, lstart - 1);
          for (int q = c + 1; q <= top; ++q) {
            if (!kfa::forward_step<float>(q, mask, lays, a.k, kField ? &fk : nullptr, hit, xr, Cr, kMat ? &mk : nullptr))
              xr[0] = NAN;  // the sweep's own propagation from here then fails the track
            float* p = a.seg + (int64_t)(q - c - 1) * 27 * n + i;
#pragma unroll
            for (int t = 0; t < 6; ++t) p[t * n] = xr[t];
#pragma unroll
            for (int t = 0; t < 21; ++t) p[(6 + t) * n] = Cr[t];
          }
          seg_base = c;
        }
        load(a.seg + (int64_t)(l - c - 1) * 27 * n + i, x, C);
      };
      // layers 0..2 receive several contributions (the seed uses their hits)
      auto emit = [&](int l, const float g[5]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) my[l * 5 + q] += g[q];
      };
      if (!kfa::track_adjoint<float>(lstart, nl - 1, mask, lays, a.k, Cs, w, hit, ckpt, emit,
                                     kField ? &fk : nullptr, kMat ? &mk : nullptr))
        for (int o = 0; o < R; ++o) my[o] = 0.f;
    }
  }
  __syncthreads();
  for (int o = threadIdx.x; o < R; o += kAdjBlock) {
    double s = 0.0;
    for (int j = 0; j < kAdjBlock; ++j) s += (double)red[j * Rp + o];
    a.part[(int64_t)o * a.n_blocks + blockIdx.x] = s;
  }
}

// Sum over blocks of part[o][0..nb) for o = (layer, parameter), fixed order, FP64.
__global__ __launch_bounds__(256) void reduce_grad_kernel(const double* __restrict__ part, int64_t nb,
                                                          float* __restrict__ dalign, float* __restrict__ dxX0) {
  __shared__ double sh[256];
  const int o = blockIdx.x;
  const int tid = threadIdx.x;
  const double* p = part + (int64_t)o * nb;
  double s = 0.0;
  for (int64_t b = tid; b < nb; b += 256) s += p[b];
  sh[tid] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) sh[tid] += sh[tid + off];
    __syncthreads();
  }
  if (tid == 0) {
    const int l = o / 5, q = o % 5;
    if (q < 4) dalign[4 * l + q] = (float)sh[0];
    else dxX0[l] = (float)sh[0];
  }
}

int64_t adjoint_blocks(int64_t n) { return (n + kAdjBlock - 1) / kAdjBlock; }

hipError_t launch_adjoint(const AdjArgs& a, float* dalign, float* dxX0, hipStream_t stream) {
  if (a.n_blocks > 0) {
    const size_t lds = (size_t)kAdjBlock * adj_row_stride(a.nl) * sizeof(float);
    const dim3 g((unsigned)a.n_blocks), b(kAdjBlock);
    const bool field = a.fr != 0.f || a.fz != 0.f, mat = a.mat_map != nullptr || a.eloss > 0.f;
    if (mat) {
      if (field) hipLaunchKernelGGL((fit_adjoint_kernel<true, true>), g, b, lds, stream, a);
      else hipLaunchKernelGGL((fit_adjoint_kernel<false, true>), g, b, lds, stream, a);
    } else {
      if (field) hipLaunchKernelGGL((fit_adjoint_kernel<true, false>), g, b, lds, stream, a);
      else hipLaunchKernelGGL((fit_adjoint_kernel<false, false>), g, b, lds, stream, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(reduce_grad_kernel, dim3((unsigned)(a.nl * 5)), dim3(256), 0, stream, a.part, a.n_blocks,
                     dalign, dxX0);
  return hipGetLastError();
}

}  // namespace kfi
