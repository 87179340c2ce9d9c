// Duplicate handling (kf_clean_seeds before building, kf_remove_duplicates after it).
//
// Both steps decide, for every item (a seed, or a built track), whether an item of
// higher priority in the same event is its duplicate; the relation itself is stated
// in kf.h.  Every duplicate pair lies within psi_window in the azimuth psi of the
// items' first hits, so the items of each event are counting-sorted into nb azimuth
// bins at least psi_window wide and an item compares itself only with the items of its
// own bin and the two next to it.  The decision (does such a j exist) does not depend
// on the order within a bin, so the atomic scatter leaves the result deterministic.
//
//   zero_kernel      counts and cursors to 0 (a kernel, so that the chain can be captured)
//   *_keys_kernel    per item: psi, the compared quantities, its bin; counts per bin
//   scan_kernel      exclusive scan of the counts (one workgroup)
//   scatter_kernel   item indices, and the compared quantities, into their bins
//   *_decide_kernel  per sorted item: scan the three bins, keep = no duplicate of higher
//                    priority
#include <cmath>

#include "kf_internal.h"

namespace kfi {

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ int psi_bin(float psi, int nb) {
  int b = (int)floorf((psi + kfd::kPi) * ((float)nb / kfd::kTwoPi));
  return b < 0 ? 0 : (b >= nb ? nb - 1 : b);
}

__global__ __launch_bounds__(kBlock) void zero_kernel(int32_t* __restrict__ p, int64_t n) {
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlock) p[k] = 0;
}

// Seeds: a seed takes part if its event and its three hits (each inside its event's
// slice of its layer) are valid.  par: psi, kappa, theta, phi, z at the first hit.
__global__ __launch_bounds__(kBlock) void seed_keys_kernel(DedupArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int32_t e = a.seed_event[i];
  bool ok = e >= 0 && e < a.n_events;
  int32_t h[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    h[l] = a.seed_hits[(int64_t)l * a.n + i];
    if (ok) {
      const int64_t* off = a.hit_off + (int64_t)e * (a.nl + 1);
      ok = h[l] >= 0 && (int64_t)h[l] < a.H && (int64_t)h[l] >= off[l] && (int64_t)h[l] < off[l + 1];
    }
  }
  if (!ok) {
    a.bin[i] = -1;
    a.keep[i] = 1;
    return;
  }
  float m[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l)
    kfd::place(a.layers[l], a.hits[h[l]], a.hits[a.H + h[l]], a.hits[2 * a.H + h[l]], m[l][0], m[l][1], m[l][2]);
  kfd::Trk k;
  kfd::seed_from_three(k, a.md, m[0][0], m[0][1], m[0][2], m[1][0], m[1][1], m[2][0], m[2][1], m[2][2], 0.f, 0.f);
  const float psi = atan2f(m[0][1], m[0][0]);
  a.par[0 * a.n + i] = psi;
  a.par[1 * a.n + i] = k.x[3];
  a.par[2 * a.n + i] = k.x[5];
  a.par[3 * a.n + i] = k.x[4];
  a.par[4 * a.n + i] = k.x[2];
  const int b = psi_bin(psi, a.nb);
  a.bin[i] = b;
  atomicAdd(&a.cnt[(int64_t)e * a.nb + b], 1);
}

// Tracks: a track takes part if its event is valid, it has hits and one of them lies
// in [0, H).  par: psi (placed first hit), kappa, theta, chi2.
__global__ __launch_bounds__(kBlock) void track_keys_kernel(DedupArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int32_t e = a.event[i];
  int first = -1;
  int32_t h = 0;
  if (e >= 0 && e < a.n_events && a.n_hits[i] > 0)
    for (int l = 0; l < a.nl && first < 0; ++l) {
      const int32_t j = a.hit_idx[(int64_t)l * a.n + i];
      if (j >= 0 && (int64_t)j < a.H) {
        first = l;
        h = j;
      }
    }
  if (first < 0) {
    a.bin[i] = -1;
    a.keep[i] = 1;
    return;
  }
  float mx, my, mz;
  kfd::place(a.layers[first], a.hits[h], a.hits[a.H + h], a.hits[2 * a.H + h], mx, my, mz);
  const float psi = atan2f(my, mx);
  a.par[0 * a.n + i] = psi;
  a.par[1 * a.n + i] = a.state[3 * a.n + i];
  a.par[2 * a.n + i] = a.state[5 * a.n + i];
  a.par[3 * a.n + i] = a.chi2[i];
  a.par[4 * a.n + i] = 0.f;
  const int b = psi_bin(psi, a.nb);
  a.bin[i] = b;
  atomicAdd(&a.cnt[(int64_t)e * a.nb + b], 1);
}

// Exclusive scan of cnt[0..m) into off[0..m] by one workgroup of 1024 lanes: each lane
// sums a contiguous chunk, the chunk sums are scanned in LDS, each lane writes its
// chunk's prefixes.
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ cnt, int32_t* __restrict__ off,
                                                    int64_t m) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (m + 1023) / 1024;
  const int64_t b = t * chunk, e = b + chunk < m ? b + chunk : m;
  int32_t s = 0;
  for (int64_t k = b; k < e; ++k) s += cnt[k];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
    const int32_t v = t >= d ? part[t - d] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int32_t run = t > 0 ? part[t - 1] : 0;
  for (int64_t k = b; k < e; ++k) {
    off[k] = run;
    run += cnt[k];
  }
  if (t == 1023) off[m] = part[1023];
}

// Item i to its place in its bin, with a copy of what the decision compares (par, and
// the seed's hits or the track's hit count) at that place, so that the decision reads
// each bin as one contiguous run.
__global__ __launch_bounds__(kBlock) void scatter_kernel(DedupArgs a, const int32_t* __restrict__ event, int seeds) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= a.n) return;
  const int b = a.bin[i];
  if (b < 0) return;
  const int64_t key = (int64_t)event[i] * a.nb + b;
  const int64_t s = a.off[key] + atomicAdd(&a.cur[key], 1);
  const int64_t n = a.n;
  a.order[s] = (int32_t)i;
  a.skey[s] = (int32_t)key;
#pragma unroll
  for (int q = 0; q < 5; ++q) a.spar[q * n + s] = a.par[q * n + i];
  if (seeds) {
#pragma unroll
    for (int l = 0; l < 3; ++l) a.sint[l * n + s] = a.seed_hits[l * n + i];
  } else {
    a.sint[s] = a.n_hits[i];
  }
}

// Visit the sorted places of bins b-1, b, b+1 (wrapped, each bin once) of the bin
// `key` belongs to.  Consecutive lanes hold consecutive places, mostly of one bin, so
// their loops run over the same places.  The places come in chunks of 8 whose azimuth,
// row `r2` of the sorted quantities and item index are loaded together (loads in
// flight together, not one by one); pre(psi_q, x_q, j) is the cheap first test,
// full(q, j) the rest of the relation; the walk stops at the first place that passes
// both.
template <class Pre, class Full>
__device__ __forceinline__ bool for_neighbours(const DedupArgs& a, int32_t key, int r2, Pre pre, Full full) {
  constexpr int kChunk = 8;
  const int b = key % a.nb;
  const int64_t e0 = (int64_t)key - b;
  const int nd = a.nb >= 3 ? 3 : a.nb;
  for (int d = 0; d < nd; ++d) {
    int bb = b + (d == 0 ? 0 : (d == 1 ? 1 : -1));
    if (bb >= a.nb) bb -= a.nb;
    if (bb < 0) bb += a.nb;
    const int32_t s1 = a.off[e0 + bb + 1];
    for (int32_t q0 = a.off[e0 + bb]; q0 < s1; q0 += kChunk) {
      float ps[kChunk], xs[kChunk];
      int32_t jj[kChunk];
#pragma unroll
      for (int k = 0; k < kChunk; ++k) {
        const int32_t q = q0 + k < s1 ? q0 + k : s1 - 1;  // in range; repeats are tested once
        ps[k] = a.spar[q];
        xs[k] = a.spar[(int64_t)r2 * a.n + q];
        jj[k] = a.order[q];
      }
#pragma unroll
      for (int k = 0; k < kChunk; ++k)
        if (q0 + k < s1 && pre(ps[k], xs[k], jj[k]) && full(q0 + k, jj[k])) return true;
    }
  }
  return false;
}

// One lane per sorted place s (item i = order[s]).
__global__ __launch_bounds__(kBlock) void clean_decide_kernel(DedupArgs a, int64_t m) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= a.off[m]) return;
  const int64_t n = a.n;
  const int32_t i = a.order[s];
  const float psi = a.spar[s], kap = a.spar[n + s], th = a.spar[2 * n + s], ph = a.spar[3 * n + s],
              z = a.spar[4 * n + s];
  int32_t h[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) h[l] = a.sint[l * n + s];
  const DedupCuts c = a.c;
  const bool dup = for_neighbours(
      a, a.skey[s], 0,
      [&](float psi_q, float, int32_t j) {  // priority (the lower index), then the window
        return j < i && fabsf(kfd::wrap_pi(psi - psi_q)) <= c.psi_window;
      },
      [&](int32_t q, int32_t) {
        int shared = 0;
#pragma unroll
        for (int l = 0; l < 3; ++l) shared += a.sint[l * n + q] == h[l];
        if (shared >= c.min_shared) return true;
        if (shared < c.min_shared_kin) return false;
        const float kj = a.spar[n + q];
        const float kcut = c.seed_kap_rel * fmaxf(fabsf(kap), fabsf(kj)) + c.seed_kap_abs;
        return fabsf(kap - kj) <= kcut && fabsf(th - a.spar[2 * n + q]) <= c.seed_theta &&
               fabsf(kfd::wrap_pi(ph - a.spar[3 * n + q])) <= c.seed_phi && fabsf(z - a.spar[4 * n + q]) <= c.seed_z;
      });
  a.keep[i] = dup ? 0 : 1;
}

__global__ __launch_bounds__(kBlock) void remove_decide_kernel(DedupArgs a, int64_t m) {
  const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (s >= a.off[m]) return;
  const int64_t n = a.n;
  const int32_t i = a.order[s];
  const float psi = a.spar[s], kap = a.spar[n + s], th = a.spar[2 * n + s], c2 = a.spar[3 * n + s];
  const int32_t nh = a.sint[s];
  const DedupCuts c = a.c;
  const bool dup = for_neighbours(
      a, a.skey[s], 2,
      [&](float psi_q, float th_q, int32_t j) {  // the window and theta reject nearly all
        return j != i && fabsf(kfd::wrap_pi(psi - psi_q)) <= c.psi_window && fabsf(th - th_q) <= c.trk_theta;
      },
      [&](int32_t q, int32_t j) {
        const int32_t nj = a.sint[q];
        const float cj = a.spar[3 * n + q];
        const bool higher = nj != nh ? nj > nh : (cj != c2 ? cj < c2 : j < i);
        if (!higher) return false;
        const float kj = a.spar[n + q];
        const float kcut = c.trk_kap_rel * fmaxf(fabsf(kap), fabsf(kj)) + c.trk_kap_abs;
        if (!(fabsf(kap - kj) <= kcut)) return false;
        int shared = 0;
        for (int l = 0; l < a.nl; ++l) {
          const int32_t hi = a.hit_idx[(int64_t)l * n + i];
          shared += hi >= 0 && hi == a.hit_idx[(int64_t)l * n + j];
        }
        return (float)shared >= c.trk_shared_frac * (float)(nj < nh ? nj : nh);
      });
  a.keep[i] = dup ? 0 : 1;
}

unsigned grid_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int dedup_bins(float psi_window) {
  // bins at least psi_window (1 + 1e-4) wide, so that every pair within the window is
  // in the same or adjacent bins despite the rounding of the bin arithmetic
  const double w = (double)psi_window * (1.0 + 1e-4);
  if (!(w > 0.0)) return 1;
  const double nb = std::floor(6.283185307179586 / w);
  return nb < 1.0 ? 1 : (nb > 4096.0 ? 4096 : (int)nb);
}

hipError_t launch_dedup(const DedupArgs& a, bool seeds, hipStream_t stream) {
  const int64_t m = (int64_t)a.n_events * a.nb;
  hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(kBlock), 0, stream, a.cnt, m);
  hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(kBlock), 0, stream, a.cur, m);
  if (seeds)
    hipLaunchKernelGGL(seed_keys_kernel, dim3(grid_of(a.n)), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(track_keys_kernel, dim3(grid_of(a.n)), dim3(kBlock), 0, stream, a);
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, stream, a.cnt, a.off, m);
  hipLaunchKernelGGL(scatter_kernel, dim3(grid_of(a.n)), dim3(kBlock), 0, stream, a,
                     seeds ? a.seed_event : a.event, seeds ? 1 : 0);
  if (seeds)
    hipLaunchKernelGGL(clean_decide_kernel, dim3(grid_of(a.n)), dim3(kBlock), 0, stream, a, m);
  else
    hipLaunchKernelGGL(remove_decide_kernel, dim3(grid_of(a.n)), dim3(kBlock), 0, stream, a, m);
  return hipGetLastError();
}

}  // namespace kfi
