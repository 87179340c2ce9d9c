// Combinatorial track finding on gfx950.
//
//  * bin_kernel: one workgroup per (event, layer) slice; places every hit on its
//    (aligned) layer and counting-sorts it into n_phi x n_z bins in LDS, writing the
//    binned records range by range from an LDS staging area.  Binned
//    records are (x, y, z, phi about the layer axis) plus the caller's hit index; the
//    same records are also written in the caller's hit order, so that a hit known by
//    its index is one 16-byte load away.
//  * find_kernel: persistent one-wave workgroups pull tiles of 64 / G seeds from a
//    counter.  A seed owns a group of G lanes (G = 4, 6 or 8); lane k holds candidate k
//    (state in registers).
//    Per layer every live candidate predicts, parks its predicted covariance in LDS,
//    scans the bins its window overlaps keeping its best hit branches in registers,
//    the group merges all branches with min-reductions of 64-bit score keys over DPP
//    lane exchanges, and each surviving slot pulls its parent's predicted state (the
//    covariance from LDS, the rest by lane shuffles) and applies its update.
//    Backpointers (parent slot and hit, one dword per layer and slot) go to a small
//    per-workgroup buffer in global memory; candidates' hit lists are rebuilt from
//    them at the end of the tile.
#include <atomic>
#include <type_traits>

#include "kf_internal.h"

namespace kfi {

namespace {

constexpr int kWave = 64;     // one wave per find workgroup
constexpr int kMaxList = 8;   // hit branches kept per candidate
// azimuth differences wrapped to (-pi, pi], or taken as they are
constexpr std::integral_constant<bool, true> kWrap{};
constexpr std::integral_constant<bool, false> kNoWrap{};
// A seed's candidates sit in a group of G consecutive lanes (G = 4, 6 or 8, >= keep);
// a wave holds kWave / G seeds (the tile) and leaves the kWave % G lanes after them idle.

// A candidate whose window overlaps more than FindArgs::wide_bins bins is scanned by
// its whole wave: the lanes read its window and the quantities its chi2 needs from
// the candidate's lane (readlane), split its hits, and their sorted lists are merged
// into the candidate's.

__device__ __forceinline__ int bin_index(float v, float lo, float scale, int nb) {
  const int b = (int)floorf((v - lo) * scale);
  return b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b);
}

}  // namespace

// The bin kernel: one workgroup of kBinThreads lanes per (event, layer) slice.  A slice
// of up to kBinThreads * kBinHold hits is sorted with its placed hits held in registers
// (lane t holds hits t, t + kBinThreads, ...): an LDS histogram, its scan, an LDS
// atomic per hit for its place, then the binned records are assembled range by range in
// LDS and written out contiguously, so that every global store is coalesced.  (Storing
// each record at its place directly scatters 16- and 4-byte writes over the slice's
// output; with a thousand slices in flight their cache lines leave the L2 part-written
// and the writes reach memory at 2.4 times their size.)  Larger slices take the direct
// scatter.
constexpr int kBinThreads = 1024;
constexpr int kBinHold = 24;
constexpr int kBinWaves = kBinThreads / 64;
constexpr int kBinStaticLds = 256;  // the static LDS (the waves' scan totals), rounded up

__global__ __launch_bounds__(kBinThreads) void bin_kernel(BinArgs a) {
  // LDS: [nbins + 1] counts, then running places; then each held hit's bin or place
  // (16 bits) and the staging of a range of binned hits (a.stage float4: position and
  // index in the slice)
  extern __shared__ __align__(16) unsigned char bin_lds[];
  int* const cnt = reinterpret_cast<int*>(bin_lds);
  __shared__ int wsum[kBinWaves];
  const int tid = threadIdx.x;
  const int seg = blockIdx.x;
  const int e = seg / a.nl, l = seg % a.nl;
  if (seg == 0 && tid == 0 && a.counter) *a.counter = 0;  // the find kernel's tile queue
  const int nb = a.nphi * a.nz;
  for (int b = tid; b <= nb; b += kBinThreads) cnt[b] = 0;
  __syncthreads();
  // slices outside [0, H] or reversed are clamped (never read out of bounds)
  int64_t beg = a.hit_off[(int64_t)e * (a.nl + 1) + l];
  int64_t end = a.hit_off[(int64_t)e * (a.nl + 1) + l + 1];
  beg = beg < 0 ? 0 : (beg > a.H ? a.H : beg);
  end = end < beg ? beg : (end > a.H ? a.H : end);
  const int n = (int)(end - beg);
  const kfd::LayerK ly =
      make_layer(l, a.radius, a.align, a.xX0, a.zhalf, a.mat_nz, a.sf.disk_z[l], a.sf.rmin[l], a.sf.rmax[l],
                 a.sf.zmax[l]);
  if (e == 0 && tid == 0) a.layers[l] = ly;
  // the bins' second coordinate: z over [-Z, Z] on a cylinder, rho over [lo, hi] on a disk
  const bool disk = ly.disk != 0.f;
  const float Z = a.zhalf[l];
  const float lo2 = disk ? ly.lo : -Z;
  const float sphi = a.nphi / kfd::kTwoPi, sz = a.nz / (disk ? ly.hi - ly.lo : 2.f * Z);
  auto azimuth = [&](float mx, float my) { return atan2f(my - ly.cy, mx - ly.cx); };
  auto bin_of = [&](float mx, float my, float mz, float ph) {
    const float ex = mx - ly.cx, ey = my - ly.cy;
    const float c2 = disk ? sqrtf(fmaf(ex, ex, ey * ey)) : mz;
    return bin_index(ph, -kfd::kPi, sphi, a.nphi) * a.nz + bin_index(c2, lo2, sz, a.nz);
  };
  auto scan = [&]() {  // cnt[b] <- the slice's exclusive prefix of the counts; boff written
    const int chunk = (nb + kBinThreads - 1) / kBinThreads;
    const int c0 = min(nb, tid * chunk), c1 = min(nb, c0 + chunk);
    int acc = 0;
    for (int b = c0; b < c1; ++b) acc += cnt[b];
    // the exclusive prefix of acc over the workgroup: an inclusive scan inside each wave
    // by lane shuffles, then one over the waves' totals (two barriers)
    const int lane = tid & 63, wid = tid >> 6;
    int v = acc;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(v, off, 64);
      if (lane >= off) v += t;
    }
    if (lane == 63) wsum[wid] = v;
    __syncthreads();
    if (wid == 0) {
      int w = lane < kBinWaves ? wsum[lane] : 0;
#pragma unroll
      for (int off = 1; off < kBinWaves; off <<= 1) {
        const int t = __shfl_up(w, off, 64);
        if (lane >= off) w += t;
      }
      if (lane < kBinWaves) wsum[lane] = w;
    }
    __syncthreads();
    int run = (wid > 0 ? wsum[wid - 1] : 0) + v - acc;
    int32_t* out_off = a.boff + ((int64_t)e * a.nl + l) * (nb + 1);
    for (int b = c0; b < c1; ++b) {
      const int c = cnt[b];
      cnt[b] = run;
      out_off[b] = (int)beg + run;
      run += c;
    }
    if (tid == 0) out_off[nb] = (int)end;
    __syncthreads();
  };
  if (n <= kBinThreads * kBinHold && a.stage > 0) {
    // each hit's bin, then its place in the slice, as 16 bits in LDS (both < 32 768)
    uint16_t* const sbin = reinterpret_cast<uint16_t*>(bin_lds + a.stage_off);
    float4* const srec = reinterpret_cast<float4*>(bin_lds + a.stage_off + a.hold_bytes);
    float px[kBinHold], py[kBinHold], pz[kBinHold];
#pragma unroll
    for (int r = 0; r < kBinHold; ++r) {
      const int q = tid + r * kBinThreads;
      if (q < n) {
        const int64_t j = beg + q;
        kfd::place(ly, a.hits[j], a.hits[a.H + j], a.hits[2 * a.H + j], px[r], py[r], pz[r]);
        const float ph = azimuth(px[r], py[r]);
        a.hpos[j] = make_float4(px[r], py[r], pz[r], ph);
        const int b = bin_of(px[r], py[r], pz[r], ph);
        sbin[q] = (uint16_t)b;
        atomicAdd(&cnt[b], 1);
      }
    }
    __syncthreads();
    scan();
    for (int q = tid; q < n; q += kBinThreads) sbin[q] = (uint16_t)atomicAdd(&cnt[sbin[q]], 1);
    // staged: the placed position and the hit's index in the slice; the azimuth is
    // evaluated again by the lane that writes the record out (the same function of the
    // same values)
    for (int p0 = 0; p0 < n; p0 += a.stage) {
      __syncthreads();  // the places are in; the previous range has been written out
#pragma unroll
      for (int r = 0; r < kBinHold; ++r) {
        const int q = tid + r * kBinThreads;
        if (q < n) {
          const int d = (int)sbin[q] - p0;
          if (d >= 0 && d < a.stage) srec[d] = make_float4(px[r], py[r], pz[r], __int_as_float(q));
        }
      }
      __syncthreads();
      const int m = min(a.stage, n - p0);
      for (int d = tid; d < m; d += kBinThreads) {
        const float4 h = srec[d];
        a.brec[beg + p0 + d] = make_float4(h.x, h.y, h.z, azimuth(h.x, h.y));
        a.bidx[beg + p0 + d] = (int32_t)beg + __float_as_int(h.w);
      }
    }
    return;
  }
  // direct scatter: each hit is placed and binned twice (count, then store)
  for (int64_t j = beg + tid; j < end; j += kBinThreads) {
    float mx, my, mz;
    kfd::place(ly, a.hits[j], a.hits[a.H + j], a.hits[2 * a.H + j], mx, my, mz);
    atomicAdd(&cnt[bin_of(mx, my, mz, azimuth(mx, my))], 1);
  }
  __syncthreads();
  scan();
  for (int64_t j = beg + tid; j < end; j += kBinThreads) {
    float mx, my, mz;
    kfd::place(ly, a.hits[j], a.hits[a.H + j], a.hits[2 * a.H + j], mx, my, mz);
    const float ph = azimuth(mx, my);
    const float4 rec = make_float4(mx, my, mz, ph);
    const int p = (int)beg + atomicAdd(&cnt[bin_of(mx, my, mz, ph)], 1);
    a.brec[p] = rec;
    a.bidx[p] = (int32_t)j;
    a.hpos[j] = rec;
  }
}

namespace {

enum : int { EMPTY = 0, LIVE = 1, TERM = 2 };
enum : int { K_NONE = 0, K_HIT = 1, K_MISS = 2, K_CARRY = 3 };

__device__ __forceinline__ bool key_lt(float c1, int h1, float c2, int h2) { return c1 < c2 || (c1 == c2 && h1 < h2); }

__device__ __forceinline__ float shfl_f(float v, int src) { return __shfl(v, src, 64); }

template <int kCtrl>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, 0xF, 0xF, false);
}

// (hi, lo) <- the minimum of the 64-bit key over the lane's 8-lane group: xor 1 and
// xor 2 inside each quad (quad_perm), then the mirrored lane of the other quad of the
// half row (row_half_mirror).  Every lane of the group must be active.
__device__ __forceinline__ void min_step(uint32_t& hi, uint32_t& lo, uint32_t ohi, uint32_t olo) {
  const bool lt = ohi < hi || (ohi == hi && olo < lo);
  hi = lt ? ohi : hi;
  lo = lt ? olo : lo;
}
// The minimum over the lane's G-lane group.  G = 8: xor 1 and xor 2 inside each quad
// (quad_perm), then the mirrored lane of the other quad of the half row
// (row_half_mirror); G = 4: the two quad steps.  Other G (<= 8): rotations by 1, 2 and 4
// inside the group by lane shuffles, which together cover every lane of it; the idle
// lanes after the last group of a wave keep their own key.
template <int G>
__device__ __forceinline__ void group_min(uint32_t& hi, uint32_t& lo, int gbase, int slot) {
  if constexpr (G == 8) {
    min_step(hi, lo, dpp<0xB1>(hi), dpp<0xB1>(lo));
    min_step(hi, lo, dpp<0x4E>(hi), dpp<0x4E>(lo));
    min_step(hi, lo, dpp<0x141>(hi), dpp<0x141>(lo));
  } else if constexpr (G == 4) {
    min_step(hi, lo, dpp<0xB1>(hi), dpp<0xB1>(lo));
    min_step(hi, lo, dpp<0x4E>(hi), dpp<0x4E>(lo));
  } else {
    const bool whole = gbase + G <= kWave;
#pragma unroll
    for (int d = 1; d < 8; d <<= 1) {
      const int src = whole ? gbase + (slot + d) % G : gbase + slot;
      const uint32_t ohi = (uint32_t)__shfl((int)hi, src, kWave);
      const uint32_t olo = (uint32_t)__shfl((int)lo, src, kWave);
      min_step(hi, lo, ohi, olo);
    }
  }
}
__device__ __forceinline__ int shfl_i(int v, int src) { return __shfl(v, src, 64); }

}  // namespace

// kVar (a Variant): the detector model (material map, energy loss, parameterised field)
// in every prediction, as the fit's model variant takes it; or bounded surfaces: a
// candidate that misses a disk or a bounded cylinder (or meets it outside its active
// area) passes it over, and a disk's window runs over (phi, rho) of its plane; or
// neither.
template <int kVar, int G>
__global__ __launch_bounds__(kWave, 4) void find_kernel(FindArgs a) {
  constexpr bool kModel = kVar == kModelV;
  constexpr bool kBounded = kVar == kBoundedV;
  constexpr int kTileSeeds = kWave / G;
  // at most G branches of one parent can survive (keep <= G), so a candidate keeps its
  // best G hit branches
  constexpr int kList = G;
  // LDS: the predicted covariance of every lane, sC [21][64] (a survivor reads its
  // parent's), and branch lists saved around wide-window scans (chi2 [8][64], hit
  // [8][64], count [64]).
  extern __shared__ __align__(16) unsigned char lds[];
  float* const sC = reinterpret_cast<float*>(lds);
  float* const stc = sC + 21 * kWave;
  int32_t* const sti = reinterpret_cast<int32_t*>(stc + kMaxList * kWave);
  int32_t* const stn = sti + kMaxList * kWave;
  const int lane = threadIdx.x;
  const int slot = lane % G;
  const int grp = lane / G;
  const int gbase = grp * G;
  const int nl = a.nl;
  const int64_t S = a.n_seeds;
  const int nb_all = a.nphi * a.nz;
  const float kphi = a.nphi / kfd::kTwoPi;
  // backpointers of this workgroup's tile, [nl][64]: ((hit + 2) << 3) | parent slot;
  // with a refit, the placed hit of each (layer, lane) that took one, [nl][3][64]
  int32_t* const bp = a.bp + (int64_t)blockIdx.x * nl * kWave;
  float* const bpos = a.bpos ? a.bpos + (int64_t)blockIdx.x * nl * 3 * kWave : nullptr;
  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  for (;;) {
    int claim = 0;
    if (lane == 0) claim = atomicAdd(a.counter, 1);
    const int64_t tile = __builtin_amdgcn_readfirstlane(claim);
    if (tile >= a.n_tiles) break;
    const int64_t s = tile * kTileSeeds + grp;
    const bool active = grp < kTileSeeds && s < S;
    // ---------------- seed and its refit over hits 0..2 ----------------
    kfd::Trk k;
    float c2 = 0.f;
    int nh = 0, nm = 0, mode = EMPTY;
    uint32_t st = 0;
    int e = 0;
    int sh[3] = {0, 0, 0};
    bool bad = false;
    if (active) {
      e = a.seed_event[s];
#pragma unroll
      for (int q = 0; q < 3; ++q) sh[q] = a.seed_hits[q * S + s];
      bad = e < 0 || e >= a.n_events;
      // hit q must lie in its event's slice of layer q (clamped to the hit array)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        int64_t lo = bad ? 0 : a.hit_off[(int64_t)e * (nl + 1) + q];
        int64_t hi = bad ? 0 : a.hit_off[(int64_t)e * (nl + 1) + q + 1];
        lo = lo < 0 ? 0 : (lo > a.H ? a.H : lo);
        hi = hi < lo ? lo : (hi > a.H ? a.H : hi);
        bad = bad || (int64_t)sh[q] < lo || (int64_t)sh[q] >= hi;
      }
      if (bad) {
        e = 0;
        sh[0] = sh[1] = sh[2] = 0;
      }
    }
    if (active && !bad) {
      float m[3][3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float4 h = a.hpos[sh[q]];  // placed on its layer by the binning
        m[q][0] = h.x;
        m[q][1] = h.y;
        m[q][2] = h.z;
      }
      if (bpos) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
          for (int c = 0; c < 3; ++c) bpos[(q * 3 + c) * kWave + lane] = m[q][c];
      }
      kfd::Model md0 = a.md;
      if (kModel) md0.kB = kfd::field_kB(a.md.kB, a.fr, a.fz, m[0][0], m[0][1], m[0][2]);  // kappa at hit 0
      kfd::seed_from_three(k, md0, m[0][0], m[0][1], m[0][2], m[1][0], m[1][1], m[2][0], m[2][1], m[2][2],
                           a.srphi, a.sz);
      kfd::init_trig(k);
      bool ok = true;
      for (int q = 0; q < 3 && ok; ++q) {
        const kfd::LayerK ly = a.layers[q];
        if (q > 0) {
          const float kB =
              kModel ? kfd::field_kB(a.md.kB, a.fr, a.fz, k.x[0] + k.xl[0], k.x[1] + k.xl[1], k.x[2]) : a.md.kB;
          kfd::Step stp;
          ok = kfd::crossing(k, ly, kB, stp);
          if (!ok) {
            st |= kfd::ST_PROP_FAIL;
            break;
          }
          kfd::transport(k, stp, kB);
        }
        const kfd::Frame f = kfd::frame_at(k, ly);
        if (kModel) {
          if (fabsf(f.cosa) < 0.3f) st |= kfd::ST_NEAR_TANGENT;
          if (q > 0 && !kfd::apply_material(k, f, ly, a.mat_map ? a.mat_map + q * a.mat_nz : nullptr, a.mat_nz,
                                            a.eloss, a.md.mass2)) {
            ok = false;
            st |= kfd::ST_PROP_FAIL;
            break;
          }
        } else {
          if (q > 0 && ly.xX0 > 0.f) kfd::add_scattering(k, f, ly.xX0, a.md.mass2);
          if (fabsf(f.cosa) < 0.3f) st |= kfd::ST_NEAR_TANGENT;
        }
        kfd::Pred p;
        kfd::prepare(k, f, a.md, p);
        if (p.fp64) st |= kfd::ST_FP64;
        const kfd::Resid r = kfd::residual(k, f, ly, p, m[q][0], m[q][1], m[q][2]);
        kfd::apply_update(k, p, a.md, r.r1, r.r2);
        c2 += r.chi2;
        ++nh;
      }
      mode = slot == 0 ? (ok ? LIVE : TERM) : EMPTY;
    }
    int ncand = active && !bad ? 1 : 0;
    // ---------------- layers 3 .. L-1 ----------------
    for (int l = 3; l < nl; ++l) {
      const kfd::LayerK ly = a.layers[l];
      const bool disk = kBounded && ly.disk != 0.f;
      float bc[kList];
      int bi[kList];
#pragma unroll
      for (int q = 0; q < kList; ++q) {
        bc[q] = INFINITY;
        bi[q] = 0x7fffffff;
      }
      int nlist = 0;
      bool predicted = false;
      bool passed = false;  // a bounded surface this live candidate passes over
      bool wide = false;
      // the prediction's window and what its chi2 needs (read by the wave for a wide
      // window)
      float phip = 0.f, zp = 0.f, wphi = 0.f, wz = 0.f;
      int blo = 0, bhi = -1, zlo = 0, zhi = -1;
      kfd::Frame f;
      f.rho = f.rx = f.ry = 0.f;
      f.cosa = f.ica = f.icpsi = 1.f;
      kfd::Pred p;
      p.Si00 = p.Si11 = p.Si12 = p.Si22 = 0.f;
      p.fp64 = false;
      p.dSi11 = p.dSi12 = p.dSi22 = 0.0;
      // One hit of the window (binned record and hit index): rectangle test, chi2 with
      // the candidate's S^-1, and the sorted insertion of a passing branch into (bc, bi).  Slot t keeps its entry if
      // that entry precedes the new one, takes the new one if only the entry before it
      // does, and otherwise takes the entry before it: one select per slot, no element
      // moves under a lane mask (register-pair copies followed by a partial overwrite
      // of the same pair have lost the new element on gfx950).
      auto in_window = [&](const float4 rec, float php, float zpp, float wph, float wzz, auto wrap)
                           __attribute__((always_inline)) {
        float dphi = rec.w - php;
        if constexpr (decltype(wrap)::value) dphi = kfd::wrap_pi(dphi);
        float dz;
        if (disk) {  // the window's second coordinate: the hit's radius about the axis
          const float ex = rec.x - ly.cx, ey = rec.y - ly.cy;
          dz = sqrtf(fmaf(ex, ex, ey * ey)) - zpp;
        } else {
          dz = rec.z - zpp;
        }
        return fabsf(dphi) <= wph && fabsf(dz) <= wzz;
      };
      auto consider = [&](const float4 rec, int hh, const kfd::Trk& kk, const kfd::Frame& ff, const kfd::Pred& pp,
                          float php, float zpp, float wph, float wzz, float cbase) __attribute__((always_inline)) {
        if (!in_window(rec, php, zpp, wph, wzz, kWrap)) return;
        const kfd::Resid r = kfd::residual(kk, ff, ly, pp, rec.x, rec.y, rec.z, disk);
        if (!(r.chi2 < a.chi2_cut)) return;
        const float cc = cbase + r.chi2;
        bool prev_lt = true;
        float oc = 0.f;
        int oh = 0;
#pragma unroll
        for (int t = 0; t < kList; ++t) {
          const bool lt = t < nlist && key_lt(bc[t], bi[t], cc, hh);
          const float ct = bc[t];
          const int ht = bi[t];
          bc[t] = lt ? ct : (prev_lt ? cc : oc);
          bi[t] = lt ? ht : (prev_lt ? hh : oh);
          prev_lt = lt;
          oc = ct;
          oh = ht;
        }
        nlist = nlist < kList ? nlist + 1 : kList;
      };
      if (mode == LIVE) {
        const float kB =
            kModel ? kfd::field_kB(a.md.kB, a.fr, a.fz, k.x[0] + k.xl[0], k.x[1] + k.xl[1], k.x[2]) : a.md.kB;
        kfd::Step stp;
        bool reach;
        if (kBounded) {
          reach = disk ? kfd::plane_crossing(k, ly, kB, stp) : kfd::crossing(k, ly, kB, stp);
          if (ly.bounded != 0.f) {  // missed, or met outside the active area: passed over
            if (reach) reach = kfd::in_area(k, ly, stp, disk);
            passed = !reach;
          }
        } else {
          reach = kfd::crossing(k, ly, kB, stp);
        }
        if (reach) {
          kfd::transport(k, stp, kB);
          if (disk) k.x[2] = ly.zp;
          f = kfd::frame_at(k, ly, disk);
          if (fabsf(f.cosa) < 0.3f) st |= kfd::ST_NEAR_TANGENT;
          if (kModel)  // a particle that stops in the layer's material ends there, transported
            reach = kfd::apply_material(k, f, ly, a.mat_map ? a.mat_map + l * a.mat_nz : nullptr, a.mat_nz, a.eloss,
                                        a.md.mass2);
          else if (ly.xX0 > 0.f)
            kfd::add_scattering(k, f, ly.xX0, a.md.mass2);
        }
        if (reach) {
          predicted = true;
          kfd::prepare(k, f, a.md, p, disk);
          phip = atan2f(f.ry, f.rx);
          zp = disk ? f.rho : k.x[2] + k.xl[2];
          wphi = a.nsigma * sqrtf(p.S11) / f.rho;
          wz = a.nsigma * sqrtf(p.S22);
          const float Z = a.zhalf[l];
          const float lo2 = disk ? ly.lo : -Z;
          const float kz = a.nz / (disk ? ly.hi - ly.lo : 2.f * Z);
          const float zq = fmaf(wz, 1e-4f, wz) + 1e-6f;
          zlo = bin_index(zp - zq, lo2, kz, a.nz);
          zhi = bin_index(zp + zq, lo2, kz, a.nz);
          const float wq = fmaf(wphi, 1e-4f, wphi) + 1e-6f;
          blo = 0;
          bhi = a.nphi - 1;
          if (wq < kfd::kPi) {
            blo = (int)floorf((phip - wq + kfd::kPi) * kphi);
            bhi = (int)floorf((phip + wq + kfd::kPi) * kphi);
            if (bhi - blo + 1 >= a.nphi) {
              blo = 0;
              bhi = a.nphi - 1;
            }
          }
          wide = (bhi - blo + 1) * (zhi - zlo + 1) > a.wide_bins;
        } else if (!passed) {
          mode = TERM;
          st |= kfd::ST_PROP_FAIL;
        }
      }
      // every lane parks its (predicted, or carried) covariance for its children
#pragma unroll
      for (int q = 0; q < 21; ++q) sC[q * kWave + lane] = k.C[q];
      if (predicted && !wide) {
        // Two passes.  The window's records are tested against the rectangle alone, and
        // the places of the first kMaxList - 1 that pass go to this lane's column of the
        // LDS list area (unused until the wide-window scans); then only those are
        // evaluated (chi2 and insertion, whose result does not depend on the order).
        // Most records fail the rectangle, and the lanes of a wave scan windows of
        // different sizes, so the costly part no longer runs once per record of the
        // wave's largest window.  A lane with more passing records than that (rare)
        // evaluates its whole window.  (The places are kept as the bits of floats: the
        // area is float-typed.)
        // The first pass needs only to keep a superset of the window: it compares a
        // record's azimuth with the prediction's shifted by 2 pi where the bin lies
        // across the -pi/pi seam (no wrap per record), with a margin for the rounding
        // of that shift; the second pass applies the exact test.  A window within two
        // bins of the whole ring keeps every azimuth.  Every record's place is written,
        // branch-free, into the next free row, and only a passing one advances it: the
        // last of the kMaxList rows is that spare once kMaxList - 1 are kept.
        const float wph1 = wphi < kfd::kPi - 2.f / kphi ? wphi + 4e-6f : INFINITY;
        const int32_t* boff = a.boff + ((int64_t)e * nl + l) * (nb_all + 1);
        int npass = 0;
        auto keep_place = [&](int q, bool pass) __attribute__((always_inline)) {
          stc[min(npass, kMaxList - 1) * kWave + lane] = __int_as_float(q);
          npass += pass ? 1 : 0;
        };
        auto place_at = [&](int t) __attribute__((always_inline)) { return __float_as_int(stc[t * kWave + lane]); };
        for (int b = blo; b <= bhi; ++b) {
          const int pb = b < 0 ? b + a.nphi : (b >= a.nphi ? b - a.nphi : b);
          const float phb = b < 0 ? phip + kfd::kTwoPi : (b >= a.nphi ? phip - kfd::kTwoPi : phip);
          const int q0 = boff[pb * a.nz + zlo], q1 = boff[pb * a.nz + zhi + 1];
          int q = q0;
          if (!kBounded) {
            // on a cylinder the rectangle needs a record's (z, phi) half only: four of
            // them in flight per iteration (record q's half is zw[2 q])
            const float2* const zw = reinterpret_cast<const float2*>(a.brec) + 1;
            auto in_zw = [&](const float2 r) __attribute__((always_inline)) {
              return in_window(make_float4(0.f, 0.f, r.x, r.y), phb, zp, wph1, wz, kNoWrap);
            };
            for (; q + 3 < q1; q += 4) {
              const float2 r0 = zw[2 * (int64_t)q], r1 = zw[2 * (int64_t)q + 2], r2 = zw[2 * (int64_t)q + 4],
                           r3 = zw[2 * (int64_t)q + 6];
              keep_place(q, in_zw(r0));
              keep_place(q + 1, in_zw(r1));
              keep_place(q + 2, in_zw(r2));
              keep_place(q + 3, in_zw(r3));
            }
          }
          // two records in flight per iteration
          for (; q + 1 < q1; q += 2) {
            const float4 r0 = a.brec[q], r1 = a.brec[q + 1];
            keep_place(q, in_window(r0, phb, zp, wph1, wz, kNoWrap));
            keep_place(q + 1, in_window(r1, phb, zp, wph1, wz, kNoWrap));
          }
          if (q < q1) keep_place(q, in_window(a.brec[q], phb, zp, wph1, wz, kNoWrap));
        }
        if (npass < kMaxList) {
          int t = 0;
          for (; t + 1 < npass; t += 2) {
            const int qa = place_at(t), qb = place_at(t + 1);
            const float4 ra = a.brec[qa], rb = a.brec[qb];
            const int ha = a.bidx[qa], hb = a.bidx[qb];
            consider(ra, ha, k, f, p, phip, zp, wphi, wz, c2);
            consider(rb, hb, k, f, p, phip, zp, wphi, wz, c2);
          }
          if (t < npass) {
            const int qa = place_at(t);
            consider(a.brec[qa], a.bidx[qa], k, f, p, phip, zp, wphi, wz, c2);
          }
        } else {
          for (int b = blo; b <= bhi; ++b) {
            const int pb = b < 0 ? b + a.nphi : (b >= a.nphi ? b - a.nphi : b);
            const int q0 = boff[pb * a.nz + zlo], q1 = boff[pb * a.nz + zhi + 1];
            for (int q = q0; q < q1; ++q) consider(a.brec[q], a.bidx[q], k, f, p, phip, zp, wphi, wz, c2);
          }
        }
      }
      // ---- wide windows: each is scanned by the whole wave ----
      unsigned long long wide_m = __ballot(wide);
      if (wide_m != 0ull) {
#pragma unroll
        for (int t = 0; t < kList; ++t) {
          stc[t * kWave + lane] = bc[t];
          sti[t * kWave + lane] = bi[t];
        }
        stn[lane] = nlist;
        wave_sync();
        while (wide_m != 0ull) {
          const int c = __ffsll((unsigned long long)wide_m) - 1;
          wide_m &= wide_m - 1ull;
          auto rdf = [c](float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), c)); };
          auto rdi = [c](int v) { return __builtin_amdgcn_readlane(v, c); };
          auto rdd = [c](double v) {
            const uint64_t u = __double_as_longlong(v);
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, c);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), c);
            return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
          };
          kfd::Trk kc;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            kc.x[q] = rdf(k.x[q]);
            kc.xl[q] = rdf(k.xl[q]);
          }
          kfd::Frame fc;
          fc.rho = rdf(f.rho);
          fc.rx = rdf(f.rx);
          fc.ry = rdf(f.ry);
          fc.cosa = fc.ica = fc.icpsi = 1.f;
          kfd::Pred pc;
          pc.Si00 = rdf(p.Si00);
          pc.Si11 = rdf(p.Si11);
          pc.Si12 = rdf(p.Si12);
          pc.Si22 = rdf(p.Si22);
          pc.fp64 = rdi(p.fp64 ? 1 : 0) != 0;
          pc.dSi11 = rdd(p.dSi11);
          pc.dSi12 = rdd(p.dSi12);
          pc.dSi22 = rdd(p.dSi22);
          const float wphip = rdf(phip), wzp = rdf(zp), wwphi = rdf(wphi), wwz = rdf(wz), wc2 = rdf(c2);
          const int wblo = rdi(blo), wbhi = rdi(bhi), wzlo = rdi(zlo), wzhi = rdi(zhi), we = rdi(e);
#pragma unroll
          for (int t = 0; t < kList; ++t) {
            bc[t] = INFINITY;
            bi[t] = 0x7fffffff;
          }
          nlist = 0;
          const int32_t* boff = a.boff + ((int64_t)we * nl + l) * (nb_all + 1);
          for (int b = wblo; b <= wbhi; ++b) {
            const int pb = b < 0 ? b + a.nphi : (b >= a.nphi ? b - a.nphi : b);
            const int q0 = boff[pb * a.nz + wzlo], q1 = boff[pb * a.nz + wzhi + 1];
            for (int q = q0 + lane; q < q1; q += kWave)
              consider(a.brec[q], a.bidx[q], kc, fc, pc, wphip, wzp, wwphi, wwz, wc2);
          }
          // the candidate's list: kList rounds of a 64-lane min over (chi2, hit) keys
          int hd = 0, cnt = 0;
          for (int r = 0; r < kList; ++r) {
            float hc = bc[0];
            int hx = bi[0];
#pragma unroll
            for (int t = 1; t < kList; ++t) {
              if (hd == t) {
                hc = bc[t];
                hx = bi[t];
              }
            }
            const bool has = hd < nlist;
            const uint32_t mhi = has ? __float_as_uint(hc) : 0xffffffffu;
            const uint32_t mlo = has ? (uint32_t)hx : 0xffffffffu;
            const unsigned long long mine = ((unsigned long long)mhi << 32) | mlo;
            unsigned long long key = mine;
#pragma unroll
            for (int m = 1; m < 64; m <<= 1) {
              const unsigned long long o = __shfl_xor(key, m, 64);
              key = o < key ? o : key;
            }
            if (key == ~0ull) break;
            if (mine == key) ++hd;
            if (lane == c) {
              stc[r * kWave + lane] = __uint_as_float((uint32_t)(key >> 32));
              sti[r * kWave + lane] = (int32_t)(uint32_t)(key & 0xffffffffull);
            }
            ++cnt;
          }
          if (lane == c) stn[lane] = cnt;
        }
        wave_sync();
#pragma unroll
        for (int t = 0; t < kList; ++t) {
          bc[t] = stc[t * kWave + lane];
          bi[t] = sti[t * kWave + lane];
        }
        nlist = stn[lane];
      }
      // ---- merge the group's branches: `keep` rounds of an 8-lane minimum ----
      // Each lane offers its best remaining branch as a 64-bit key: more hits, smaller
      // total chi2, lower parent slot, with the branch kind in the two lowest bits (a
      // lane offers one branch per round, so the kind never decides).  The minimum over
      // the 8 lanes of a seed takes three DPP exchanges.  The key names the winner's
      // slot, kind and total chi2; the slot that the round fills takes the winner's hit
      // index by one lane shuffle.  The list is never shifted: its head is an index
      // resolved by a chain of selects.
      bool other_used = false;   // the miss (live) or carry (terminated) branch was taken
      int head = 0;
      int my_par = slot, my_kind = K_NONE, my_hit = -2;
      float my_c = 0.f;
      int new_n = 0;
      for (int r = 0; r < a.keep; ++r) {
        int hk = K_NONE, hn = 0;
        float hc = bc[0];
        int hx = bi[0];
#pragma unroll
        for (int t = 1; t < kList; ++t)
          if (head == t) {
            hc = bc[t];
            hx = bi[t];
          }
        if (head < nlist) {
          hk = K_HIT;
          hn = nh + 1;
        } else if (!other_used && mode == LIVE && predicted) {
          hk = K_MISS;
          hc = c2;
          hn = nh;
        } else if (!other_used && (mode == TERM || passed)) {
          hk = K_CARRY;
          hc = c2;
          hn = nh;
        }
        const bool has = hk != K_NONE;
        uint32_t khi = has ? ((uint32_t)(255 - hn) << 8) | (__float_as_uint(hc) >> 24) : 0xffffffffu;
        uint32_t klo = has ? (__float_as_uint(hc) << 8) | ((uint32_t)slot << 2) | (uint32_t)hk : 0xffffffffu;
        group_min<G>(khi, klo, gbase, slot);
        if (khi == 0xffffffffu && klo == 0xffffffffu) break;
        const int w = (int)((klo >> 2) & 7u);
        const int wk = (int)(klo & 3u);
        const int whit = shfl_i(hx, gbase + w);
        if (slot == r) {
          my_par = w;
          my_kind = wk;
          my_c = __uint_as_float((khi << 24) | (klo >> 8));
          my_hit = whit;
        }
        if (slot == w) {
          if (hk == K_HIT) ++head;
          else other_used = true;
        }
        ++new_n;
      }
      // ---- every surviving slot takes its parent's (predicted) candidate ----
      // (a hit branch's placed position is loaded first, so that its latency hides
      // behind the exchange of the parent's state)
      float4 hwin = make_float4(0.f, 0.f, 0.f, 0.f);
      if (active && slot < new_n && my_kind == K_HIT) hwin = a.hpos[my_hit];
      const int src = gbase + my_par;
      wave_sync();
#pragma unroll
      for (int q = 0; q < 21; ++q) k.C[q] = sC[q * kWave + src];
#pragma unroll
      for (int q = 0; q < 6; ++q) k.x[q] = shfl_f(k.x[q], src);
#pragma unroll
      for (int q = 0; q < 2; ++q) k.xl[q] = shfl_f(k.xl[q], src);  // xl[2] is always 0
      k.cp = shfl_f(k.cp, src);
      k.sp = shfl_f(k.sp, src);
      k.ct = shfl_f(k.ct, src);
      k.st = shfl_f(k.st, src);
      k.rst = shfl_f(k.rst, src);
      c2 = shfl_f(c2, src);
      nh = shfl_i(nh, src);
      nm = shfl_i(nm, src);
      mode = shfl_i(mode, src);
      st = (uint32_t)shfl_i((int)st, src);
      wave_sync();  // every lane has read sC before the next layer overwrites it
      if (active) {
        if (slot < new_n) {
          if (my_kind == K_HIT) {
            const kfd::Frame fu = kfd::frame_at(k, ly, disk);
            if (fabsf(fu.cosa) < 0.3f) st |= kfd::ST_NEAR_TANGENT;
            kfd::Pred pu;
            kfd::prepare(k, fu, a.md, pu, disk);
            if (pu.fp64) st |= kfd::ST_FP64;
            const float mx = hwin.x, my = hwin.y, mz = hwin.z;  // placed on its layer by the binning
            if (bpos) {
              bpos[(l * 3 + 0) * kWave + lane] = mx;
              bpos[(l * 3 + 1) * kWave + lane] = my;
              bpos[(l * 3 + 2) * kWave + lane] = mz;
            }
            const kfd::Resid r = kfd::residual(k, fu, ly, pu, mx, my, mz, disk);
            kfd::apply_update(k, pu, a.md, r.r1, r.r2, disk);
            c2 = my_c;
            nh += 1;
          } else if (my_kind == K_MISS) {
            nm += 1;
            my_hit = -1;
            if (nm >= a.max_miss) {
              mode = TERM;
              st |= kfd::ST_TERM_MISSES;
            }
          } else {
            my_hit = -2;
          }
          bp[l * kWave + lane] = ((my_hit + 2) << 3) | my_par;
        } else {
          mode = EMPTY;
        }
      }
      ncand = new_n;
    }
    // the tile's backpointers, written by the lanes of this wave, are read back below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    // ---------------- outputs ----------------
    // The output rows' strides are rebuilt here from an opaque copy of the seed count,
    // so that the compiler does not keep ~30 precomputed row addresses live through the
    // whole tile loop.
    int64_t So = S;
    asm volatile("" : "+s"(So));
    const bool writer = active && slot < a.keep;
    const bool have = writer && slot < ncand;
    const bool rank0 = writer && slot == 0 && bpos != nullptr;
    // The candidates' hit lists, from the last layer down: every lane loads its own
    // backpointers (and placed hits) of eight layers at once, and each candidate follows
    // its chain of ancestors by lane shuffles within its group, so that the walk waits
    // on memory once per eight layers rather than once per layer.  All lanes take part
    // in the shuffles; only the writers store.
    {
      int cur = slot;
      uint32_t rmask = 0;
      for (int l0 = nl - 1; l0 >= 0; l0 -= 8) {
        int v[8];
        float px[8], py[8], pz[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int l = l0 - j;
          v[j] = l >= 3 ? bp[l * kWave + lane] : 0;
          if (bpos && l >= 0) {
            px[j] = bpos[(l * 3 + 0) * kWave + lane];
            py[j] = bpos[(l * 3 + 1) * kWave + lane];
            pz[j] = bpos[(l * 3 + 2) * kWave + lane];
          } else {
            px[j] = py[j] = pz[j] = 0.f;
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int l = l0 - j;
          if (l < 0) break;
          const int at_lane = gbase + cur;  // the lane of this candidate's ancestor on layer l
          const int vv = shfl_i(v[j], at_lane);
          int h = -2;
          if (have) {
            if (l >= 3) {
              h = (vv >> 3) - 2;
              cur = vv & 7;
            } else {
              h = sh[l];
            }
          }
          if (writer) a.hit_idx[((int64_t)slot * nl + l) * So + s] = h;
          if (bpos) {
            const float qx = shfl_f(px[j], at_lane), qy = shfl_f(py[j], at_lane), qz = shfl_f(pz[j], at_lane);
            if (rank0 && h >= 0) {  // the rank-0 candidate's placed hits, for the refit
              a.rpos[((int64_t)l * 3 + 0) * So + s] = qx;
              a.rpos[((int64_t)l * 3 + 1) * So + s] = qy;
              a.rpos[((int64_t)l * 3 + 2) * So + s] = qz;
              rmask |= 1u << l;
            }
          }
        }
      }
      if (rank0) a.rmask[s] = rmask;
    }
    if (active) {
      const int keep = a.keep;
      if (slot < keep) {
        auto at = [&](int kk, int64_t inner) { return ((int64_t)kk * inner) * So + s; };
        a.n_hits[at(slot, 1)] = have ? nh : 0;
        a.n_miss[at(slot, 1)] = have ? nm : 0;
        a.chi2[at(slot, 1)] = have ? c2 : 0.f;
        a.status[at(slot, 1)] = have ? st : 0u;
#pragma unroll
        for (int q = 0; q < 6; ++q)
          a.state[((int64_t)slot * 6 + q) * So + s] =
              have ? (q < 3 ? k.x[q] + k.xl[q] : (q == 4 ? kfd::wrap_pi(k.x[q]) : k.x[q])) : 0.f;
#pragma unroll
        for (int q = 0; q < 21; ++q) a.cov[((int64_t)slot * 21 + q) * So + s] = have ? k.C[q] : 0.f;
      }
      if (slot == 0) {
        a.n_cand[s] = ncand;
        if (bad) a.status[s] = kfd::ST_BAD_INPUT;
      }
    }
    // the next tile overwrites the backpointers only after every lane has read them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
}

namespace {
// dynamic LDS the bin kernel may take (its static part aside); set by prepare_bin,
// which contexts on several host threads may call
std::atomic<int> bin_lds_budget{0};
}  // namespace

hipError_t prepare_bin(int nbins) {
  int dev = 0, per_block = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err == hipSuccess) err = hipDeviceGetAttribute(&per_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (err != hipSuccess) return err;
  const int budget = per_block - kBinStaticLds;
  if (budget < (nbins + 1) * (int)sizeof(int)) return hipErrorInvalidValue;
  err = hipFuncSetAttribute(reinterpret_cast<const void*>(bin_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            budget);
  if (err == hipSuccess) bin_lds_budget.store(budget, std::memory_order_relaxed);
  return err;
}

hipError_t launch_bin(BinArgs a, hipStream_t stream) {
  // the counts, the held hits' 16-bit bins or places, then as many staged hits (16
  // bytes) as the rest of the budget holds
  const int budget = bin_lds_budget.load(std::memory_order_relaxed);
  const int cnt_bytes = ((a.nphi * a.nz + 1) * (int)sizeof(int) + 15) & ~15;
  a.hold_bytes = kBinThreads * kBinHold * (int)sizeof(uint16_t);
  const int room = (budget - cnt_bytes - a.hold_bytes) / (int)sizeof(float4);
  a.stage_off = cnt_bytes;
  a.stage = room >= 256 ? room : 0;  // below that, the direct scatter
  const size_t lds = a.stage > 0 ? (size_t)budget : (size_t)cnt_bytes;
  hipLaunchKernelGGL(bin_kernel, dim3((unsigned)(a.n_events * a.nl)), dim3(kBinThreads), lds, stream, a);
  return hipGetLastError();
}

int find_tile_seeds(int lanes_per_seed) { return kWave / lanes_per_seed; }

size_t find_lds_bytes(int nl) {
  (void)nl;
  return (size_t)(21 + 2 * kMaxList + 1) * kWave * 4;
}

size_t find_bp_bytes(int nl, int64_t grid) { return (size_t)grid * nl * kWave * sizeof(int32_t); }

namespace {

template <int kVar, int G>
hipError_t max_blocks(int nl, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, find_kernel<kVar, G>, kWave,
                                                      find_lds_bytes(nl));
}

template <int kVar>
hipError_t max_blocks_group(int nl, int lanes_per_seed, int* blocks_per_cu) {
  if (lanes_per_seed == 4) return max_blocks<kVar, 4>(nl, blocks_per_cu);
  if (lanes_per_seed == 6) return max_blocks<kVar, 6>(nl, blocks_per_cu);
  return max_blocks<kVar, 8>(nl, blocks_per_cu);
}

template <int kVar, int G>
void launch_variant(const FindArgs& a, int grid, hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop) {
  const dim3 g((unsigned)grid), b(kWave);
  const size_t lds = find_lds_bytes(a.nl);
  if (ev_start && ev_stop)  // timing hook: the events bracket the kernel's own execution
    hipExtLaunchKernelGGL((find_kernel<kVar, G>), g, b, lds, stream, ev_start, ev_stop, 0, a);
  else
    hipLaunchKernelGGL((find_kernel<kVar, G>), g, b, lds, stream, a);
}

template <int kVar>
hipError_t launch_group(const FindArgs& a, int lanes_per_seed, int grid, hipStream_t stream, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
  if (lanes_per_seed == 4) launch_variant<kVar, 4>(a, grid, stream, ev_start, ev_stop);
  else if (lanes_per_seed == 6) launch_variant<kVar, 6>(a, grid, stream, ev_start, ev_stop);
  else launch_variant<kVar, 8>(a, grid, stream, ev_start, ev_stop);
  return hipGetLastError();
}

// The variant of a launch (the API refuses the detector model with bounded surfaces).
int find_variant(const FindArgs& a) {
  if (a.mat_map != nullptr || a.eloss > 0.f || a.fr != 0.f || a.fz != 0.f) return kModelV;
  return a.bounded ? kBoundedV : kPlain;
}

}  // namespace

hipError_t find_max_blocks(int nl, int variant, int lanes_per_seed, int* blocks_per_cu) {
  switch (variant) {
    case kModelV: return max_blocks_group<kModelV>(nl, lanes_per_seed, blocks_per_cu);
    case kBoundedV: return max_blocks_group<kBoundedV>(nl, lanes_per_seed, blocks_per_cu);
    default: return max_blocks_group<kPlain>(nl, lanes_per_seed, blocks_per_cu);
  }
}

hipError_t launch_find(const FindArgs& a, int lanes_per_seed, int grid, hipStream_t stream, hipEvent_t ev_start,
                       hipEvent_t ev_stop) {
  switch (find_variant(a)) {
    case kModelV: return launch_group<kModelV>(a, lanes_per_seed, grid, stream, ev_start, ev_stop);
    case kBoundedV: return launch_group<kBoundedV>(a, lanes_per_seed, grid, stream, ev_start, ev_stop);
    default: return launch_group<kPlain>(a, lanes_per_seed, grid, stream, ev_start, ev_stop);
  }
}

}  // namespace kfi
