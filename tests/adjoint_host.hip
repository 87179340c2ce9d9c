// Host-side FP64 instantiation of the library's fit adjoint (kf_adjoint.h), for the
// CPU test that checks the hand-derived reverse sweep against the oracle's forward-
// mode dual-number gradient.  Runs the same forward steps in double, checkpoints
// every layer, and accumulates sum_i w_i d chi2_i / d(align, xX0) in track order.
// fr, fz != 0: the parameterised field B (1 + fr r^2 + fz z^2), each step in the field
// at its start and the seed's curvature in the field at its first hit.
#include <vector>

#include "../paper_1906_11744_amd/csrc/kf_adjoint.h"

extern "C" int adjoint_host_fp64(int nl, const double* radius, double B, double srphi, double sz, double sr,
                                 double mass, const double* align, const double* xX0, long n, const float* hits,
                                 const uint32_t* mask, const double* w, double* g_align, double* g_xX0,
                                 double fr, double fz) {
  using T = double;
  kfa::Consts<T> k;
  k.kB = 0.299792458e-2 * B;
  k.v_r = sr * sr;
  k.v_rphi = srphi * srphi;
  k.v_z = sz * sz;
  k.mass2 = mass * mass;
  std::vector<kfa::Lay<T>> lays(nl);
  for (int l = 0; l < nl; ++l) {
    lays[l].r = radius[l];
    lays[l].cx = align[4 * l + 0];
    lays[l].cy = align[4 * l + 1];
    lays[l].dz = align[4 * l + 2];
    lays[l].cphi = std::cos(align[4 * l + 3]);
    lays[l].sphi = std::sin(align[4 * l + 3]);
    lays[l].xX0 = xX0[l];
    lays[l].pad = 0;
  }
  T Cs[21];
  kfa::seed_cov<T>(srphi, sz, radius[2] - radius[0], k.kB, Cs);
  const kfa::FieldK<T> fk{fr, fz, srphi, sz, radius[2] - radius[0]};
  const bool field = fr != 0.0 || fz != 0.0;
  std::vector<T> acc(nl * 5, 0.0);
  std::vector<T> ck(nl * 27);
  for (long i = 0; i < n; ++i) {
    const uint32_t m = mask[i];
    if ((m & 7u) != 7u) continue;
    auto hit = [&](int l, T h[3]) {
      for (int q = 0; q < 3; ++q) h[q] = hits[((long)l * 3 + q) * n + i];
    };
    // forward with checkpoints
    T hm[3][3], pm[3][3];
    for (int l = 0; l < 3; ++l) {
      hit(l, hm[l]);
      kfa::place(lays[l], hm[l][0], hm[l][1], hm[l][2], pm[l]);
    }
    kfa::Seed<T> E;
    T x[6], C[21];
    kfa::Consts<T> k0 = k;
    if (field) k0.kB = kfa::field_kB(k, fk, pm[0][0], pm[0][1], pm[0][2]);
    kfa::seed(pm[0], pm[1], pm[2], k0, E, x);
    kfa::seed_cov<T>(srphi, sz, radius[2] - radius[0], k0.kB, C);
    kfa::Upd<T> U;
    kfa::update(x, C, lays[0], k, pm[0][0], pm[0][1], pm[0][2], U);
    for (int q = 0; q < 6; ++q) ck[q] = x[q];
    for (int q = 0; q < 21; ++q) ck[6 + q] = C[q];
    int last = 31 - __builtin_clz(m);
    if (last > nl - 1) last = nl - 1;
    int lupd = 0;
    for (int l = 1; l <= last; ++l) {
      kfa::Consts<T> ks = k;
      if (field) ks.kB = kfa::field_kB(k, fk, x[0], x[1], x[2]);
      kfa::Prop<T> P;
      T xp[6];
      if (!kfa::propagate(x, lays[l], ks, P, xp)) break;
      T Bm[6][6], Cp[21];
      kfa::transport_cov(P, C, Bm, Cp);
      const kfa::Frm<T> fr = kfa::frame(xp, lays[l]);
      kfa::Scat<T> Q;
      kfa::scatter(xp, fr, lays[l], k, Q, Cp);
      for (int q = 0; q < 6; ++q) x[q] = xp[q];
      for (int q = 0; q < 21; ++q) C[q] = Cp[q];
      if ((m >> l) & 1u) {
        T h[3], pmh[3];
        hit(l, h);
        kfa::place(lays[l], h[0], h[1], h[2], pmh);
        kfa::update(x, C, lays[l], k, pmh[0], pmh[1], pmh[2], U);
        lupd = l;
      }
      for (int q = 0; q < 6; ++q) ck[l * 27 + q] = x[q];
      for (int q = 0; q < 21; ++q) ck[l * 27 + 6 + q] = C[q];
    }
    auto ckpt = [&](int l, T xx[6], T CC[21]) {
      for (int q = 0; q < 6; ++q) xx[q] = ck[l * 27 + q];
      for (int q = 0; q < 21; ++q) CC[q] = ck[l * 27 + 6 + q];
    };
    std::vector<T> gi(nl * 5, 0.0);
    auto emit = [&](int l, const T g[5]) {
      for (int q = 0; q < 5; ++q) gi[l * 5 + q] += g[q];
    };
    if (!kfa::track_adjoint<T>(lupd, nl - 1, m, lays.data(), k, Cs, w ? w[i] : 1.0, hit, ckpt, emit,
                               field ? &fk : nullptr))
      return -1;
    for (int q = 0; q < nl * 5; ++q) acc[q] += gi[q];
  }
  for (int l = 0; l < nl; ++l) {
    for (int q = 0; q < 4; ++q) g_align[4 * l + q] = acc[l * 5 + q];
    g_xX0[l] = acc[l * 5 + 4];
  }
  return 0;
}

// The same with the material model: a map [nl][nz] (float32, null: xX0 per layer) over
// each layer's [-zhalf, zhalf] and the mean energy loss per radiation length; the
// forward steps are the library's own (kfa::forward_step).
extern "C" int adjoint_host_model_fp64(int nl, const double* radius, const double* zhalf, double B, double srphi,
                                       double sz, double sr, double mass, const double* align, const double* xX0,
                                       const float* map, int nz, double eloss, long n, const float* hits,
                                       const uint32_t* mask, const double* w, double* g_align, double* g_xX0) {
  using T = double;
  kfa::Consts<T> k;
  k.kB = 0.299792458e-2 * B;
  k.v_r = sr * sr;
  k.v_rphi = srphi * srphi;
  k.v_z = sz * sz;
  k.mass2 = mass * mass;
  std::vector<kfa::Lay<T>> lays(nl);
  for (int l = 0; l < nl; ++l) {
    lays[l].r = radius[l];
    lays[l].cx = align[4 * l + 0];
    lays[l].cy = align[4 * l + 1];
    lays[l].dz = align[4 * l + 2];
    lays[l].cphi = std::cos(align[4 * l + 3]);
    lays[l].sphi = std::sin(align[4 * l + 3]);
    lays[l].xX0 = xX0[l];
    lays[l].pad = 0;
    lays[l].zs = (map && nz > 1) ? (double)nz / (2.0 * zhalf[l]) : 0.0;
    lays[l].zo = 0.5 * nz - 0.5;
  }
  const kfa::MatK<T> mk{map, nz, eloss};
  T Cs[21];
  kfa::seed_cov<T>(srphi, sz, radius[2] - radius[0], k.kB, Cs);
  std::vector<T> acc(nl * 5, 0.0);
  std::vector<T> ck(nl * 27);
  for (long i = 0; i < n; ++i) {
    const uint32_t m = mask[i];
    if ((m & 7u) != 7u) continue;
    auto hit = [&](int l, T h[3]) {
      for (int q = 0; q < 3; ++q) h[q] = hits[((long)l * 3 + q) * n + i];
    };
    T hm[3][3], pm[3][3];
    for (int l = 0; l < 3; ++l) {
      hit(l, hm[l]);
      kfa::place(lays[l], hm[l][0], hm[l][1], hm[l][2], pm[l]);
    }
    kfa::Seed<T> E;
    T x[6], C[21];
    kfa::seed(pm[0], pm[1], pm[2], k, E, x);
    for (int q = 0; q < 21; ++q) C[q] = Cs[q];
    kfa::Upd<T> U;
    kfa::update(x, C, lays[0], k, pm[0][0], pm[0][1], pm[0][2], U);
    for (int q = 0; q < 6; ++q) ck[q] = x[q];
    for (int q = 0; q < 21; ++q) ck[6 + q] = C[q];
    int last = 31 - __builtin_clz(m);
    if (last > nl - 1) last = nl - 1;
    int lupd = 0;
    bool ok = true;
    for (int l = 1; l <= last && ok; ++l) {
      ok = kfa::forward_step<T>(l, m, lays.data(), k, nullptr, hit, x, C, &mk);
      if (!ok) break;
      if ((m >> l) & 1u) lupd = l;
      for (int q = 0; q < 6; ++q) ck[l * 27 + q] = x[q];
      for (int q = 0; q < 21; ++q) ck[l * 27 + 6 + q] = C[q];
    }
    if (!ok) continue;   // a particle that stops: its fit ends there (left out here)
    auto ckpt = [&](int l, T xx[6], T CC[21]) {
      for (int q = 0; q < 6; ++q) xx[q] = ck[l * 27 + q];
      for (int q = 0; q < 21; ++q) CC[q] = ck[l * 27 + 6 + q];
    };
    std::vector<T> gi(nl * 5, 0.0);
    auto emit = [&](int l, const T g[5]) {
      for (int q = 0; q < 5; ++q) gi[l * 5 + q] += g[q];
    };
    if (!kfa::track_adjoint<T>(lupd, nl - 1, m, lays.data(), k, Cs, w ? w[i] : 1.0, hit, ckpt, emit, nullptr, &mk))
      return -1;
    for (int q = 0; q < nl * 5; ++q) acc[q] += gi[q];
  }
  for (int l = 0; l < nl; ++l) {
    for (int q = 0; q < 4; ++q) g_align[4 * l + q] = acc[l * 5 + q];
    g_xX0[l] = acc[l * 5 + 4];
  }
  return 0;
}
