// Host-side instantiations of the library's smoother step (kf_smooth.h), for the CPU
// tests against the FP64 oracle smoother on the oracle's own filtered estimates: in
// double the two must agree to rounding (the library's covariance form is the
// textbook one rearranged), in float what is left is the step's float arithmetic.
#include <cmath>
#include <vector>

#include "../paper_1906_11744_amd/csrc/kf_smooth.h"

// map [nl][nz] (float32, null: none), zhalf [nl], eloss, fr, fz: the detector model;
// use_model = 0 runs the plain step.
// kF32: the step's C_p^-1 block in float with its condition check (det_thr), counting
// in *fallbacks the steps that redo it in double.
template <class T, bool kF32 = false>
static int smooth_host(int nl, const double* radius, double B, double srphi, double sz, double sr, double mass,
                       const double* align, const double* xX0, long n, const double* rec, const int* lend,
                       double* xs_out, double* Cs_out, int use_model = 0, const float* map = nullptr, int nz = 0,
                       const double* zhalf = nullptr, double eloss = 0.0, double fr = 0.0, double fz = 0.0,
                       double det_thr = 1e-2) {
  kfa::Consts<T> k;
  k.kB = (T)(0.299792458e-2 * B);
  k.v_r = (T)(sr * sr);
  k.v_rphi = (T)(srphi * srphi);
  k.v_z = (T)(sz * sz);
  k.mass2 = (T)(mass * mass);
  k.det_thr = (T)det_thr;
  std::vector<kfa::Lay<T>> lays(nl);
  for (int l = 0; l < nl; ++l) {
    lays[l].r = (T)radius[l];
    lays[l].cx = (T)align[4 * l + 0];
    lays[l].cy = (T)align[4 * l + 1];
    lays[l].dz = (T)align[4 * l + 2];
    lays[l].cphi = (T)std::cos(align[4 * l + 3]);
    lays[l].sphi = (T)std::sin(align[4 * l + 3]);
    lays[l].xX0 = (T)xX0[l];
    lays[l].pad = 0;
    lays[l].zs = (map && nz > 1) ? (T)((double)nz / (2.0 * zhalf[l])) : T(0);
    lays[l].zo = (T)(0.5 * nz - 0.5);
  }
  int bad = 0;
  for (long i = 0; i < n; ++i) {
    const int le = lend[i];
    if (le < 0) continue;
    const double* r = rec + i * (long)nl * 27;
    T xf1[6], ds[6], Cs1[21], xs[6];
    for (int q = 0; q < 6; ++q) xf1[q] = (T)r[(long)le * 27 + q];
    for (int q = 0; q < 6; ++q) ds[q] = T(0);
    for (int q = 0; q < 21; ++q) Cs1[q] = (T)r[(long)le * 27 + 6 + q];
    auto put = [&](int l, const T* x, const T* C) {
      for (int q = 0; q < 6; ++q) xs_out[((long)l * 6 + q) * n + i] = x[q];
      for (int q = 0; q < 21; ++q) Cs_out[((long)l * 21 + q) * n + i] = C[q];
    };
    put(le, xf1, Cs1);
    for (int l = le - 1; l >= 0; --l) {
      T xf[6], Cf[21];
      for (int q = 0; q < 6; ++q) xf[q] = (T)r[(long)l * 27 + q];
      for (int q = 0; q < 21; ++q) Cf[q] = (T)r[(long)l * 27 + 6 + q];
      kfs::StepModel<T> sm{map ? map + (long)(l + 1) * nz : nullptr, nz, (T)eloss, (T)fr, (T)fz};
      if (!kfs::rts_step<T, kF32>(xf, Cf, xf1, lays[l + 1], k, ds, Cs1, use_model ? &sm : nullptr)) {
        ++bad;
        break;
      }
      kfs::smoothed_state<T>(xf, ds, xs);
      put(l, xs, Cs1);
      for (int q = 0; q < 6; ++q) xf1[q] = xf[q];
    }
  }
  return bad;
}

extern "C" int smooth_host_f32(int nl, const double* radius, double B, double srphi, double sz, double sr,
                               double mass, const double* align, const double* xX0, long n, const double* rec,
                               const int* lend, double* xs_out, double* Cs_out) {
  return smooth_host<float>(nl, radius, B, srphi, sz, sr, mass, align, xX0, n, rec, lend, xs_out, Cs_out);
}

extern "C" int smooth_host_f64(int nl, const double* radius, double B, double srphi, double sz, double sr,
                               double mass, const double* align, const double* xX0, long n, const double* rec,
                               const int* lend, double* xs_out, double* Cs_out) {
  return smooth_host<double>(nl, radius, B, srphi, sz, sr, mass, align, xX0, n, rec, lend, xs_out, Cs_out);
}

extern "C" int smooth_host_model_f32(int nl, const double* radius, double B, double srphi, double sz, double sr,
                                     double mass, const double* align, const double* xX0, long n, const double* rec,
                                     const int* lend, double* xs_out, double* Cs_out, const float* map, int nz,
                                     const double* zhalf, double eloss, double fr, double fz) {
  return smooth_host<float>(nl, radius, B, srphi, sz, sr, mass, align, xX0, n, rec, lend, xs_out, Cs_out, 1, map, nz,
                            zhalf, eloss, fr, fz);
}

extern "C" int smooth_host_model_f64(int nl, const double* radius, double B, double srphi, double sz, double sr,
                                     double mass, const double* align, const double* xX0, long n, const double* rec,
                                     const int* lend, double* xs_out, double* Cs_out, const float* map, int nz,
                                     const double* zhalf, double eloss, double fr, double fz) {
  return smooth_host<double>(nl, radius, B, srphi, sz, sr, mass, align, xX0, n, rec, lend, xs_out, Cs_out, 1, map, nz,
                             zhalf, eloss, fr, fz);
}

extern "C" int smooth_host_f32_check(int nl, const double* radius, double B, double srphi, double sz, double sr,
                                     double mass, const double* align, const double* xX0, long n, const double* rec,
                                     const int* lend, double* xs_out, double* Cs_out, double det_thr) {
  return smooth_host<float, true>(nl, radius, B, srphi, sz, sr, mass, align, xX0, n, rec, lend, xs_out, Cs_out, 0,
                                  nullptr, 0, nullptr, 0.0, 0.0, 0.0, det_thr);
}
