// One backward step of the fixed-interval (Rauch-Tung-Striebel) smoother over the
// batched fit, templated on the scalar type and usable on host and device.
//
// The paper's tracking chain ends with a backward pass and a final fit of the built
// tracks (Sec. 4.2, Sec. 5); here it is the smoother on the filter's own
// linearisation.  From the filtered estimate (x_f, C_f) at layer l, the step to layer
// l + 1 is predicted exactly as the fit does it (crossing, fixed-arc transport
// J, Highland noise Q) to (x_p, C_p = J C_f J^T + Q); with the smoothed (x_s1, C_s1)
// at l + 1,
//   G   = C_f J^T C_p^-1,
//   x_s = x_f + G (x_s1 - x_p)          (azimuth difference wrapped),
//   C_s = C_f + G (C_s1 - C_p) G^T.
// In float the textbook covariance update cancels: at the inner layers C_s is orders
// of magnitude below C_f.  It is evaluated instead as the equivalent sum of
// positive semi-definite terms
//   C_s = M C_f M^T + G (Q + C_s1) G^T,   M = I - G J = J^-1 W J,   G = J^-1 (I - W),
// with W = Q C_p^-1 (J^-1 = I - N + N^2 exactly, N the six off-diagonal transport
// terms, since N^3 = 0), and the first term reduced to a 3x3 product (see below).  Without material W = 0, G = J^-1 and C_s is C_s1 carried back through the
// step.
#pragma once

#include "kf_adjoint.h"

namespace kfs {

using kfa::tri;

template <class T>
KFA_HD T wrap(T a) {
  const T pi = T(3.14159265358979323846), two_pi = T(6.28318530717958647692);
  if (a > pi) a -= two_pi;
  if (a <= -pi) a += two_pi;
  return a;
}

// (I + A) C (I + A)^T for an A with the transport's six off-diagonal positions (0|1,
// 3|4), (2, 5), (4, 3), accumulated in the precision U from C.  J^-1 = I - N + N^2 has
// the same pattern as J = I + N.
template <class U, class T>
KFA_HD void sandwich_n(U a03, U a04, U a13, U a14, U a25, U a43, const T C[21], U Co[21]) {
  auto c = [&](int i, int j) { return (U)C[tri(i, j)]; };
  U B[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    B[0][j] = c(0, j) + a03 * c(3, j) + a04 * c(4, j);
    B[1][j] = c(1, j) + a13 * c(3, j) + a14 * c(4, j);
    B[2][j] = c(2, j) + a25 * c(5, j);
    B[3][j] = c(3, j);
    B[4][j] = c(4, j) + a43 * c(3, j);
    B[5][j] = c(5, j);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    Co[tri(i, 0)] = B[i][0] + a03 * B[i][3] + a04 * B[i][4];
    if (i >= 1) Co[tri(i, 1)] = B[i][1] + a13 * B[i][3] + a14 * B[i][4];
    if (i >= 2) Co[tri(i, 2)] = B[i][2] + a25 * B[i][5];
    if (i >= 3) Co[tri(i, 3)] = B[i][3];
    if (i >= 4) Co[tri(i, 4)] = B[i][4] + a43 * B[i][3];
    if (i >= 5) Co[tri(i, 5)] = B[i][5];
  }
}

// J C J^T (J = I + N, the transport of the step) accumulated in the precision U from
// C: in double the transported covariance keeps what a float C itself holds, which
// the C_p^-1 block below can need.
template <class U, class T>
KFA_HD void transport_cov_u(const kfa::Prop<T>& P, const T C[21], U Co[21]) {
  sandwich_n<U>((U)P.a03, (U)P.a04, (U)P.a13, (U)P.a14, (U)P.a25, (U)P.a43, C, Co);
}

// Structural non-zeros of J^-1 = I - N + N^2 for the transport's six off-diagonal
// terms N (at (0|1, 3|4), (2, 5), (4, 3); N^2 adds only to (0|1, 3)): products with the
// other entries, exactly zero, are skipped (a float product with a literal zero is not
// folded away, since the other factor could be infinite).
KFA_HD constexpr bool ji_nz(int i, int j) {
  return i == j || ((i == 0 || i == 1) && (j == 3 || j == 4)) || (i == 2 && j == 5) || (i == 4 && j == 3);
}

// The smoothed state is carried as its offset from the filtered one, ds = x_s - x_f:
// offsets are small, so their float rounding is relative to the offset and does not
// accumulate over the layers (a smoothed theta carried whole, rounded at every step,
// would drift by ulps that the 100 cm lever arm turns into ~1e-4 cm in z).
template <class T>
KFA_HD void smoothed_state(const T xf[6], const T ds[6], T xs[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) xs[q] = xf[q] + ds[q];
  xs[4] = wrap(xs[4]);
}

// The detector model of one step (Sec. 3), as the fit takes it: the material map's
// row of the layer stepped to (null: that layer's x/X0), the mean ionisation loss per
// radiation length and the field B_z(r, z) = B (1 + fr r^2 + fz z^2).
template <class T>
struct StepModel {
  const float* row;
  int nz;
  T eloss, fr, fz;
};

// x/X0 of a layer at z (global) from its map row: linear between the centres of nz
// equal bins over [-Z, Z] of the layer's frame (u = (z - dz) zs + zo, in bins),
// constant beyond the outer centres.
template <class T>
KFA_HD T map_value(const float* row, int nz, const kfa::Lay<T>& ly, T z) {
  if (nz == 1) return (T)row[0];
  T u = (z - ly.dz) * ly.zs + ly.zo;
  u = u < T(0) ? T(0) : (u > T(nz - 1) ? T(nz - 1) : u);
  int b = (int)u;
  if (b > nz - 2) b = nz - 2;
  const T t = u - (T)b;
  const T v0 = (T)row[b];
  return v0 + t * ((T)row[b + 1] - v0);
}

// The mean energy loss at a predicted state as a map of kappa: kappa' = g kappa with
// g = p / p', and its derivatives D = dkappa'/dkappa, Tt = dkappa'/dtheta (the path
// length x/X0 / (sin theta |cos alpha|) held fixed), written without cancellation:
// with W = p X / p'^3 and X = dE (m^2/E + E') + 2 eloss x_eff m^2 E' / p^2,
// D = p/p' + W and Tt = kappa cot(theta) W.  False if the particle stops.
template <class T>
KFA_HD bool loss_map(T kap, T st, T ct, T cosa, T xx, T eloss, T mass2, T& g, T& D, T& Tt) {
  using std::fabs; using std::sqrt;
  const T ks = fabs(kap) * st;
  const T p = T(1) / ks;
  const T c = eloss * xx / (st * fabs(cosa));
  const T ib2 = T(1) + mass2 * ks * ks;
  const T E = p * sqrt(ib2);
  const T dE = c * ib2;
  const T E1 = E - dE;
  const T q2 = E1 * E1 - mass2;
  if (!(E1 > T(0)) || !(q2 > T(0))) return false;
  const T ip1 = T(1) / sqrt(q2);
  const T X = dE * (mass2 / E + E1) + T(2) * c * mass2 * E1 * ks * ks;
  const T W = p * X * (ip1 * ip1 * ip1);
  g = p * ip1;
  D = g + W;
  Tt = kap * (ct / st) * W;
  return true;
}

// C_p = J C_f J^T + Q factorised, and what the step needs of C_p^-1, formed in the
// precision U: W = Q C_p^-1 (rows 3..5; Q is non-zero in its (kappa, phi, theta) block
// Q3 only) and T3 = Q3 R Q3 (I - R Q3), R the (3..5, 3..5) block of C_p^-1.  pivot
// receives the smallest pivot of the factorisation of C_p equilibrated to unit
// diagonal, or the smallest diagonal element of I - R Q3 if that is smaller; false if
// C_p is not positive definite (to U's rounding).
template <class U, class T>
KFA_HD bool cp_terms(const kfa::Prop<T>& P, const T Cf[21], const T Q[21], T W[6][6], T T3[3][3], T& pivot) {
  using std::sqrt;
  U dsc[6], L[21], linv[6];
  transport_cov_u<U>(P, Cf, L);
#pragma unroll
  for (int i = 3; i < 6; ++i)
#pragma unroll
    for (int j = 3; j <= i; ++j) L[tri(i, j)] += (U)Q[tri(i, j)];  // Q's (kappa, phi, theta) block
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const U cii = L[tri(i, i)];
    if (!(cii > U(1e-30) && cii < U(1e30))) return false;
    dsc[i] = (U)(1.0f / sqrt((float)cii));
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    U djj = L[tri(j, j)] * dsc[j] * dsc[j];
#pragma unroll
    for (int q = 0; q < j; ++q) djj -= L[tri(j, q)] * L[tri(j, q)];
    if (!(djj > U(1e-30))) return false;  // not positive definite (to U's rounding)
    pivot = j == 0 ? (T)djj : (pivot < (T)djj ? pivot : (T)djj);
    U r = (U)(1.0f / sqrt((float)djj));
    r = r * (U(1.5) - U(0.5) * djj * r * r);
    r = r * (U(1.5) - U(0.5) * djj * r * r);
    L[tri(j, j)] = djj * r;
    linv[j] = r;
#pragma unroll
    for (int i = j + 1; i < 6; ++i) {
      U a = L[tri(i, j)] * dsc[i] * dsc[j];
#pragma unroll
      for (int q = 0; q < j; ++q) a -= L[tri(i, q)] * L[tri(j, q)];
      L[tri(i, j)] = a * r;
    }
  }
  U Y[3][6];  // Y[b] = C_p^-1 e_(3+b); the forward sweep starts at row 3+b
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int c = 3 + b;
    U y[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i < c) {
        y[i] = U(0);
        continue;
      }
      U a = i == c ? dsc[i] : U(0);
#pragma unroll
      for (int q = c; q < i; ++q) a -= L[tri(i, q)] * y[q];
      y[i] = a * linv[i];
    }
#pragma unroll
    for (int i = 5; i >= 0; --i) {
      U a = y[i];
#pragma unroll
      for (int q = i + 1; q < 6; ++q) a -= L[tri(q, i)] * y[q];
      y[i] = a * linv[i];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) Y[b][i] = y[i] * dsc[i];
  }
  U Q3[3][3], A[3][3], Tm[3][3], V[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Q3[a][b] = (U)Q[tri(3 + a, 3 + b)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      U w = U(0);
#pragma unroll
      for (int b = 0; b < 3; ++b) w += Q3[a][b] * Y[b][i];
      W[3 + a][i] = (T)w;
      if (i >= 3) A[a][i - 3] = w;  // Q3 R
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      U v = a == b ? U(1) : U(0), t = U(0);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        v -= Y[q][3 + a] * Q3[q][b];  // (I - R Q3)
        t += A[a][q] * Q3[q][b];      // Q3 R Q3
      }
      V[a][b] = v;
      Tm[a][b] = t;
      if (a == b) pivot = pivot < (T)v ? pivot : (T)v;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      U t = U(0);
#pragma unroll
      for (int q = 0; q < 3; ++q) t += Tm[a][q] * V[q][b];
      T3[a][b] = (T)t;
    }
  return true;
}

// One step in place: on entry (ds, Cs) is the smoothed estimate at layer l + 1 (ds its
// offset from the filtered state xf1 there), on return the one at layer l (ds the
// offset from xf).  xf, Cf: filtered estimate at l (packed lower C); ly1: the
// constants of layer l + 1; sm: the detector model of the step (null: one x/X0 per
// layer, uniform field).  Returns false (ds, Cs unchanged) if layer l + 1 is not
// reached from x_f, the particle stops in its material, or C_p is not positive
// definite.
// With energy loss the step's linearisation is A J, A the identity but for the kappa
// row (D, Tt of loss_map), and C_p = A (J C_f J^T + Q) A^T, so the gain is
// G = C_f J^T (J C_f J^T + Q)^-1 A^-1: the step below, written for A = I, applies
// unchanged to A^-1 (x_s1 - x_p) and A^-1 C_s1 A^-T.
template <class T, bool kF32 = false>
KFA_HD bool rts_step(const T xf[6], const T Cf[21], const T xf1[6], const kfa::Lay<T>& ly1,
                     const kfa::Consts<T>& k0, T ds[6], T Cs[21], const StepModel<T>* sm = nullptr) {
  using std::sqrt;
  kfa::Consts<T> k = k0;
  if (sm) k.kB = k0.kB * (T(1) + sm->fr * (xf[0] * xf[0] + xf[1] * xf[1]) + sm->fz * xf[2] * xf[2]);
  kfa::Prop<T> P;
  T xp[6];
  if (!kfa::propagate(xf, ly1, k, P, xp)) return false;
  kfa::Lay<T> lym = ly1;
  if (sm && sm->row) lym.xX0 = map_value<T>(sm->row, sm->nz, ly1, xp[2]);
  T gl = T(1), Dl = T(1), Tl = T(0);
  const bool loss = sm && sm->eloss > T(0) && lym.xX0 > T(0);
  T Q[21];
  const kfa::Frm<T> fr = kfa::frame(xp, lym);
  if (loss && !loss_map<T>(xp[3], P.st, P.ct, fr.rx * P.cpe + fr.ry * P.spe, lym.xX0, sm->eloss, k.mass2, gl, Dl, Tl))
    return false;
  kfa::Scat<T> S;
#pragma unroll
  for (int q = 0; q < 21; ++q) Q[q] = T(0);
  kfa::scatter(xp, fr, lym, k, S, Q);  // Q alone: (kappa, phi, theta) block
  // J = I + N and J^-1 = I - N + N^2, as dense 6x6
  T N[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) N[i][j] = T(0);
  N[0][3] = P.a03;
  N[0][4] = P.a04;
  N[1][3] = P.a13;
  N[1][4] = P.a14;
  N[2][5] = P.a25;
  N[4][3] = P.a43;
  T Ji[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) Ji[i][j] = (i == j ? T(1) : T(0)) - N[i][j];
  Ji[0][3] += N[0][4] * N[4][3];
  Ji[1][3] += N[1][4] * N[4][3];
  // Only Q's (kappa, phi, theta) block Q3 is non-zero, so W = Q C_p^-1 has non-zero
  // rows 3..5 only: W[3+a][i] = sum_b Q3[a][b] (C_p^-1)[3+b][i].  With R the same block
  // of C_p^-1 and J C_f J^T = C_p - Q, the first term of C_s is
  //   M C_f M^T = J^-1 W (C_p - Q) W^T J^-T = K T K^T,  T = Q3 R Q3 (I - R Q3),
  // K = columns 3..5 of J^-1: a 3x3 product in place of the 6x6 sandwich of C_f,
  // which at layers the fit saw through few hits (C_f orders of magnitude above C_s)
  // would cancel.  C_p^-1's three columns come from a Cholesky factorisation of C_p
  // equilibrated to unit diagonal (cp_terms), formed in double from C_p = J C_f J^T +
  // Q accumulated in double: C_p's condition number after equilibration can reach ~1e5,
  // and where the scattering dominates the filtered angles I - R Q3 recovers the part
  // of J C_f J^T that a float C_p would round away.  kF32: the block in float instead,
  // formed again in double where its condition check fails: the factorisation's
  // smallest pivot (the fraction of a component's variance left once the earlier
  // components are known) or the smallest diagonal element of I - R Q3 below
  // k0.det_thr.  (That variant meets the 1e-4 bar at det_thr 1e-2 with a tenth of the
  // steps in double; in 64-lane waves nearly every wave then runs both paths.)  No
  // correctly rounded division or square root is needed: the equilibration scale is
  // any positive number near C_p's diagonal^-1/2 (it is undone exactly), and the
  // pivots' inverse square roots are float estimates refined by two Newton steps.
  T W[6][6];  // rows 3..5 only
  T T3[3][3];
  T piv = T(0);
  if (!kF32 || !cp_terms<T, T>(P, Cf, Q, W, T3, piv) || !(piv >= k0.det_thr)) {
    if (!cp_terms<double, T>(P, Cf, Q, W, T3, piv)) return false;
  }
  // G = J^-1 V with V = I - W, which differs from I in rows 3..5 only (V3 below); G is
  // applied as its two factors
  T V3[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 6; ++j) V3[a][j] = (j == 3 + a ? T(1) : T(0)) - W[3 + a][j];
  // state: x_s - x_f = G (x_s1 - x_p), with x_s1 - x_p = ds1 + (x_f1 - x_p) and x_f1 -
  // x_p taken as the difference of the two filtered states less the step (exact or
  // nearly so in float: the rounding of x_p's ~100 cm coordinates would otherwise cost
  // ~4e-6 cm against differences of ~1e-3 cm)
  T d[6];
  d[0] = ds[0] + ((xf1[0] - xf[0]) - P.dx);
  d[1] = ds[1] + ((xf1[1] - xf[1]) - P.dy);
  d[2] = ds[2] + ((xf1[2] - xf[2]) - P.s * P.ct / P.st);
  d[3] = ds[3] + (xf1[3] - gl * xf[3]);  // x_p's kappa: the loss scales the filtered one
  d[4] = ds[4] + (wrap(xf1[4] - xf[4]) - P.u);
  d[5] = ds[5] + (xf1[5] - xf[5]);
  if (loss) {  // back through the loss: d <- A^-1 d, C_s1 <- A^-1 C_s1 A^-T
    const T iD = T(1) / Dl, a = Tl * iD;
    d[3] = iD * d[3] - a * d[5];
    const T c33 = Cs[tri(3, 3)], c53 = Cs[tri(5, 3)], c55 = Cs[tri(5, 5)];
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j != 3) Cs[tri(3, j)] = iD * Cs[tri(3, j)] - a * Cs[tri(5, j)];
    Cs[tri(5, 3)] = iD * c53 - a * c55;
    Cs[tri(3, 3)] = iD * iD * c33 - T(2) * iD * a * c53 + a * a * c55;
  }
  T vd[6];  // V d
#pragma unroll
  for (int i = 0; i < 3; ++i) vd[i] = d[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T v = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) v += V3[a][j] * d[j];
    vd[3 + a] = v;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T a = T(0);
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (ji_nz(i, q)) a += Ji[i][q] * vd[q];
    ds[i] = a;
  }
  // covariance: C_s = K T K^T + J^-1 F J^-T with F = V E V^T, E = Q + C_s1 (Q is zero
  // outside its (kappa, phi, theta) block): V's identity rows leave rows and columns
  // 0..2 of E as they are, so only rows 3..5 of V E (P3) and the (3..5, 3..5) block of
  // F are products; J^-1 has the transport's sparsity
  T E[21];
#pragma unroll
  for (int q = 0; q < 21; ++q) E[q] = Cs[q];
#pragma unroll
  for (int i = 3; i < 6; ++i)
#pragma unroll
    for (int j = 3; j <= i; ++j) E[tri(i, j)] += Q[tri(i, j)];
  T P3[3][6];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      T v = T(0);
#pragma unroll
      for (int q = 0; q < 6; ++q) v += V3[a][q] * E[tri(q, j)];
      P3[a][j] = v;
    }
  T F[21];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      if (i < 3) {
        F[tri(i, j)] = E[tri(i, j)];
      } else if (j < 3) {
        F[tri(i, j)] = P3[i - 3][j];
      } else {
        T v = T(0);
#pragma unroll
        for (int q = 0; q < 6; ++q) v += P3[i - 3][q] * V3[j - 3][q];
        F[tri(i, j)] = v;
      }
    }
  sandwich_n<T>(Ji[0][3], Ji[0][4], Ji[1][3], Ji[1][4], Ji[2][5], Ji[4][3], F, Cs);
  T KT[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (ji_nz(i, 3 + q)) a += Ji[i][3 + q] * (T(0.5) * (T3[q][b] + T3[b][q]));
      KT[i][b] = a;
    }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T acc = Cs[tri(i, j)];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (ji_nz(j, 3 + q)) acc += KT[i][q] * Ji[j][3 + q];
      Cs[tri(i, j)] = acc;
    }
  return true;
}

}  // namespace kfs
