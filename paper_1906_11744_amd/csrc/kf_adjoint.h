// Reverse-mode (adjoint) of one track's Kalman fit, templated on the scalar type and
// usable on host and device.  The fit runs forward once and checkpoints the state and
// covariance after every layer; the reverse sweep recomputes each step from the
// checkpoint before it and propagates adjoints backwards through
//   update (frame, H, S, S^-1, residual, chi2, gain, covariance),
//   multiple-scattering noise Q (Highland width, crossing angle, material x/X0),
//   transport (the helix map at fixed arc, C <- J C J^T, and the arc itself, whose
//   dependence on the state and the layer axis follows from |p(s) - c|^2 = r^2 by
//   implicit differentiation),
// down to the three-hit seed, and finally into the per-layer alignment (hit
// placement and layer axis) and material parameters.
//
// The covariance update is differentiated as C+ = C - (HC)^T S^-1 (HC): with the
// optimal gain the Joseph form equals it and is stationary in the gain, so both have
// the same derivatives.  Covariance adjoints are symmetric matrices G with
// dL = sum_ij G_ij dC_ij over all 36 entries, stored packed.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <cmath>

#define KFA_HD __host__ __device__ __forceinline__

namespace kfa {

KFA_HD constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Per-layer constants; the float layout is that of the fit kernels' layer table.
template <class T>
struct Lay {
  T r, cx, cy, dz, cphi, sphi, xX0, pad, zs, zo;  // pad: unused here; zs, zo: the material map's z bins (smoother)
  T endcap[5];  // endcap surface fields of the forward table: unused (cylinders only here)
};

template <class T>
struct Consts {
  T kB, v_r, v_rphi, v_z, mass2;
  // float S^-1: below this determinant of the equilibrated S (unit diagonal) the
  // inverse is formed in double, as the forward fit does (> 1 forces it everywhere)
  T det_thr = T(1e-2);
};

// ---------------------------------------------------------------------------------
// forward pieces (pure functions of their inputs)
// ---------------------------------------------------------------------------------

// Helix step to the first forward crossing: tape of everything its adjoint needs.
template <class T>
struct Prop {
  T s, u, w;         // arc, turning angle, omega
  T cp, sp;          // start direction
  T cpe, spe;        // end direction
  T dx, dy;          // displacement
  T F1, F2, F1d, F2d;  // d(displacement)/d(omega) = s^2 (F1 t + F2 n), and dF/du
  T a03, a13, a04, a14, a25, a43;  // transport Jacobian terms
  T st, ct;          // sin, cos theta
  T ex, ey;          // end point relative to the layer axis
  T Ds;              // e' . t' (d|p - c|^2 / ds / 2)
};

// sin and cos of one angle (one range reduction for both in float)
KFA_HD void sin_cos(float a, float& s, float& c) { sincosf(a, &s, &c); }
KFA_HD void sin_cos(double a, double& s, double& c) { s = std::sin(a); c = std::cos(a); }

template <class T>
KFA_HD bool propagate(const T x[6], const Lay<T>& ly, const Consts<T>& k, Prop<T>& P, T xo[6]) {
  using std::atan; using std::cos; using std::sin; using std::sqrt; using std::fabs;
  sin_cos(x[4], P.sp, P.cp);
  sin_cos(x[5], P.st, P.ct);
  const T ex = x[0] - ly.cx, ey = x[1] - ly.cy;
  const T a = ex * P.cp + ey * P.sp;
  const T b = ey * P.cp - ex * P.sp;
  const T c0 = ex * ex + ey * ey - ly.r * ly.r;
  const T w = -k.kB * x[3];
  const T A = T(2) + T(2) * w * b + T(0.5) * w * w * c0;
  const T D = a * a - T(0.5) * A * c0;
  if (!(c0 < T(0)) || !(D >= T(0))) return false;
  const T den = a + sqrt(D);
  if (!(den > T(0))) return false;
  const T sig = -c0 / (T(2) * den);
  const T tau = w * sig;
  const T tau2 = tau * tau;
  // atan(tau)/tau by its Taylor series where the truncation is below the type's
  // rounding: to tau^12 below |tau| = 0.3 in float (< 3e-9), to tau^4 below 1e-2 in
  // double (< 2e-13); atan beyond
  T q;
  if constexpr (sizeof(T) == 4) {
    if (fabs(tau) < T(0.3))
      q = T(1) + tau2 * (T(-1) / T(3) + tau2 * (T(0.2) + tau2 * (T(-1) / T(7) + tau2 * (T(1) / T(9) +
          tau2 * (T(-1) / T(11) + tau2 * (T(1) / T(13)))))));
    else
      q = atan(tau) / tau;
  } else {
    q = fabs(tau) < T(1e-2) ? T(1) + tau2 * (T(-1) / T(3) + tau2 * T(0.2)) : atan(tau) / tau;
  }
  const T f = T(2) * sig / (T(1) + tau2);
  P.w = w;
  P.s = T(2) * sig * q;
  P.u = T(2) * tau * q;
  P.dx = f * (P.cp - tau * P.sp);
  P.dy = f * (P.sp + tau * P.cp);
  const T inv1 = T(1) / (T(1) + tau2);
  const T cu = (T(1) - tau2) * inv1, su = T(2) * tau * inv1;
  P.cpe = P.cp * cu - P.sp * su;
  P.spe = P.sp * cu + P.cp * su;
  const T u = P.u, u2 = u * u;
  if (fabs(u) < T(0.3)) {
    P.F1 = u * (T(-1) / T(3) + u2 * (T(1) / T(30) - u2 / T(840)));
    P.F2 = T(0.5) + u2 * (T(-0.125) + u2 * (T(1) / T(144) - u2 / T(5760)));
    P.F1d = T(-1) / T(3) + u2 * (T(0.1) - u2 / T(168));
    P.F2d = u * (T(-0.25) + u2 * (T(1) / T(36) - u2 / T(960)));
  } else {
    const T cs = cos(u), sn = sin(u);
    P.F1 = (u * cs - sn) / u2;
    P.F2 = (u * sn - T(1) + cs) / u2;
    P.F1d = (-u2 * sn - T(2) * u * cs + T(2) * sn) / (u2 * u);
    P.F2d = (u2 * cs - T(2) * u * sn + T(2) - T(2) * cs) / (u2 * u);
  }
  const T ks2 = -k.kB * P.s * P.s;
  P.a04 = -P.dy;
  P.a14 = P.dx;
  P.a03 = ks2 * (P.F1 * P.cp - P.F2 * P.sp);
  P.a13 = ks2 * (P.F1 * P.sp + P.F2 * P.cp);
  P.a25 = -P.s / (P.st * P.st);
  P.a43 = -k.kB * P.s;
  xo[0] = x[0] + P.dx;
  xo[1] = x[1] + P.dy;
  xo[2] = x[2] + P.s * P.ct / P.st;
  xo[3] = x[3];
  xo[4] = x[4] + P.u;
  xo[5] = x[5];
  P.ex = xo[0] - ly.cx;
  P.ey = xo[1] - ly.cy;
  P.Ds = P.ex * P.cpe + P.ey * P.spe;
  return true;
}

// C' = J C J^T with the sparse J of the step; B = J C is kept for the adjoint.
template <class T>
KFA_HD void transport_cov(const Prop<T>& P, const T C[21], T B[6][6], T Co[21]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    B[0][j] = C[tri(0, j)] + P.a03 * C[tri(3, j)] + P.a04 * C[tri(4, j)];
    B[1][j] = C[tri(1, j)] + P.a13 * C[tri(3, j)] + P.a14 * C[tri(4, j)];
    B[2][j] = C[tri(2, j)] + P.a25 * C[tri(5, j)];
    B[3][j] = C[tri(3, j)];
    B[4][j] = C[tri(4, j)] + P.a43 * C[tri(3, j)];
    B[5][j] = C[tri(5, j)];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    Co[tri(i, 0)] = B[i][0] + P.a03 * B[i][3] + P.a04 * B[i][4];
    if (i >= 1) Co[tri(i, 1)] = B[i][1] + P.a13 * B[i][3] + P.a14 * B[i][4];
    if (i >= 2) Co[tri(i, 2)] = B[i][2] + P.a25 * B[i][5];
    if (i >= 3) Co[tri(i, 3)] = B[i][3];
    if (i >= 4) Co[tri(i, 4)] = B[i][4] + P.a43 * B[i][3];
    if (i >= 5) Co[tri(i, 5)] = B[i][5];
  }
}

// Local frame at a point of a layer.
template <class T>
struct Frm {
  T ex, ey, rho, rx, ry;
};

template <class T>
KFA_HD Frm<T> frame(const T x[6], const Lay<T>& ly) {
  using std::sqrt;
  Frm<T> f;
  f.ex = x[0] - ly.cx;
  f.ey = x[1] - ly.cy;
  f.rho = sqrt(f.ex * f.ex + f.ey * f.ey);
  f.rx = f.ex / f.rho;
  f.ry = f.ey / f.rho;
  return f;
}

// Highland noise: tape and the four changed covariance entries.
template <class T>
struct Scat {
  T th2, lg, xe, ks, cota, st, ct, ca, tx, ty;
  bool on;
};

template <class T>
KFA_HD void scatter(const T x[6], const Frm<T>& f, const Lay<T>& ly, const Consts<T>& k, Scat<T>& Q, T C[21]) {
  using std::cos; using std::sin; using std::log; using std::fabs;
  Q.on = ly.xX0 > T(0);
  if (!Q.on) return;
  Q.st = sin(x[5]);
  Q.ct = cos(x[5]);
  Q.tx = cos(x[4]);
  Q.ty = sin(x[4]);
  Q.ca = f.rx * Q.tx + f.ry * Q.ty;
  Q.ks = x[3] * Q.st;
  Q.xe = ly.xX0 / (Q.st * fabs(Q.ca));
  Q.lg = T(1) + T(0.038) * log(Q.xe);
  const T ks2 = Q.ks * Q.ks;
  Q.th2 = T(0.0136) * T(0.0136) * ks2 * (T(1) + k.mass2 * ks2) * Q.xe * Q.lg * Q.lg;
  Q.cota = Q.ct / Q.st;
  const T kc = x[3] * Q.cota;
  C[tri(4, 4)] += Q.th2 / (Q.st * Q.st);
  C[tri(5, 5)] += Q.th2;
  C[tri(3, 3)] += kc * kc * Q.th2;
  C[tri(5, 3)] -= kc * Q.th2;
}

// Measurement model and update at a predicted state.
template <class T>
struct Upd {
  Frm<T> f;
  T tx, ty, ca, sa, tana, cot, q;
  T h1x, h1y, h2x, h2y;
  T A1[6], A2[6];   // rows 1, 2 of H C
  T Si11, Si12, Si22, Si00;
  T dx, dy, X, Y, psi, r0, r1, r2, rm, g1, g2;
  T mex, mey;       // m - c
};

template <class T>
KFA_HD T update(T x[6], T C[21], const Lay<T>& ly, const Consts<T>& k, T mx, T my, T mz, Upd<T>& U) {
  using std::atan2; using std::cos; using std::sin; using std::sqrt;
  U.f = frame(x, ly);
  U.tx = cos(x[4]);
  U.ty = sin(x[4]);
  U.ca = U.f.rx * U.tx + U.f.ry * U.ty;
  U.sa = -U.f.ry * U.tx + U.f.rx * U.ty;
  U.tana = U.sa / U.ca;
  U.cot = cos(x[5]) / sin(x[5]);
  U.q = U.cot / U.ca;
  U.h1x = -U.f.ry - U.tana * U.f.rx;
  U.h1y = U.f.rx - U.tana * U.f.ry;
  U.h2x = -U.q * U.f.rx;
  U.h2y = -U.q * U.f.ry;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    U.A1[j] = U.h1x * C[tri(0, j)] + U.h1y * C[tri(1, j)];
    U.A2[j] = U.h2x * C[tri(0, j)] + U.h2y * C[tri(1, j)] + C[tri(2, j)];
  }
  const T S11 = U.A1[0] * U.h1x + U.A1[1] * U.h1y + k.v_rphi;
  const T S12 = U.A1[0] * U.h2x + U.A1[1] * U.h2y + U.A1[2];
  const T S22 = U.A2[0] * U.h2x + U.A2[1] * U.h2y + U.A2[2] + k.v_z;
  if constexpr (sizeof(T) == 4) {
    // the forward fit's inverse: equilibrated to unit diagonal, with its condition check
    // and the FP64 path, so that the sweep differentiates the S^-1 the fit used
    const T d1 = T(1) / sqrt(S11), d2 = T(1) / sqrt(S22);
    const T r12 = S12 * d1 * d2;
    const T det = T(1) - r12 * r12;
    if (det >= k.det_thr) {
      const T idet = T(1) / det;
      U.Si11 = d1 * d1 * idet;
      U.Si22 = d2 * d2 * idet;
      U.Si12 = -r12 * d1 * d2 * idet;
    } else {
      const double s11 = S11, s12 = S12, s22 = S22;
      const double dd = s11 * s22 - s12 * s12;
      U.Si11 = (T)(s22 / dd);
      U.Si22 = (T)(s11 / dd);
      U.Si12 = (T)(-s12 / dd);
    }
  } else {
    const T det = S11 * S22 - S12 * S12;
    U.Si11 = S22 / det;
    U.Si22 = S11 / det;
    U.Si12 = -S12 / det;
  }
  U.Si00 = T(1) / k.v_r;
  U.dx = mx - x[0];
  U.dy = my - x[1];
  const T rd = U.f.rx * U.dx + U.f.ry * U.dy;
  U.Y = U.f.rx * U.dy - U.f.ry * U.dx;
  U.X = U.f.rho + rd;
  U.psi = atan2(U.Y, U.X);
  U.r1 = U.f.rho * U.psi;
  U.r2 = mz - x[2];
  U.mex = mx - ly.cx;
  U.mey = my - ly.cy;
  U.rm = sqrt(U.mex * U.mex + U.mey * U.mey);
  U.r0 = U.rm - U.f.rho;
  U.g1 = U.Si11 * U.r1 + U.Si12 * U.r2;
  U.g2 = U.Si12 * U.r1 + U.Si22 * U.r2;
  const T chi2 = U.r1 * U.g1 + U.r2 * U.g2 + U.Si00 * U.r0 * U.r0;
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] += U.A1[i] * U.g1 + U.A2[i] * U.g2;
  // C - A^T S^-1 A
  T W1[6], W2[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    W1[i] = U.Si11 * U.A1[i] + U.Si12 * U.A2[i];
    W2[i] = U.Si12 * U.A1[i] + U.Si22 * U.A2[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) C[tri(i, j)] -= U.A1[i] * W1[j] + U.A2[i] * W2[j];
  return chi2;
}

// Seed: helix through three placed hits (tape and state).
template <class T>
struct Seed {
  T ax, ay, bx, by, cx, cy, la, lb, lc, cr, w, qa, qc, g, gd, arc, dz;
};

template <class T>
KFA_HD void seed(const T m0[3], const T m1[3], const T m2[3], const Consts<T>& k, Seed<T>& E, T x[6]) {
  using std::asin; using std::atan2; using std::sqrt; using std::fabs;
  E.ax = m1[0] - m0[0];
  E.ay = m1[1] - m0[1];
  E.bx = m2[0] - m1[0];
  E.by = m2[1] - m1[1];
  E.cx = m2[0] - m0[0];
  E.cy = m2[1] - m0[1];
  E.la = sqrt(E.ax * E.ax + E.ay * E.ay);
  E.lb = sqrt(E.bx * E.bx + E.by * E.by);
  E.lc = sqrt(E.cx * E.cx + E.cy * E.cy);
  E.cr = E.ax * E.by - E.ay * E.bx;
  E.w = T(2) * E.cr / (E.la * E.lb * E.lc);
  E.qa = T(0.5) * E.w * E.la;
  E.qc = T(0.5) * E.w * E.lc;
  const T q2 = E.qc * E.qc;
  if (fabs(E.qc) < T(1e-2)) {  // asin(q)/q and its derivative, by their series
    E.g = T(1) + q2 * (T(1) / T(6) + q2 * T(0.075));
    E.gd = E.qc * (T(1) / T(3) + q2 * T(0.3));
  } else {
    E.g = asin(E.qc) / E.qc;
    E.gd = (E.qc / sqrt(T(1) - q2) - asin(E.qc)) / q2;
  }
  E.arc = E.lc * E.g;
  E.dz = m2[2] - m0[2];
  x[0] = m0[0];
  x[1] = m0[1];
  x[2] = m0[2];
  x[3] = -E.w / k.kB;
  x[4] = atan2(E.ay, E.ax) - asin(E.qa);
  x[5] = atan2(E.arc, E.dz);
}

// ---------------------------------------------------------------------------------
// adjoints
// ---------------------------------------------------------------------------------

// Adjoint of the frame: rho and r_hat from e = p - c.
template <class T>
KFA_HD void frame_adj(const Frm<T>& f, T rhob, T rxb, T ryb, T& pxb, T& pyb, T& cxb, T& cyb) {
  const T rr = rxb * f.rx + ryb * f.ry;
  const T ebx = rhob * f.rx + (rxb - rr * f.rx) / f.rho;
  const T eby = rhob * f.ry + (ryb - rr * f.ry) / f.rho;
  pxb += ebx;
  pyb += eby;
  cxb -= ebx;
  cyb -= eby;
}

// Adjoint of update: in xb/Cb the adjoints of the updated state; out the adjoints of
// the predicted state.  chib: d loss / d chi2.  Adds to m*b (placed hit) and c*b.
template <class T>
KFA_HD void update_adj(const T x[6], const T C[21], const Upd<T>& U, T chib, T xb[6], T Cb[21], T& mxb, T& myb,
                       T& mzb, T& cxb, T& cyb) {
  using std::cos; using std::sin;
  // x+ = x + A^T g
  T A1b[6], A2b[6];
  T g1b = 0, g2b = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    A1b[j] = U.g1 * xb[j];
    A2b[j] = U.g2 * xb[j];
    g1b += U.A1[j] * xb[j];
    g2b += U.A2[j] * xb[j];
  }
  // chi2 = r^T Si r + Si00 r0^2 ; g = Si r
  T r1b = T(2) * chib * U.g1 + U.Si11 * g1b + U.Si12 * g2b;
  T r2b = T(2) * chib * U.g2 + U.Si12 * g1b + U.Si22 * g2b;
  const T r0b = T(2) * chib * U.Si00 * U.r0;
  // Si adjoint (symmetrised): chi2 term r r^T, g term sym(gb r^T)
  T Sb11 = chib * U.r1 * U.r1 + g1b * U.r1;
  T Sb22 = chib * U.r2 * U.r2 + g2b * U.r2;
  T Sb12 = chib * U.r1 * U.r2 + T(0.5) * (g1b * U.r2 + g2b * U.r1);
  // C+ = C - A^T Si A : Cb passes; Ab += -2 Si A Cb+ ; Sib += -A Cb+ A^T
  T AC1[6], AC2[6];  // A Cb+ (rows)
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    T s1 = 0, s2 = 0;
#pragma unroll
    for (int kk = 0; kk < 6; ++kk) {
      s1 += U.A1[kk] * Cb[tri(kk, j)];
      s2 += U.A2[kk] * Cb[tri(kk, j)];
    }
    AC1[j] = s1;
    AC2[j] = s2;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    A1b[j] -= T(2) * (U.Si11 * AC1[j] + U.Si12 * AC2[j]);
    A2b[j] -= T(2) * (U.Si12 * AC1[j] + U.Si22 * AC2[j]);
  }
  T q11 = 0, q12 = 0, q22 = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    q11 += AC1[j] * U.A1[j];
    q12 += AC1[j] * U.A2[j];
    q22 += AC2[j] * U.A2[j];
  }
  Sb11 -= q11;
  Sb12 -= q12;
  Sb22 -= q22;
  // S = H C H^T + V : Sb_S = -Si Sb Si
  const T t11 = U.Si11 * Sb11 + U.Si12 * Sb12, t12 = U.Si11 * Sb12 + U.Si12 * Sb22;
  const T t21 = U.Si12 * Sb11 + U.Si22 * Sb12, t22 = U.Si12 * Sb12 + U.Si22 * Sb22;
  const T SS11 = -(t11 * U.Si11 + t12 * U.Si12);
  const T SS12 = -(t11 * U.Si12 + t12 * U.Si22);
  const T SS22 = -(t21 * U.Si12 + t22 * U.Si22);
  // H rows as 3-vectors on (x, y, z) (other columns zero)
  const T H1[3] = {U.h1x, U.h1y, T(0)};
  const T H2[3] = {U.h2x, U.h2y, T(1)};
  // Cb += H^T SS H (positions block) ; Hb += 2 SS H C
  // plus A = H C : Cb += sym(H^T Ab), Hb += Ab C
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      Cb[tri(i, j)] += SS11 * H1[i] * H1[j] + SS12 * (H1[i] * H2[j] + H2[i] * H1[j]) + SS22 * H2[i] * H2[j];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T v = 0;
      if (j < 3) v += H1[j] * A1b[i] + H2[j] * A2b[i];
      if (i < 3) v += H1[i] * A1b[j] + H2[i] * A2b[j];
      Cb[tri(i, j)] += T(0.5) * v;
    }
  // Hb for the variable entries h1x, h1y, h2x, h2y (columns x, y)
  T h1xb = 0, h1yb = 0, h2xb = 0, h2yb = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    h1xb += A1b[j] * C[tri(0, j)];
    h1yb += A1b[j] * C[tri(1, j)];
    h2xb += A2b[j] * C[tri(0, j)];
    h2yb += A2b[j] * C[tri(1, j)];
  }
  {  // 2 SS H C, rows 1, 2 over columns x, y
    T HC1x = 0, HC1y = 0, HC2x = 0, HC2y = 0;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
      HC1x += H1[kk] * C[tri(kk, 0)];
      HC1y += H1[kk] * C[tri(kk, 1)];
      HC2x += H2[kk] * C[tri(kk, 0)];
      HC2y += H2[kk] * C[tri(kk, 1)];
    }
    h1xb += T(2) * (SS11 * HC1x + SS12 * HC2x);
    h1yb += T(2) * (SS11 * HC1y + SS12 * HC2y);
    h2xb += T(2) * (SS12 * HC1x + SS22 * HC2x);
    h2yb += T(2) * (SS12 * HC1y + SS22 * HC2y);
  }
  // H entries -> r_hat, t, cot
  const Frm<T>& f = U.f;
  T rxb = 0, ryb = 0, rhob = 0, txb = 0, tyb = 0;
  const T tanab = -h1xb * f.rx - h1yb * f.ry;
  const T qb = -h2xb * f.rx - h2yb * f.ry;
  rxb += -U.tana * h1xb + h1yb - U.q * h2xb;
  ryb += -h1xb - U.tana * h1yb - U.q * h2yb;
  const T sab = tanab / U.ca;
  T cab = -tanab * U.sa / (U.ca * U.ca) - qb * U.cot / (U.ca * U.ca);
  const T cotb = qb / U.ca;
  rxb += sab * U.ty + cab * U.tx;
  ryb += -sab * U.tx + cab * U.ty;
  txb += -sab * f.ry + cab * f.rx;
  tyb += sab * f.rx + cab * f.ry;
  const T st = sin(x[5]);
  T thb = -cotb / (st * st);
  T phb = -txb * U.ty + tyb * U.tx;
  // residual r1 = rho psi, psi = atan2(Y, X), X = rho + r_hat.d, Y = r_hat x d, d = m - p
  rhob += r1b * U.psi;
  const T psib = r1b * f.rho;
  const T den = U.X * U.X + U.Y * U.Y;
  const T Yb = psib * U.X / den, Xb = -psib * U.Y / den;
  rhob += Xb;
  const T rdb = Xb;
  rxb += Yb * U.dy + rdb * U.dx;
  ryb += -Yb * U.dx + rdb * U.dy;
  const T dxb = -Yb * f.ry + rdb * f.rx;
  const T dyb = Yb * f.rx + rdb * f.ry;
  mxb += dxb;
  myb += dyb;
  T pxb = -dxb, pyb = -dyb;
  // r2 = mz - z
  mzb += r2b;
  xb[2] -= r2b;
  // r0 = |m - c| - rho
  mxb += r0b * U.mex / U.rm;
  myb += r0b * U.mey / U.rm;
  cxb -= r0b * U.mex / U.rm;
  cyb -= r0b * U.mey / U.rm;
  rhob -= r0b;
  frame_adj(f, rhob, rxb, ryb, pxb, pyb, cxb, cyb);
  xb[0] += pxb;
  xb[1] += pyb;
  xb[4] += phb;
  xb[5] += thb;
}

// Adjoint of the scattering noise: Cb (of C + Q) is unchanged; adds to xb, the frame
// (through cos alpha), cxb/cyb and the material adjoint.  xeb_more: an adjoint of the
// path length x_e = x/X0 / (sin theta |cos alpha|) from elsewhere (the energy loss),
// passed on with the scattering's own.
template <class T>
KFA_HD void scatter_adj(const T x[6], const Frm<T>& f, const Lay<T>& ly, const Consts<T>& k, const Scat<T>& Q,
                        const T Cb[21], T xb[6], T& cxb, T& cyb, T& xX0b, T xeb_more = T(0)) {
  using std::fabs;
  if (!Q.on) return;
  const T kap = x[3];
  const T kc = kap * Q.cota;
  // L = Cb44 th2/st^2 + Cb55 th2 + Cb33 kc^2 th2 - 2 Cb35 kc th2
  const T c44 = Cb[tri(4, 4)], c55 = Cb[tri(5, 5)], c33 = Cb[tri(3, 3)], c35 = Cb[tri(5, 3)];
  const T G = c44 / (Q.st * Q.st) + c55 + c33 * kc * kc - T(2) * c35 * kc;
  const T kcb = Q.th2 * (T(2) * c33 * kc - T(2) * c35);
  T stb = -T(2) * c44 * Q.th2 / (Q.st * Q.st * Q.st);
  T kapb = kcb * Q.cota;
  T cotb = kcb * kap;
  // th2 = A0^2 ks^2 (1 + m^2 ks^2) xe lg^2
  const T ks2 = Q.ks * Q.ks;
  const T ksb = G * Q.th2 * (T(2) / Q.ks + T(2) * k.mass2 * Q.ks / (T(1) + k.mass2 * ks2));
  const T xeb = G * Q.th2 / Q.xe * (T(1) + T(0.076) / Q.lg) + xeb_more;  // (xeb_more: the energy loss's)
  kapb += ksb * Q.st;
  stb += ksb * kap;
  // xe = xX0 / (st |ca|)
  xX0b += xeb * Q.xe / ly.xX0;
  stb += -xeb * Q.xe / Q.st;
  const T cab = -xeb * Q.xe / Q.ca;  // d|ca|/dca = sign(ca): xe/|ca| * sign = xe/ca
  // cot = ct/st
  T thb = -cotb / (Q.st * Q.st) + stb * Q.ct;
  // ca = r_hat . t
  const T rxb = cab * Q.tx, ryb = cab * Q.ty;
  const T txb = cab * f.rx, tyb = cab * f.ry;
  T pxb = 0, pyb = 0;
  frame_adj(f, T(0), rxb, ryb, pxb, pyb, cxb, cyb);
  xb[0] += pxb;
  xb[1] += pyb;
  xb[3] += kapb;
  xb[4] += -txb * Q.ty + tyb * Q.tx;
  xb[5] += thb;
}

// Adjoint of the propagation step: in xb/Cb the adjoints at the end, out at the start;
// adds the adjoint of the layer axis and, if kBb is given, returns the adjoint of the
// step's k_B (which enters through omega = -k_B kappa, the arc that omega fixes, and
// the Jacobian's d(x, y)/dkappa and dphi/dkappa).
template <class T>
KFA_HD void propagate_adj(const T x[6], const T C[21], const T B[6][6], const Prop<T>& P, const Consts<T>& k,
                          T xb[6], T Cb[21], T& cxb, T& cyb, T* kBb = nullptr) {
  // J-bar = 2 Cb' J C = 2 Cb' B (only the six variable entries)
  auto jb = [&](int i, int j) {
    T s = 0;
#pragma unroll
    for (int kk = 0; kk < 6; ++kk) s += Cb[tri(i, kk)] * B[kk][j];
    return T(2) * s;
  };
  const T b04 = jb(0, 4), b14 = jb(1, 4), b03 = jb(0, 3), b13 = jb(1, 3), b25 = jb(2, 5), b43 = jb(4, 3);
  // Cb_start = J^T Cb' J
  T Y[6][6];  // Cb' J
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < 6; ++j) Y[i][j] = Cb[tri(i, j)];
    Y[i][3] += Cb[tri(i, 0)] * P.a03 + Cb[tri(i, 1)] * P.a13 + Cb[tri(i, 4)] * P.a43;
    Y[i][4] += Cb[tri(i, 0)] * P.a04 + Cb[tri(i, 1)] * P.a14;
    Y[i][5] += Cb[tri(i, 2)] * P.a25;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      T v = Y[i][j];
      if (i == 3) v += P.a03 * Y[0][j] + P.a13 * Y[1][j] + P.a43 * Y[4][j];
      if (i == 4) v += P.a04 * Y[0][j] + P.a14 * Y[1][j];
      if (i == 5) v += P.a25 * Y[2][j];
      Cb[tri(i, j)] = v;
    }
  // x' = f(x, s):  xb_start = J^T xb' ; sb = df/ds . xb'
  const T xe0 = xb[0], xe1 = xb[1], xe2 = xb[2], xe4 = xb[4];
  T sb = xe0 * P.cpe + xe1 * P.spe + xe2 * P.ct / P.st + xe4 * P.w;
  xb[3] += P.a03 * xe0 + P.a13 * xe1 + P.a43 * xe4;
  xb[4] += P.a04 * xe0 + P.a14 * xe1;
  xb[5] += P.a25 * xe2;
  // J-bar through the displacement, F1, F2, theta and s
  T phb = 0, wb = 0, thb = 0, ub = 0;
  // a04 = -dy, a14 = dx
  const T dxb = b14, dyb = -b04;
  phb += -P.dy * dxb + P.dx * dyb;
  const T s2 = P.s * P.s;
  const T vx = P.F1 * P.cp - P.F2 * P.sp, vy = P.F1 * P.sp + P.F2 * P.cp;  // F1 t + F2 n
  T kBx = 0;  // explicit k_B of the Jacobian terms (a03, a13, a43)
  {
    wb += s2 * (vx * dxb + vy * dyb);
    sb += P.cpe * dxb + P.spe * dyb;
    // (a03, a13) = -kB s^2 (F1 t + F2 n)
    phb += -b03 * P.a13 + b13 * P.a03;
    const T vt = b03 * P.cp + b13 * P.sp, vn = -b03 * P.sp + b13 * P.cp;
    const T F1b = -k.kB * s2 * vt, F2b = -k.kB * s2 * vn;
    sb += -T(2) * k.kB * P.s * (P.F1 * vt + P.F2 * vn);
    ub += F1b * P.F1d + F2b * P.F2d;
    kBx += -s2 * (P.F1 * vt + P.F2 * vn);
  }
  sb += -b25 / (P.st * P.st);
  thb += b25 * T(2) * P.s * P.ct / (P.st * P.st * P.st);
  sb += -k.kB * b43;
  kBx += -P.s * b43;
  // u = omega s
  wb += P.s * ub;
  sb += P.w * ub;
  // s(x, c) from |p(s) - c|^2 = r^2: ds/dx_i = -e'.(dp'/dx_i)/Ds, ds/dc = e'/Ds
  const T is = sb / P.Ds;
  xb[0] += -P.ex * is;
  xb[1] += -P.ey * is;
  xb[3] += -(P.ex * P.a03 + P.ey * P.a13) * is;
  xb[4] += -(P.ex * P.a04 + P.ey * P.a14) * is;
  cxb += P.ex * is;
  cyb += P.ey * is;
  xb[3] += -k.kB * wb;
  xb[4] += phb;
  xb[5] += thb;
  if (kBb) {
    // every kappa term above is -kB times an omega adjoint: the end state's (x, y) and
    // phi at fixed arc, the Jacobian's displacement and turning terms (wb), and the
    // arc's implicit dependence; k_B takes -kappa times the same sum
    const T wall = s2 * (vx * xe0 + vy * xe1) + P.s * xe4 + wb - s2 * (P.ex * vx + P.ey * vy) * is;
    *kBb += -x[3] * wall + kBx;
  }
}

// Adjoint of the seed: state adjoint -> adjoints of the three placed hits.
template <class T>
KFA_HD void seed_adj(const Seed<T>& E, const Consts<T>& k, const T xb[6], T m0b[3], T m1b[3], T m2b[3]) {
  using std::sqrt;
  m0b[0] += xb[0];
  m0b[1] += xb[1];
  m0b[2] += xb[2];
  // theta = atan2(arc, dz)
  const T den = E.arc * E.arc + E.dz * E.dz;
  const T arcb = xb[5] * E.dz / den;
  const T dzb = -xb[5] * E.arc / den;
  m2b[2] += dzb;
  m0b[2] -= dzb;
  // arc = lc g(qc), qc = w lc / 2
  T lcb = arcb * E.g;
  const T qcb = arcb * E.lc * E.gd;
  T wb = qcb * T(0.5) * E.lc;
  lcb += qcb * T(0.5) * E.w;
  // phi0 = atan2(ay, ax) - asin(qa), qa = w la / 2
  const T la2 = E.la * E.la;
  T axb = -xb[4] * E.ay / la2, ayb = xb[4] * E.ax / la2;
  const T qab = -xb[4] / sqrt(T(1) - E.qa * E.qa);
  wb += qab * T(0.5) * E.la;
  T lab = qab * T(0.5) * E.w;
  // kappa = -w / kB
  wb += -xb[3] / k.kB;
  // w = 2 cr / (la lb lc)
  const T crb = wb * T(2) / (E.la * E.lb * E.lc);
  lab += -wb * E.w / E.la;
  T lbb = -wb * E.w / E.lb;
  lcb += -wb * E.w / E.lc;
  axb += crb * E.by + lab * E.ax / E.la;
  ayb += -crb * E.bx + lab * E.ay / E.la;
  T bxb = -crb * E.ay + lbb * E.bx / E.lb;
  T byb = crb * E.ax + lbb * E.by / E.lb;
  const T cxb = lcb * E.cx / E.lc, cyb = lcb * E.cy / E.lc;
  m1b[0] += axb - bxb;
  m1b[1] += ayb - byb;
  m0b[0] -= axb + cxb;
  m0b[1] -= ayb + cyb;
  m2b[0] += bxb + cxb;
  m2b[1] += byb + cyb;
}

// Adjoint of placing a nominal-frame hit h on its layer: m = c + R(dphi) h, mz = hz + dz.
template <class T>
KFA_HD void place_adj(const Lay<T>& ly, T hx, T hy, T mxb, T myb, T mzb, T g[5]) {
  g[0] += mxb;
  g[1] += myb;
  g[2] += mzb;
  g[3] += mxb * (-ly.sphi * hx - ly.cphi * hy) + myb * (ly.cphi * hx - ly.sphi * hy);
}

}  // namespace kfa

namespace kfa {

// Seed covariance (a constant of the geometry): ten times the diagonal prior.
template <class T>
KFA_HD void seed_cov(T srphi, T sz, T dr02, T kB, T C[21]) {
  using std::sqrt;
  const T sphi = sqrt(T(2)) * srphi / dr02, sth = sqrt(T(2)) * sz / dr02;
  const T skap = T(8) * sqrt(T(1.5)) * srphi / (dr02 * dr02 * kB);
  for (int q = 0; q < 21; ++q) C[q] = T(0);
  C[tri(0, 0)] = T(10) * srphi * srphi;
  C[tri(1, 1)] = T(10) * srphi * srphi;
  C[tri(2, 2)] = T(10) * sz * sz;
  C[tri(3, 3)] = T(10) * skap * skap;
  C[tri(4, 4)] = T(10) * sphi * sphi;
  C[tri(5, 5)] = T(10) * sth * sth;
}

// The parameterised field B_z(r, z) = B (1 + fr r^2 + fz z^2) (Sec. 3), with what the
// seed covariance needs to follow it.  Each step takes the field at its start and the
// seed at its first hit; those points move with the parameters, and the sweep carries
// the field's change with them (field_adj).
template <class T>
struct FieldK {
  T fr, fz;
  T srphi, sz, dr02;
};

template <class T>
KFA_HD T field_kB(const Consts<T>& k, const FieldK<T>& f, T x, T y, T z) {
  return k.kB * (T(1) + f.fr * (x * x + y * y) + f.fz * z * z);
}

// Adjoint of field_kB at (x, y, z): adds kBb dk_B/d(x, y, z).
template <class T>
KFA_HD void field_adj(const Consts<T>& k, const FieldK<T>& f, T x, T y, T z, T kBb, T& xb, T& yb, T& zb) {
  const T g = T(2) * k.kB * kBb;
  xb += g * f.fr * x;
  yb += g * f.fr * y;
  zb += g * f.fz * z;
}

template <class T>
KFA_HD void place(const Lay<T>& ly, T hx, T hy, T hz, T m[3]) {
  m[0] = ly.cx + ly.cphi * hx - ly.sphi * hy;
  m[1] = ly.cy + ly.sphi * hx + ly.cphi * hy;
  m[2] = hz + ly.dz;
}

// ---------------------------------------------------------------------------------
// the detector model of Sec. 3 in the sweep: material map and mean energy loss
// ---------------------------------------------------------------------------------

// A material map [L][nz] (float32, null: each layer's x/X0) and the mean ionisation loss
// per radiation length (0: none).
template <class T>
struct MatK {
  const float* map;
  int nz;
  T eloss;
};

// x/X0 of a layer at z from its map row, as the fit reads it (linear between the centres
// of nz equal bins over the layer's frame, constant beyond the outer centres), and its
// slope in z (0 beyond the centres).
template <class T>
KFA_HD T map_lookup(const float* row, int nz, const Lay<T>& ly, T z, T& slope) {
  slope = T(0);
  if (nz == 1) return (T)row[0];
  const T u0 = (z - ly.dz) * ly.zs + ly.zo;
  const T u = u0 < T(0) ? T(0) : (u0 > T(nz - 1) ? T(nz - 1) : u0);
  int b = (int)u;
  if (b > nz - 2) b = nz - 2;
  const T t = u - (T)b;
  const T v0 = (T)row[b], d = (T)row[b + 1] - v0;
  if (u0 > T(0) && u0 < T(nz - 1)) slope = d * ly.zs;
  return v0 + t * d;
}

// A value with its derivatives in three variables (forward mode), for the Jacobian of
// the energy loss's local map below.
template <class T>
struct D3 {
  T v, d[3];
};
template <class T>
KFA_HD D3<T> d3(T v, int i) {
  D3<T> r{v, {T(0), T(0), T(0)}};
  if (i >= 0) r.d[i] = T(1);
  return r;
}
template <class T> KFA_HD T vof(const D3<T>& a) { return a.v; }
template <class T> KFA_HD T vof(T a) { return a; }
template <class T> KFA_HD D3<T> operator+(const D3<T>& a, const D3<T>& b) { return {a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1], a.d[2] + b.d[2]}}; }
template <class T> KFA_HD D3<T> operator-(const D3<T>& a, const D3<T>& b) { return {a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1], a.d[2] - b.d[2]}}; }
template <class T> KFA_HD D3<T> operator*(const D3<T>& a, const D3<T>& b) {
  return {a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1], a.d[2] * b.v + a.v * b.d[2]}};
}
template <class T> KFA_HD D3<T> operator*(const D3<T>& a, T b) { return {a.v * b, {a.d[0] * b, a.d[1] * b, a.d[2] * b}}; }
template <class T> KFA_HD D3<T> operator*(T b, const D3<T>& a) { return a * b; }
template <class T> KFA_HD D3<T> operator+(const D3<T>& a, T b) { return {a.v + b, {a.d[0], a.d[1], a.d[2]}}; }
template <class T> KFA_HD D3<T> operator+(T b, const D3<T>& a) { return a + b; }
template <class T> KFA_HD D3<T> operator-(const D3<T>& a, T b) { return {a.v - b, {a.d[0], a.d[1], a.d[2]}}; }
template <class T> KFA_HD D3<T> inv(const D3<T>& a) {
  const T r = T(1) / a.v, r2 = -r * r;
  return {r, {a.d[0] * r2, a.d[1] * r2, a.d[2] * r2}};
}
template <class T> KFA_HD D3<T> operator/(const D3<T>& a, const D3<T>& b) { return a * inv(b); }
template <class T> KFA_HD D3<T> operator/(T a, const D3<T>& b) { return inv(b) * a; }
template <class T> KFA_HD D3<T> sqrt(const D3<T>& a) {
  using std::sqrt;
  const T s = sqrt(a.v), h = T(0.5) / s;
  return {s, {a.d[0] * h, a.d[1] * h, a.d[2] * h}};
}
template <class T> KFA_HD D3<T> fabs(const D3<T>& a) { return a.v < T(0) ? a * T(-1) : a; }
template <class T> KFA_HD void sin_cos(const D3<T>& a, D3<T>& s, D3<T>& c) {
  T sv, cv;
  sin_cos(a.v, sv, cv);
  s = {sv, {a.d[0] * cv, a.d[1] * cv, a.d[2] * cv}};
  c = {cv, {-a.d[0] * sv, -a.d[1] * sv, -a.d[2] * sv}};
}

// The mean energy loss over a path of xe radiation lengths as a map of kappa (the fit's:
// p = 1 / (|kappa| sin theta), E = p sqrt(1 + m^2 / p^2), dE = eloss xe / beta^2,
// E1 = E - dE, kappa1 = kappa p / p1), with its derivatives D = dkappa1/dkappa and
// Tt = dkappa1/dtheta at fixed xe (the covariance's linearisation), evaluated as the fit
// evaluates them.  S = T, or D3<T> to differentiate (kappa1, D, Tt) in (kappa, theta, xe).
// False if the particle stops.
template <class S, class T>
KFA_HD bool loss_kappa(const S& kap, const S& th, const S& xe, T eloss, T mass2, S& k1, S& D, S& Tt) {
  using std::fabs; using std::sqrt;
  S st, ct;
  sin_cos(th, st, ct);
  const S ks = fabs(kap) * st;
  const S p = T(1) / ks;
  const S c = xe * eloss;
  const S ib2 = T(1) + ks * ks * mass2;
  const S E = p * sqrt(ib2);
  const S dE = c * ib2;
  const S E1 = E - dE;
  const S q2 = E1 * E1 - mass2;
  if (!(vof(E1) > T(0)) || !(vof(q2) > T(0))) return false;
  const S ip1 = T(1) / sqrt(q2);
  const S X = dE * (mass2 / E + E1) + T(2) * mass2 * c * E1 * ks * ks;
  const S W = p * X * (ip1 * ip1 * ip1);
  const S g = p * ip1;
  D = g + W;
  Tt = kap * (ct / st) * W;
  k1 = g * kap;
  return true;
}

// Tape of a step's material beyond the scattering: the map's slope at the crossing and
// the loss's Jacobian J[o][i] of (kappa1, D, Tt) in (kappa, theta, x_e).
template <class T>
struct MatT {
  T xx, slope;   // x/X0 at the crossing and its slope in z (map)
  bool loss;
  T D, Tt, J[3][3];
};

// The step's material after its transport (x, C: the transported state and covariance):
// x/X0 (from the map's row of layer l, else the layer's), the scattering term, then the
// energy loss on kappa with C <- A C A^T (A the identity but for kappa's row: D at
// kappa, Tt at theta).  Cl receives C before the loss.  False if the particle stops.
template <class T>
KFA_HD bool material_fwd(int l, const Lay<T>& ly, const Consts<T>& k, const MatK<T>* mk, const Frm<T>& fr, T x[6],
                         T C[21], Scat<T>& Q, MatT<T>& M, T Cl[21]) {
  Lay<T> lym = ly;
  M.slope = T(0);
  M.loss = false;
  if (mk && mk->map) lym.xX0 = map_lookup(mk->map + (int64_t)l * mk->nz, mk->nz, ly, x[2], M.slope);
  M.xx = lym.xX0;
  scatter(x, fr, lym, k, Q, C);
  if (!mk || !(mk->eloss > T(0)) || !(M.xx > T(0))) return true;
  D3<T> k1, D, Tt;
  if (!loss_kappa(d3(x[3], 0), d3(x[5], 1), d3(Q.xe, 2), mk->eloss, k.mass2, k1, D, Tt)) return false;
  M.loss = true;
  M.D = D.v;
  M.Tt = Tt.v;
  for (int i = 0; i < 3; ++i) {
    M.J[0][i] = k1.d[i];
    M.J[1][i] = D.d[i];
    M.J[2][i] = Tt.d[i];
  }
  for (int q = 0; q < 21; ++q) Cl[q] = C[q];
  const T c53 = C[tri(5, 3)], c55 = C[tri(5, 5)], c33 = C[tri(3, 3)];
  for (int j = 0; j < 6; ++j)
    if (j != 3 && j != 5) C[tri(3, j)] = M.D * C[tri(3, j)] + M.Tt * C[tri(5, j)];
  C[tri(5, 3)] = M.D * c53 + M.Tt * c55;
  C[tri(3, 3)] = M.D * M.D * c33 + T(2) * M.D * M.Tt * c53 + M.Tt * M.Tt * c55;
  x[3] = k1.v;
  return true;
}

// Adjoint of the energy loss: xb, Cb of (x, C) after the loss in, of them before it out
// (x: the state before the loss; Cl: C before it); returns the adjoint of x_e.  The
// covariance map C' = A C A^T gives C-bar = A^T C'-bar A and A-bar = 2 C'-bar A C.
template <class T>
KFA_HD T loss_adj(const T x[6], const T Cl[21], const MatT<T>& M, T xb[6], T Cb[21]) {
  T CbF[6][6], AC3[6], AC5[6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) CbF[i][j] = Cb[tri(i, j)];
  // columns 3 and 5 of A C (only A's row 3 differs from the identity)
  for (int kk = 0; kk < 6; ++kk) {
    AC3[kk] = kk == 3 ? M.D * Cl[tri(3, 3)] + M.Tt * Cl[tri(5, 3)] : Cl[tri(kk, 3)];
    AC5[kk] = kk == 3 ? M.D * Cl[tri(3, 5)] + M.Tt * Cl[tri(5, 5)] : Cl[tri(kk, 5)];
  }
  T Db = T(0), Ttb = T(0);
  for (int kk = 0; kk < 6; ++kk) {
    Db += CbF[3][kk] * AC3[kk];
    Ttb += CbF[3][kk] * AC5[kk];
  }
  Db *= T(2);
  Ttb *= T(2);
  // C-bar = A^T C'-bar A: column i of A is e_i, but D e_3 for i = 3 and e_5 + Tt e_3
  // for i = 5
  T V[6][6];  // C'-bar A
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j)
      V[i][j] = j == 3 ? M.D * CbF[i][3] : (j == 5 ? CbF[i][5] + M.Tt * CbF[i][3] : CbF[i][j]);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j <= i; ++j) {
      auto col = [&](int r, int c) {  // (A^T V)(r, c) = sum_k A(k, r) V(k, c)
        return r == 3 ? M.D * V[3][c] : (r == 5 ? V[5][c] + M.Tt * V[3][c] : V[r][c]);
      };
      Cb[tri(i, j)] = col(i, j);
    }
  // kappa1, D, Tt in (kappa, theta, x_e)
  const T k1b = xb[3];
  xb[3] = k1b * M.J[0][0] + Db * M.J[1][0] + Ttb * M.J[2][0];
  xb[5] += k1b * M.J[0][1] + Db * M.J[1][1] + Ttb * M.J[2][1];
  (void)x;
  return k1b * M.J[0][2] + Db * M.J[1][2] + Ttb * M.J[2][2];
}

// One forward step of the fit, in place, from the filtered estimate after layer l - 1
// to the one after layer l: propagation, transport, the layer's scattering and, where
// the track has a hit on l (mask bit l), the update; under a parameterised field (fk)
// the helix of the field at the step's start.  The adjoint uses it to recompute the
// layers between sparse checkpoints.  False if layer l is not reached.
template <class T, class Hit>
KFA_HD bool forward_step(int l, uint32_t mask, const Lay<T>* lays, const Consts<T>& k, const FieldK<T>* fk, Hit hit,
                         T x[6], T C[21], const MatK<T>* mk = nullptr) {
  const Lay<T>& ly = lays[l];
  Consts<T> ks = k;
  if (fk) ks.kB = field_kB(k, *fk, x[0], x[1], x[2]);
  Prop<T> P;
  T xp[6];
  if (!propagate(x, ly, ks, P, xp)) return false;
  T B[6][6], Cp[21];
  transport_cov(P, C, B, Cp);
  const Frm<T> fr = frame(xp, ly);
  Scat<T> Q;
  MatT<T> M;
  T Cl[21];
  if (!material_fwd(l, ly, ks, mk, fr, xp, Cp, Q, M, Cl)) return false;
  if ((mask >> l) & 1u) {
    T h[3], m[3];
    hit(l, h);
    place(ly, h[0], h[1], h[2], m);
    Upd<T> U;
    update(xp, Cp, ly, ks, m[0], m[1], m[2], U);
  }
  for (int q = 0; q < 6; ++q) x[q] = xp[q];
  for (int q = 0; q < 21; ++q) C[q] = Cp[q];
  return true;
}

// Reverse sweep of one track.
//   hit(l, h[3])     nominal hit on layer l;
//   ckpt(l, x, C)    state and covariance after layer l of the forward fit;
//   lstart           last layer the forward updated (all layers up to it processed);
//   ltop             first layer index of the sweep (>= lstart): layers above lstart
//                    are passed over, so that lanes of a wave that start the sweep at
//                    the same ltop visit the same layer in every iteration;
//   emit(l, g[5])    gradient contribution of layer l (d/d cx, cy, dz, dphi, xX0),
//                    called once per layer from lstart down to 0, then for 1 and 2
//                    again with the seed's share;
//   fk               null: the uniform field of k, with seed covariance Cs; else the
//                    parameterised field (Cs is then recomputed for the seed's field).
// Returns false if a recomputed step fails (no contribution then).
template <class T, class Hit, class Ckpt, class Emit>
KFA_HD bool track_adjoint(int lstart, int ltop, uint32_t mask, const Lay<T>* lays, const Consts<T>& k,
                          const T Cs[21], T w, Hit hit, Ckpt ckpt, Emit emit, const FieldK<T>* fk = nullptr,
                          const MatK<T>* mk = nullptr) {
  T xb[6] = {0, 0, 0, 0, 0, 0};
  T Cb[21];
  for (int q = 0; q < 21; ++q) Cb[q] = T(0);
  for (int l = ltop; l >= 1; --l) {
    if (l > lstart) continue;
    const Lay<T>& ly = lays[l];
    T x[6], C[21];
    ckpt(l - 1, x, C);
    Consts<T> ks = k;
    if (fk) ks.kB = field_kB(k, *fk, x[0], x[1], x[2]);  // the field at the step's start
    Prop<T> P;
    T xp[6];
    if (!propagate(x, ly, ks, P, xp)) return false;
    T B[6][6], Cp[21];
    transport_cov(P, C, B, Cp);
    const Frm<T> fr = frame(xp, ly);
    Scat<T> Q;
    MatT<T> M;
    T Cl[21], xl[6];  // C and x before the energy loss (with a loss)
    for (int q = 0; q < 6; ++q) xl[q] = xp[q];
    if (!material_fwd(l, ly, ks, mk, fr, xp, Cp, Q, M, Cl)) return false;
    T g[5] = {0, 0, 0, 0, 0};
    if ((mask >> l) & 1u) {
      T h[3], m[3];
      hit(l, h);
      place(ly, h[0], h[1], h[2], m);
      Upd<T> U;
      T xu[6], Cu[21];
      for (int q = 0; q < 6; ++q) xu[q] = xp[q];
      for (int q = 0; q < 21; ++q) Cu[q] = Cp[q];
      update(xu, Cu, ly, ks, m[0], m[1], m[2], U);
      T mb[3] = {0, 0, 0};
      update_adj(xp, Cp, U, w, xb, Cb, mb[0], mb[1], mb[2], g[0], g[1]);
      place_adj(ly, h[0], h[1], mb[0], mb[1], mb[2], g);
    }
    const T xeb = M.loss ? loss_adj(xl, Cl, M, xb, Cb) : T(0);
    Lay<T> lym = ly;
    lym.xX0 = M.xx;
    T xxb = T(0);
    scatter_adj(xl, fr, lym, ks, Q, Cb, xb, g[0], g[1], xxb, xeb);
    if (mk && mk->map) {  // the map's row offset, and its slope at the crossing's z - dz
      xb[2] += xxb * M.slope;
      g[2] -= xxb * M.slope;
    }
    g[4] += xxb;
    T kBb = 0;
    propagate_adj(x, C, B, P, ks, xb, Cb, g[0], g[1], fk ? &kBb : nullptr);
    if (fk) field_adj(k, *fk, x[0], x[1], x[2], kBb, xb[0], xb[1], xb[2]);  // the step's start point
    emit(l, g);
  }
  // seed and the layer-0 update
  T h[3][3], m[3][3];
  for (int l = 0; l < 3; ++l) {
    hit(l, h[l]);
    place(lays[l], h[l][0], h[l][1], h[l][2], m[l]);
  }
  Consts<T> k0 = k;
  T Cf[21];
  const T* C0 = Cs;
  if (fk) {  // curvature from the field at the first hit, and the seed covariance with it
    k0.kB = field_kB(k, *fk, m[0][0], m[0][1], m[0][2]);
    seed_cov(fk->srphi, fk->sz, fk->dr02, k0.kB, Cf);
    C0 = Cf;
  }
  Seed<T> E;
  T xs[6];
  seed(m[0], m[1], m[2], k0, E, xs);
  Upd<T> U;
  T xu[6], Cu[21];
  for (int q = 0; q < 6; ++q) xu[q] = xs[q];
  for (int q = 0; q < 21; ++q) Cu[q] = C0[q];
  update(xu, Cu, lays[0], k0, m[0][0], m[0][1], m[0][2], U);
  T g0[5] = {0, 0, 0, 0, 0};
  T mb[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  update_adj(xs, C0, U, w, xb, Cb, mb[0][0], mb[0][1], mb[0][2], g0[0], g0[1]);
  if (fk) {
    // the seed's k_B at hit 0: kappa = -omega / k_B and the prior's C[kappa][kappa],
    // which scales as 1 / k_B^2
    const T kBb = -(xb[3] * xs[3] + T(2) * Cb[tri(3, 3)] * C0[tri(3, 3)]) / k0.kB;
    field_adj(k, *fk, m[0][0], m[0][1], m[0][2], kBb, mb[0][0], mb[0][1], mb[0][2]);
  }
  seed_adj(E, k0, xb, mb[0], mb[1], mb[2]);
  place_adj(lays[0], h[0][0], h[0][1], mb[0][0], mb[0][1], mb[0][2], g0);
  emit(0, g0);
  for (int l = 1; l < 3; ++l) {
    T gl[5] = {0, 0, 0, 0, 0};
    place_adj(lays[l], h[l][0], h[l][1], mb[l][0], mb[l][1], mb[l][2], gl);
    emit(l, gl);
  }
  return true;
}

// Last layer updated by the forward fit, from its hit count: the layer of the n-th hit.
KFA_HD int last_updated_layer(uint32_t mask, int n_hits, int nl) {
  int c = 0;
  for (int l = 0; l < nl; ++l)
    if ((mask >> l) & 1u) {
      if (++c == n_hits) return l;
    }
  return -1;
}

}  // namespace kfa
