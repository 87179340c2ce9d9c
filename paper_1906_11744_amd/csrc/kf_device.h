// Device-side Kalman step for gfx950: one track candidate per lane, state and packed
// covariance in VGPRs, FP32 arithmetic (FP64 only for an ill-conditioned S).
//
// The paper (Sec. 2) vectorises the 6x6 covariance algebra across tracks and skips
// matrix elements known to be 0 or 1.  Here every product is written out with those
// zeros removed at compile time: the transport Jacobian has six off-diagonal terms,
// the measurement matrix touches only the position columns and its radial row is zero.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kfd {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kTwoPi = 6.28318530717958647692f;

constexpr uint32_t ST_PROP_FAIL = 1u, ST_NEAR_TANGENT = 2u, ST_FP64 = 4u, ST_NONFINITE = 8u,
                   ST_BAD_INPUT = 16u, ST_TERM_MISSES = 32u;

// Hardware reciprocal, square root and reciprocal square root (v_rcp_f32, v_sqrt_f32,
// v_rsq_f32; about 1 ulp, no denormal fix-up: every operand on the path is a normal
// number or the result is not used).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float hsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float hrsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// packed lower-triangular index
__host__ __device__ constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// Per-layer constants of one launch (uniform across lanes).
struct LayerK {
  float r, cx, cy, dz, cphi, sphi, xX0;
  float moved;  // 1 if the alignment moves the layer (any of cx, cy, dz, its rotation), else 0
  float zs, zo; // material map: fractional bin u = z * zs + zo of a z in the layer's frame
  // Endcap geometry.  disk = 1: the plane z = zp (its nominal z plus dz), active for
  // lo <= rho <= hi about the axis.  A cylinder with hi > 0 is active for |z - dz| <= hi.
  // bounded = 1 for a disk or a bounded cylinder (passed over where a track has no hit).
  float disk, bounded, zp, lo, hi;
};

// Constants of the hit model and the field.
struct Model {
  float kB;        // 0.299792458e-2 * B
  float v_r, v_rphi, v_z;  // hit variances (radial regulariser, r*phi, z)
  float mass2;     // particle mass squared
  float det_thr;   // FP64 fallback threshold on det of the equilibrated S (> 1 forces)
  float dr02;      // radius[2] - radius[0], for the seed prior
};

// A track candidate: state, covariance and the carried trigonometry of phi and theta.
// The transverse position is a compensated sum x[i] + xl[i] (i < 2): at 100 cm one
// float ulp is 7.6e-6 cm, and rounding every step's increments into x alone
// random-walks the trajectory by ~3e-5 cm over 17 layers, which a 1 m sagitta turns
// into ~2e-6/GeV of curvature.  xl keeps each addition's rounding error.  z has no
// such lever (its error only tilts theta by ~1e-7): xl[2] is kept at 0.
struct Trk {
  float x[6];   // x y z kappa phi theta
  float xl[3];  // low parts of x y z
  float C[21];
  float cp, sp; // cos, sin of phi
  float ct, st; // cos, sin of theta
  float rst;    // 1 / sin(theta), kept with them (every step needs it; one reciprocal per update)
};

// x + d as a compensated sum (Knuth's two-sum; the rounding error goes to lo).  lo is
// not renormalised into x: it collects at most one half ulp of x per addition, tens of
// ulps over a track, far inside float range, and x + lo stays exact to ~1 ulp of lo.
__device__ __forceinline__ void add_pos(float& x, float& lo, float d) {
  const float s = x + d;
  const float bb = s - x;
  const float err = (x - (s - bb)) + (d - bb);
  lo += err;
  x = s;
}

// Position relative to a point, from both parts.
__device__ __forceinline__ float rel_pos(float x, float lo, float c) { return (x - c) + lo; }

__device__ __forceinline__ float wrap_pi(float a) {
  if (a > kPi) a -= kTwoPi;
  if (a <= -kPi) a += kTwoPi;
  return a;
}

// cos/sin of x[4], x[5] from scratch.
__device__ __forceinline__ void init_trig(Trk& t) {
  sincosf(t.x[4], &t.sp, &t.cp);
  sincosf(t.x[5], &t.st, &t.ct);
  t.rst = rcp(t.st);
}

// Rotate (c, s) = (cos a, sin a) to a + d; small d by its Taylor series, otherwise
// exactly from the new angle.
__device__ __forceinline__ void rotate_small(float& c, float& s, float d, float anew) {
  if (fabsf(d) < 0.03f) {
    const float d2 = d * d;
    const float cd = 1.f - d2 * (0.5f - d2 * (1.f / 24.f));
    const float sd = d * (1.f - d2 * (1.f / 6.f - d2 * (1.f / 120.f)));
    const float c2 = c * cd - s * sd;
    const float s2 = s * cd + c * sd;
    c = c2;
    s = s2;
  } else {
    sincosf(anew, &s, &c);
  }
}

// ---------------------------------------------------------------------------------
// propagation to the first forward crossing with a cylinder, and the transport
// Jacobian at fixed transverse arc applied to C (C <- J C J^T).
//
// With p0 = (x, y) - c, a = p0.t, b = p0.n, c0 = |p0|^2 - r^2 and the tangent half
// angle tau = tan(u/2) = omega * sigma, |p(s)|^2 = r^2 becomes the quadratic
// A sigma^2 + 2 a sigma + c0/2 = 0 with A = 2 + 2 omega b + omega^2 c0 / 2; its
// stable positive root is sigma = -c0 / (2 (a + sqrt(a^2 - A c0 / 2))).  Then
// s = 2 atan(tau) / omega, displacement 2 sigma / (1 + tau^2) (t + tau n), phi += u.
// ---------------------------------------------------------------------------------
struct Step {
  float s;      // transverse arc
  float tau;    // tan(u/2)
  float inv1;   // 1 / (1 + tau^2)
  float dx, dy; // transverse displacement
  float u;      // turning angle
};

__device__ __forceinline__ bool crossing(const Trk& k, const LayerK& ly, float kB, Step& st) {
  const float ex = rel_pos(k.x[0], k.xl[0], ly.cx), ey = rel_pos(k.x[1], k.xl[1], ly.cy);
  const float a = fmaf(ex, k.cp, ey * k.sp);
  const float b = fmaf(ey, k.cp, -ex * k.sp);
  const float c0 = fmaf(ex, ex, fmaf(ey, ey, -ly.r * ly.r));
  const float w = -kB * k.x[3];
  const float A = fmaf(2.f * w, b, fmaf(0.5f * w * w, c0, 2.f));
  const float D = fmaf(a, a, -0.5f * A * c0);
  if (!(c0 < 0.f) || !(D >= 0.f)) return false;
  const float den = a + hsqrt(D);
  if (!(den > 0.f)) return false;
  const float sig = -0.5f * c0 * rcp(den);
  const float tau = w * sig;
  const float tau2 = tau * tau;
  // atan(tau)/tau, exact at tau = 0: its Taylor series to tau^12 below |tau| = 0.3
  // (truncation < tau^14/15 = 3e-9), atanf beyond
  float q;
  if (fabsf(tau) < 0.3f) {
    q = fmaf(tau2, fmaf(tau2, fmaf(tau2, fmaf(tau2, fmaf(tau2, fmaf(tau2, 1.f / 13.f, -1.f / 11.f), 1.f / 9.f),
                                                      -1.f / 7.f), 0.2f), -1.f / 3.f), 1.f);
  } else {
    q = atanf(tau) / tau;
  }
  st.inv1 = rcp(1.f + tau2);
  const float f = 2.f * sig * st.inv1;
  st.s = 2.f * sig * q;
  st.u = 2.f * tau * q;
  st.tau = tau;
  st.dx = f * fmaf(-tau, k.sp, k.cp);
  st.dy = f * fmaf(tau, k.cp, k.sp);
  return true;
}

// Moves k along the step and transports its covariance with the fixed-arc Jacobian
// J = I + {d(x,y)/dphi, d(x,y)/dkappa, dz/dtheta, dphi/dkappa}.
__device__ __forceinline__ void transport(Trk& k, const Step& st, float kB) {
  const float s = st.s, u = st.u;
  float F1, F2;  // d(displacement)/d(omega) = s^2 (F1 t + F2 n)
  const float tau2 = st.tau * st.tau;
  const float inv1 = st.inv1;
  const float cu = (1.f - tau2) * inv1, su = 2.f * st.tau * inv1;
  if (fabsf(u) < 0.3f) {
    const float u2 = u * u;
    F1 = u * fmaf(u2, fmaf(u2, -1.f / 840.f, 1.f / 30.f), -1.f / 3.f);
    F2 = fmaf(u2, fmaf(u2, fmaf(u2, -1.f / 5760.f, 1.f / 144.f), -0.125f), 0.5f);
  } else {
    const float iu2 = 1.f / (u * u);
    F1 = fmaf(u, cu, -su) * iu2;
    F2 = fmaf(u, su, -2.f * tau2 * inv1) * iu2;
  }
  const float ks2 = -kB * s * s;
  const float rst = k.rst;
  const float a04 = -st.dy, a14 = st.dx;
  const float a03 = ks2 * fmaf(F1, k.cp, -F2 * k.sp);
  const float a13 = ks2 * fmaf(F1, k.sp, F2 * k.cp);
  const float a25 = -s * rst * rst;
  const float a43 = -kB * s;
  float* C = k.C;
#define CC(i, j) C[tri(i, j)]
  // B = J C (rows 0, 1, 2, 4 change)
  float B0[6], B1[6], B2[6], B4[6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    B0[j] = fmaf(a03, CC(3, j), fmaf(a04, CC(4, j), CC(0, j)));
    B1[j] = fmaf(a13, CC(3, j), fmaf(a14, CC(4, j), CC(1, j)));
    B2[j] = fmaf(a25, CC(5, j), CC(2, j));
    B4[j] = fmaf(a43, CC(3, j), CC(4, j));
  }
  // C' = B J^T, lower triangle; column j of J^T adds a_jk B[i][k]
  float R[21];
  auto Brow = [&](int i, int j) -> float {
    return i == 0 ? B0[j] : i == 1 ? B1[j] : i == 2 ? B2[j] : i == 4 ? B4[j] : CC(i, j);
  };
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R[tri(i, 0)] = fmaf(a03, Brow(i, 3), fmaf(a04, Brow(i, 4), Brow(i, 0)));
    if (i >= 1) R[tri(i, 1)] = fmaf(a13, Brow(i, 3), fmaf(a14, Brow(i, 4), Brow(i, 1)));
    if (i >= 2) R[tri(i, 2)] = fmaf(a25, Brow(i, 5), Brow(i, 2));
    if (i >= 3) R[tri(i, 3)] = Brow(i, 3);
    if (i >= 4) R[tri(i, 4)] = fmaf(a43, Brow(i, 3), Brow(i, 4));
    if (i >= 5) R[tri(i, 5)] = Brow(i, 5);
  }
#undef CC
#pragma unroll
  for (int q = 0; q < 21; ++q) C[q] = R[q];
  // state
  add_pos(k.x[0], k.xl[0], st.dx);
  add_pos(k.x[1], k.xl[1], st.dy);
  k.x[2] = fmaf(s * rst, k.ct, k.x[2]);  // z needs no compensation (xl[2] stays 0)
  k.x[4] += u;  // wrapped where it is stored: the step uses (cp, sp), not phi
  const float cp = k.cp * cu - k.sp * su;
  const float sp = k.sp * cu + k.cp * su;
  const float nrm = hrsqrt(fmaf(cp, cp, sp * sp));
  k.cp = cp * nrm;
  k.sp = sp * nrm;
}

// Propagation to the plane z = ly.zp of a disk: transverse arc s = (zp - z) tan(theta),
// which must be positive (the plane ahead) with |u| = |omega s| < pi; then tau = tan(u/2)
// and the displacement 2 sigma / (1 + tau^2) (t + tau n) with sigma = tau / omega =
// (s/2) tan(u/2) / (u/2) (its series below |u/2| = 0.1, truncation < 1e-12), the same
// Step as a cylinder crossing.
__device__ __forceinline__ bool plane_crossing(const Trk& k, const LayerK& ly, float kB, Step& st) {
  if (k.ct == 0.f) return false;
  const float s = (ly.zp - k.x[2]) * k.st * rcp(k.ct);
  if (!(s > 0.f)) return false;
  const float u = -kB * k.x[3] * s;
  if (!(fabsf(u) < kPi)) return false;
  const float v = 0.5f * u;
  float tq;  // tan(v) / v
  if (fabsf(v) < 0.1f) {
    const float v2 = v * v;
    tq = fmaf(v2, fmaf(v2, fmaf(v2, fmaf(v2, 62.f / 2835.f, 17.f / 315.f), 2.f / 15.f), 1.f / 3.f), 1.f);
  } else {
    tq = tanf(v) / v;
  }
  const float tau = v * tq;
  st.inv1 = rcp(fmaf(tau, tau, 1.f));
  const float f = s * tq * st.inv1;
  st.s = s;
  st.u = u;
  st.tau = tau;
  st.dx = f * fmaf(-tau, k.sp, k.cp);
  st.dy = f * fmaf(tau, k.cp, k.sp);
  return true;
}

// Whether the crossing of a step lies in a bounded surface's active area: a disk's
// radii, a bounded cylinder's |z - dz| <= hi (the same positions transport() reaches).
__device__ __forceinline__ bool in_area(const Trk& k, const LayerK& ly, const Step& st, bool disk) {
  if (disk) {
    const float px = rel_pos(k.x[0], k.xl[0], ly.cx) + st.dx, py = rel_pos(k.x[1], k.xl[1], ly.cy) + st.dy;
    const float rho = hsqrt(fmaf(px, px, py * py));
    return rho >= ly.lo && rho <= ly.hi;
  }
  const float z = fmaf(st.s * k.rst, k.ct, k.x[2]);
  return fabsf(z - ly.dz) <= ly.hi;
}

// ---------------------------------------------------------------------------------
// local cylindrical frame at the prediction and the measurement model
// ---------------------------------------------------------------------------------
struct Frame {
  float rho, rx, ry;  // radius about the layer axis and radial unit vector
  float cosa;         // cosine of the angle between the track and the surface normal:
                      // r_hat . t on a cylinder, cos(theta) on a disk
  float ica;          // 1 / cosa (cylinders)
  float icpsi;        // 1 / the same cosine for the 3-D direction (the material's path is
                      // xX0 * icpsi): 1 / (sin(theta) |cosa|) on a cylinder, 1 / |cos theta| on a disk
};

__device__ __forceinline__ Frame frame_at(const Trk& k, const LayerK& ly, bool disk = false) {
  Frame f;
  const float ex = rel_pos(k.x[0], k.xl[0], ly.cx), ey = rel_pos(k.x[1], k.xl[1], ly.cy);
  const float r2 = fmaf(ex, ex, ey * ey);
  const float ir = hrsqrt(r2);
  f.rho = r2 * ir;
  f.rx = ex * ir;
  f.ry = ey * ir;
  if (disk) {
    f.cosa = k.ct;
    f.ica = 1.f;
    f.icpsi = rcp(fabsf(k.ct));
  } else {
    f.cosa = fmaf(f.rx, k.cp, f.ry * k.sp);
    f.ica = rcp(f.cosa);
    f.icpsi = k.rst * fabsf(f.ica);
  }
  return f;
}

// Highland multiple scattering of a thin layer, added to (kappa, phi, theta):
// theta0^2 = (0.0136/(beta p))^2 x (1 + 0.038 ln x)^2, x = xX0 icpsi (a cylinder:
// 1 / (sin(theta) |cos alpha|); a disk: 1 / |cos theta|),
// 1/(beta p) = |kappa| sin(theta) sqrt(1 + m^2 kappa^2 sin^2(theta)).
__device__ __forceinline__ void add_scattering(Trk& k, const Frame& f, float xX0, float mass2) {
  const float kap = k.x[3];
  const float ks = kap * k.st;
  const float ks2 = ks * ks;
  const float xe = xX0 * f.icpsi;
  // 0.038 ln x as 0.038 ln(2) log2(x): the hardware base-2 logarithm (v_log_f32, ~1 ulp)
  const float lg = fmaf(0.038f * 0.69314718f, __builtin_amdgcn_logf(xe), 1.f);
  const float th2 = 0.0136f * 0.0136f * ks2 * fmaf(mass2, ks2, 1.f) * xe * lg * lg;
  const float rst = k.rst;
  const float cot = k.ct * rst;
  const float kc = kap * cot;
  k.C[tri(4, 4)] = fmaf(th2 * rst, rst, k.C[tri(4, 4)]);
  k.C[tri(5, 5)] += th2;
  k.C[tri(3, 3)] = fmaf(kc * kc, th2, k.C[tri(3, 3)]);
  k.C[tri(5, 3)] = fmaf(-kc, th2, k.C[tri(5, 3)]);
}

// x/X0 of a layer at z (its own frame) from its row of the material map: nz values at
// the centres of nz equal bins over [-Z, Z], interpolated linearly, constant beyond
// the outer centres (u = (z + Z) nz / 2Z - 1/2 is the position in units of bins).
__device__ __forceinline__ float map_xX0(const float* __restrict__ row, int nz, const LayerK& ly, float z) {
  if (nz == 1) return row[0];
  const float u = fminf(fmaxf(fmaf(z - ly.dz, ly.zs, ly.zo), 0.f), (float)(nz - 1));
  const int b = min((int)u, nz - 2);
  const float t = u - (float)b;
  const float v0 = row[b];
  return fmaf(t, row[b + 1] - v0, v0);
}

// Mean ionisation loss of a thin layer after its scattering (Sec. 3: energy loss from
// the material description): dE = eloss * x_eff / beta^2 with the scattering term's path
// length x_eff and beta at the incoming momentum p = 1 / (|kappa| sin theta); the
// energy drops to E' = E - dE at fixed direction, so kappa' = kappa p / p'.  The
// covariance follows kappa'(kappa, theta): C <- A C A^T with A = I but for the kappa
// row (D at kappa, T at theta), where, with W = p X / p'^3 and
// X = dE (m^2/E + E') + 2 eloss x_eff m^2 E' / p^2 (a sum of positive terms: the
// derivative written this way does not cancel),
//   D = dkappa'/dkappa = p/p' + W,   T = dkappa'/dtheta = kappa cot(theta) W.
// False if the particle is left without kinetic energy.
__device__ __forceinline__ bool energy_loss(Trk& k, const Frame& f, float xX0, float eloss, float mass2) {
  const float kap = k.x[3];
  const float ks = fabsf(kap) * k.st;          // 1 / p
  const float p = rcp(ks);
  const float c = eloss * xX0 * f.icpsi;
  const float ib2 = fmaf(mass2, ks * ks, 1.f); // 1 / beta^2
  const float E = p * hsqrt(ib2);
  const float dE = c * ib2;
  const float E1 = E - dE;
  const float q2 = fmaf(E1, E1, -mass2);       // p'^2
  if (!(E1 > 0.f) || !(q2 > 0.f)) return false;
  const float ip1 = hrsqrt(q2);                // 1 / p'
  const float X = fmaf(dE, fmaf(mass2, rcp(E), E1), 2.f * c * mass2 * E1 * ks * ks);
  const float W = p * X * (ip1 * ip1 * ip1);
  const float g = p * ip1;
  const float D = g + W;
  const float T = kap * (k.ct * k.rst) * W;
  float* C = k.C;
  const float c53 = C[tri(5, 3)], c55 = C[tri(5, 5)], c33 = C[tri(3, 3)];
  C[tri(3, 0)] = fmaf(D, C[tri(3, 0)], T * C[tri(5, 0)]);
  C[tri(3, 1)] = fmaf(D, C[tri(3, 1)], T * C[tri(5, 1)]);
  C[tri(3, 2)] = fmaf(D, C[tri(3, 2)], T * C[tri(5, 2)]);
  C[tri(4, 3)] = fmaf(D, C[tri(4, 3)], T * C[tri(5, 4)]);
  C[tri(5, 3)] = fmaf(D, c53, T * c55);
  C[tri(3, 3)] = fmaf(D * D, c33, T * fmaf(2.f * D, c53, T * c55));
  k.x[3] = kap * g;
  return true;
}

// k_B of the parameterised field B_z(r, z) = B (1 + fr r^2 + fz z^2) at (x, y, z), for a
// step that starts there; exactly kB when both coefficients are zero.
__device__ __forceinline__ float field_kB(float kB, float fr, float fz, float x, float y, float z) {
  return kB * fmaf(fz, z * z, fmaf(fr, fmaf(x, x, y * y), 1.f));
}

// The material of a layer crossed after the seed layer under the detector model: x/X0
// from the map row (null: the layer's constant), its scattering term, then the mean
// energy loss.  False if the particle stops in it (the state then holds the
// transported prediction with the scattering term added).
__device__ __forceinline__ bool apply_material(Trk& k, const Frame& f, const LayerK& ly, const float* row, int nz,
                                               float eloss, float mass2) {
  const float xx = row ? map_xX0(row, nz, ly, k.x[2]) : ly.xX0;
  bool ok = true;
  if (xx > 0.f) {
    add_scattering(k, f, xx, mass2);
    if (eloss > 0.f) ok = energy_loss(k, f, xx, eloss, mass2);
  }
  return ok;
}

// What a prediction needs for every hit of a layer: the projection rows
// h1 = phi_hat - tan(alpha) r_hat, h2 = (-cot(theta)/cos(alpha) r_hat, 1), the
// products HC (rows 1, 2 of H C) and S^-1 (S = H C H^T + V is block diagonal: its
// radial entry is the regulariser alone).  On a disk the rows project onto the plane
// along the tangent: h1 = (phi_hat, -(phi_hat . t) / cot(theta)), h2 = (r_hat,
// -(r_hat . t) / cot(theta)) for (rho * phi, rho), and the regulariser's row is z.
struct Pred {
  float h1x, h1y, h2x, h2y;
  float h1z, h2z;  // z components on a disk (a cylinder's are 0 and 1)
  float HC1[6], HC2[6];
  float S11, S12, S22;
  float Si00, Si11, Si12, Si22;
  bool fp64;
  double dSi11, dSi12, dSi22;
};

__device__ __forceinline__ void prepare(const Trk& k, const Frame& f, const Model& md, Pred& p, bool disk = false) {
  const float fx = -f.ry, fy = f.rx;
  const float* C = k.C;
  if (disk) {
    const float icot = k.st * rcp(k.ct);
    p.h1x = fx;
    p.h1y = fy;
    p.h1z = -fmaf(fx, k.cp, fy * k.sp) * icot;
    p.h2x = f.rx;
    p.h2y = f.ry;
    p.h2z = -fmaf(f.rx, k.cp, f.ry * k.sp) * icot;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      p.HC1[j] = fmaf(p.h1x, C[tri(0, j)], fmaf(p.h1y, C[tri(1, j)], p.h1z * C[tri(2, j)]));
      p.HC2[j] = fmaf(p.h2x, C[tri(0, j)], fmaf(p.h2y, C[tri(1, j)], p.h2z * C[tri(2, j)]));
    }
    p.S11 = fmaf(p.HC1[0], p.h1x, fmaf(p.HC1[1], p.h1y, fmaf(p.HC1[2], p.h1z, md.v_rphi)));
    p.S12 = fmaf(p.HC1[0], p.h2x, fmaf(p.HC1[1], p.h2y, p.HC1[2] * p.h2z));
    p.S22 = fmaf(p.HC2[0], p.h2x, fmaf(p.HC2[1], p.h2y, fmaf(p.HC2[2], p.h2z, md.v_z)));
  } else {
    const float ica = f.ica;
    const float tana = fmaf(fx, k.cp, fy * k.sp) * ica;
    const float cot = k.ct * k.rst;
    p.h1x = fmaf(-tana, f.rx, fx);
    p.h1y = fmaf(-tana, f.ry, fy);
    const float g = -cot * ica;
    p.h2x = g * f.rx;
    p.h2y = g * f.ry;
    p.h1z = 0.f;
    p.h2z = 1.f;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      p.HC1[j] = fmaf(p.h1x, C[tri(0, j)], p.h1y * C[tri(1, j)]);
      p.HC2[j] = fmaf(p.h2x, C[tri(0, j)], fmaf(p.h2y, C[tri(1, j)], C[tri(2, j)]));
    }
    p.S11 = fmaf(p.HC1[0], p.h1x, fmaf(p.HC1[1], p.h1y, md.v_rphi));
    p.S12 = fmaf(p.HC1[0], p.h2x, fmaf(p.HC1[1], p.h2y, p.HC1[2]));
    p.S22 = fmaf(p.HC2[0], p.h2x, fmaf(p.HC2[1], p.h2y, p.HC2[2] + md.v_z));
  }
  // equilibrated inverse: S~ = D^-1/2 S D^-1/2 has unit diagonal; its radial row is
  // (1, 0, 0), so det S~ = 1 - rho12^2.
  p.Si00 = 1.f / md.v_r;
  const float d1 = hrsqrt(p.S11), d2 = hrsqrt(p.S22);
  const float r12 = p.S12 * d1 * d2;
  const float det = fmaf(-r12, r12, 1.f);
  // det <= 1 always, so a threshold above 1 fails every check; a non-positive or
  // non-finite S11, S22 or S12 makes det NaN or -inf, which fails it too
  const bool good = det >= md.det_thr;
  p.fp64 = !good;
  if (good) {
    const float idet = rcp(det);
    p.Si11 = d1 * d1 * idet;
    p.Si22 = d2 * d2 * idet;
    p.Si12 = -r12 * d1 * d2 * idet;
  } else {
    const double s11 = p.S11, s12 = p.S12, s22 = p.S22;
    const double dd = s11 * s22 - s12 * s12;
    p.dSi11 = s22 / dd;
    p.dSi22 = s11 / dd;
    p.dSi12 = -s12 / dd;
    p.Si11 = (float)p.dSi11;
    p.Si22 = (float)p.dSi22;
    p.Si12 = (float)p.dSi12;
  }
}

// Residual of a placed hit m in the prediction's frame: (rho_m - rho_p,
// rho_p * angle(r_hat, m - c), z_m - z_p) on a cylinder, (z_m - z_p, rho_p * angle,
// rho_m - rho_p) on a disk, and its chi2.  Everything is formed from
// the small offset d = m - p (p: the predicted point, hi + lo parts): since r_hat is
// parallel to p - c, r_hat x (m - c) = r_hat x d, and
// rho_m - rho_p = (2 rho_p r_hat.d + |d|^2) / (rho_m + rho_p).  Products of the
// ~100 cm coordinates would cancel to the ~0.01 cm residual.
struct Resid {
  float r0, r1, r2, chi2;
};

__device__ __forceinline__ Resid residual(const Trk& k, const Frame& f, const LayerK& ly, const Pred& p, float mx,
                                          float my, float mz, bool disk = false) {
  (void)ly;
  Resid r;
  const float dx = (mx - k.x[0]) - k.xl[0], dy = (my - k.x[1]) - k.xl[1];
  const float rd = fmaf(f.rx, dx, f.ry * dy);
  const float cr = fmaf(f.rx, dy, -f.ry * dx);
  const float d2 = fmaf(dx, dx, dy * dy);
  const float num = fmaf(2.f * f.rho, rd, d2);
  const float rm = hsqrt(fmaf(f.rho, f.rho, num));
  r.r0 = num * rcp(rm + f.rho);
  // angle of d about the axis seen from the prediction: atan(x), x = cr / (rho + rd),
  // by its series to x^9 for |x| < 0.1 (truncation < x^11/11 = 1e-12), atan2f otherwise
  const float den = f.rho + rd;
  if (den > 0.f && fabsf(cr) < 0.1f * den) {
    const float x = cr * rcp(den), x2 = x * x;
    r.r1 = f.rho * (x * fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.f / 9.f, -1.f / 7.f), 0.2f), -1.f / 3.f), 1.f));
  } else {
    r.r1 = f.rho * atan2f(cr, den);
  }
  r.r2 = (mz - k.x[2]) - k.xl[2];
  if (disk) {  // the radial difference measures rho, the z difference is the regulariser's
    const float t = r.r0;
    r.r0 = r.r2;
    r.r2 = t;
  }
  if (!p.fp64) {
    const float q = fmaf(r.r1 * r.r1, p.Si11, fmaf(2.f * r.r1 * r.r2, p.Si12, r.r2 * r.r2 * p.Si22));
    r.chi2 = fmaf(r.r0 * r.r0, p.Si00, q);
  } else {
    const double a = r.r1, b = r.r2;
    const double q = a * a * p.dSi11 + 2.0 * a * b * p.dSi12 + b * b * p.dSi22;
    r.chi2 = (float)(q + (double)r.r0 * r.r0 * (double)p.Si00);
  }
  r.chi2 = fmaxf(r.chi2, 0.f);
  return r;
}

// Gain and Joseph-form update: K = C H^T S^-1 (its radial column is zero),
// x += K r, C <- (I - K H) C (I - K H)^T + K V K^T.  With M = (I - K H) C =
// C - K (H C) and v_a = M h_a^T, C' = M - (v_1 k_1^T + v_2 k_2^T) + K V K^T, lower
// triangle only.
__device__ __forceinline__ void apply_update(Trk& k, const Pred& p, const Model& md, float r1, float r2,
                                             bool disk = false) {
  float K1[6], K2[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    K1[i] = fmaf(p.HC1[i], p.Si11, p.HC2[i] * p.Si12);
    K2[i] = fmaf(p.HC1[i], p.Si12, p.HC2[i] * p.Si22);
  }
  const float dphi = fmaf(K1[4], r1, K2[4] * r2);
  const float dth = fmaf(K1[5], r1, K2[5] * r2);
#pragma unroll
  for (int i = 0; i < 2; ++i) add_pos(k.x[i], k.xl[i], fmaf(K1[i], r1, K2[i] * r2));
  k.x[2] = fmaf(K1[2], r1, fmaf(K2[2], r2, k.x[2]));
#pragma unroll
  for (int i = 3; i < 6; ++i) k.x[i] = fmaf(K1[i], r1, fmaf(K2[i], r2, k.x[i]));
  rotate_small(k.cp, k.sp, dphi, k.x[4]);
  rotate_small(k.ct, k.st, dth, k.x[5]);
  k.rst = rcp(k.st);
  float* C = k.C;
  // M[i][j] for the lower triangle and for columns 0..2 of every row
  float M[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j <= i || j < 3) M[i][j] = fmaf(-K1[i], p.HC1[j], fmaf(-K2[i], p.HC2[j], C[tri(i, j)]));
  // w_a = V_a K_a - M h_a^T; evaluating M h_a^T from the rounded M (rather than by its
  // closed form) keeps the covariance error at the few-ulp level
  float w1[6], w2[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float v1 = disk ? fmaf(M[i][0], p.h1x, fmaf(M[i][1], p.h1y, M[i][2] * p.h1z))
                          : fmaf(M[i][0], p.h1x, M[i][1] * p.h1y);
    const float v2 = disk ? fmaf(M[i][0], p.h2x, fmaf(M[i][1], p.h2y, M[i][2] * p.h2z))
                          : fmaf(M[i][0], p.h2x, fmaf(M[i][1], p.h2y, M[i][2]));
    w1[i] = fmaf(md.v_rphi, K1[i], -v1);
    w2[i] = fmaf(md.v_z, K2[i], -v2);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) C[tri(i, j)] = fmaf(K1[j], w1[i], fmaf(K2[j], w2[i], M[i][j]));
}

// Place a nominal-frame hit on its (aligned) layer.
__device__ __forceinline__ void place(const LayerK& ly, float hx, float hy, float hz, float& mx, float& my,
                                      float& mz) {
  if (ly.moved != 0.f) {  // (the identity transform gives the same bits)
    mx = ly.cx + fmaf(ly.cphi, hx, -ly.sphi * hy);
    my = ly.cy + fmaf(ly.sphi, hx, ly.cphi * hy);
    mz = hz + ly.dz;
  } else {
    mx = hx;
    my = hy;
    mz = hz;
  }
}

// Seed: the helix through three placed hits (signed Menger curvature, chord angles),
// at the first hit, with the diagonal prior inflated ten times in variance.
__device__ __forceinline__ void seed_from_three(Trk& k, const Model& md, float x0, float y0, float z0, float x1,
                                                float y1, float x2, float y2, float z2, float srphi, float sz) {
  const float ax = x1 - x0, ay = y1 - y0;
  const float bx = x2 - x1, by = y2 - y1;
  const float cx = x2 - x0, cy = y2 - y0;
  const float la = sqrtf(fmaf(ax, ax, ay * ay));
  const float lb = sqrtf(fmaf(bx, bx, by * by));
  const float lc = sqrtf(fmaf(cx, cx, cy * cy));
  const float w = 2.f * fmaf(ax, by, -ay * bx) / (la * lb * lc);
  const float qa = fminf(fmaxf(0.5f * w * la, -1.f), 1.f);
  const float qc = fminf(fmaxf(0.5f * w * lc, -1.f), 1.f);
  const float phi0 = atan2f(ay, ax) - asinf(qa);
  const float qc2 = qc * qc;
  const float arc = fabsf(qc) < 1e-2f ? lc * fmaf(qc2, fmaf(qc2, 0.075f, 1.f / 6.f), 1.f) : lc * asinf(qc) / qc;
  k.x[0] = x0;
  k.x[1] = y0;
  k.x[2] = z0;
  k.xl[0] = k.xl[1] = k.xl[2] = 0.f;
  k.x[3] = -w / md.kB;
  k.x[4] = wrap_pi(phi0);
  k.x[5] = atan2f(arc, z2 - z0);
  const float dr = md.dr02;
  const float sphi = 1.41421356237f * srphi / dr, sth = 1.41421356237f * sz / dr;
  const float skap = 8.f * 1.22474487139f * srphi / (dr * dr * md.kB);
#pragma unroll
  for (int q = 0; q < 21; ++q) k.C[q] = 0.f;
  k.C[tri(0, 0)] = 10.f * srphi * srphi;
  k.C[tri(1, 1)] = 10.f * srphi * srphi;
  k.C[tri(2, 2)] = 10.f * sz * sz;
  k.C[tri(3, 3)] = 10.f * skap * skap;
  k.C[tri(4, 4)] = 10.f * sphi * sphi;
  k.C[tri(5, 5)] = 10.f * sth * sth;
}

}  // namespace kfd
