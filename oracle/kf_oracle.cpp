// FP64 oracle of the batched Kalman fit, the combinatorial track finder, the
// gradient of the fit's total chi2 with respect to per-layer alignment and material,
// and the fixed-interval (Rauch-Tung-Striebel) smoother over the fit.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
// this file: it exists so that tests, the smoke check and the CPU baseline of the
// benchmark can compare the GPU library against a plain, slow, independently
// written implementation.  It shares no code, header or constant table with the
// GPU library.
//
// What it follows.  The paper (Sec. 2) states that track building and fitting are
// the Kalman filter method applied layer by layer to symmetric 6x6 covariances,
// that the geometry supplies layer positions, search windows and radiation
// lengths for multiple scattering (Sec. 3), that the field is a constant 3.8 T
// (Sec. 4), and that candidates are ranked by scores inside search windows
// (Sec. 4.3).  It prints no formula; every formula below is the textbook reading
// of those statements (extended Kalman filter, helix in a uniform solenoidal
// field, Highland multiple scattering), as listed in the design notes.
//
// Deliberately different numerical routes from the GPU library:
//   * the crossing of the helix with a layer is bracketed by marching along the helix,
//     bisected, then polished by Newton steps on the transverse arc length;
//   * the residual's azimuth difference is a difference of two atan2 values;
//   * S is inverted by Gauss-Jordan elimination with partial pivoting on the full
//     3x3 matrix; every matrix product is a dense loop over all indices.
//
// Everything is templated on the scalar type so that forward-mode dual numbers
// give the FP64 reference gradient (Dual<N> below).
//
// Parity pins (tests/test_oracle_*.py): linear-Gaussian filter = batch weighted
// least squares; straight-line limit of the crossing; noiseless hits return the
// generating helix; covariances stay symmetric positive definite; pulls and
// chi2/ndf of simulated tracks have unit scale; Jacobians agree with central
// differences of the oracle's own maps; binned search = brute-force search;
// dual-number gradient = central finite differences; global translation and
// rotation leave the total chi2 unchanged; RTS on a linear-Gaussian chain = the joint
// posterior of all states, noiseless smoothed states = the helix at every layer to
// second order, smoothed pulls have unit scale and C_s <= C_f; a material map of
// constant rows without energy loss is the per-layer model bit for bit, one material
// step matches its definition (covariance row by central differences), and tracks
// simulated through the map with energy loss give unit pulls; a field with zero
// coefficients is the uniform one bit for bit, noiseless tracks in a non-uniform field
// return the generating state, and its pulls have unit scale.  Parity unpinned: the candidate score
// and its tie rule, and the Highland variant, which are conventions.

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <type_traits>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846;

// ------------------------------------------------------------------------------
// forward-mode dual numbers
// ------------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0) { for (int i = 0; i < N; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0; }  // NOLINT
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) { Dual<N> r; r.v = a.v / b.v; for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) { Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a * (1.0 / b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) { a = a * b; return a; }
template <int N> Dual<N> chain(const Dual<N>& a, double f, double df) { Dual<N> r; r.v = f; for (int i = 0; i < N; ++i) r.d[i] = df * a.d[i]; return r; }
template <int N> Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> Dual<N> atan(const Dual<N>& a) { return chain(a, std::atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
template <int N> Dual<N> asin(const Dual<N>& a) { return chain(a, std::asin(a.v), 1.0 / std::sqrt(1.0 - a.v * a.v)); }
template <int N> Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> Dual<N> fabs(const Dual<N>& a) { return a.v < 0 ? -a : a; }
template <int N> Dual<N> atan2(const Dual<N>& y, const Dual<N>& x) {
  Dual<N> r; r.v = std::atan2(y.v, x.v);
  double q = x.v * x.v + y.v * y.v;
  for (int i = 0; i < N; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / q;
  return r;
}

inline double val(double x) { return x; }
template <int N> double val(const Dual<N>& x) { return x.v; }

template <class T> T wrap_pi(const T& a) {  // to (-pi, pi]
  double k = std::floor((val(a) + kPi) / (2 * kPi));
  T r = a - 2 * kPi * k;
  if (val(r) <= -kPi) r = r + 2 * kPi;
  if (val(r) > kPi) r = r - 2 * kPi;
  return r;
}

// ------------------------------------------------------------------------------
// geometry, options, status
// ------------------------------------------------------------------------------
}  // namespace

extern "C" {
// Mirrors the Python-side ctypes structure in oracle/__init__.py.
struct OGeom {
  int32_t n_layers, n_phi_bins, n_z_bins, pad;
  double B, sigma_rphi, sigma_z, sigma_r, mass;
  double radius[32];
  double zhalf[32];
  // endcap disks: layer l is the plane z = disk_z[l] (!= 0) active for radii
  // disk_rmin[l] .. disk_rmax[l]; other layers are cylinders active for |z| <= cyl_zmax[l]
  // (0: unbounded)
  double disk_z[32], disk_rmin[32], disk_rmax[32], cyl_zmax[32];
};
}

namespace {

enum : uint32_t {
  ST_PROP_FAIL = 1u,      // the helix does not reach a layer it has to cross
  ST_NEAR_TANGENT = 2u,   // some crossing has |cos alpha| < 0.3
  ST_ILLCOND = 4u,        // equilibrated det(S) below the FP32 trust threshold
  ST_NONFINITE = 8u,
  ST_BAD_INPUT = 16u,     // hit mask lacks the seed layers
  ST_TERM_MISSES = 32u,   // finder: candidate stopped after max_miss missing layers
};

constexpr double kHighlandA = 0.0136, kHighlandB = 0.038;
constexpr double kIllCond = 1e-2;

template <class T>
struct Layer {
  T cx, cy, dz, cphi, sphi, xX0;  // alignment (centre, z shift, rotation) and x/X0
  T moff = T(0.0);  // additive offset of the layer's material-map row (0; a gradient seed)
  double r;
  int idx = 0;  // layer index (row of a material map)
  // a disk: the plane z = zd + dz, active for rmin <= rho <= rmax (rho about its axis);
  // a cylinder: active for |z - dz| <= zmax (0: unbounded)
  bool disk = false;
  double zd = 0, rmin = 0, rmax = 0, zmax = 0;
  bool bounded() const { return disk || zmax > 0; }
};

struct Geo {
  int nl;
  double kB, srphi, sz, sr, mass;
  double radius[32], zhalf[32];
  double disk_z[32], disk_rmin[32], disk_rmax[32], cyl_zmax[32];
  int nphi, nz;
  // Material beyond one x/X0 per layer (Sec. 3: a per-layer table of x/X0 over z,
  // multiple scattering and energy loss): map [nl][map_nz] of x/X0 at the centres of
  // map_nz equal z bins over each layer's [-zhalf, zhalf] (null: the layer's xX0), and
  // the mean ionisation loss per radiation length at minimum ionisation (0: none).
  const double* map = nullptr;
  int map_nz = 0;
  double eloss = 0.0;
  // Parameterised field (Sec. 3): B_z(r, z) = B (1 + fr r^2 + fz z^2), cm, global frame;
  // each step is the helix of the field at its starting point.
  double fr = 0.0, fz = 0.0;
};

// k_B of the field at (x, y, z).  Templated on the scalar type: with dual numbers the
// field's dependence on the point (which moves with the alignment parameters) is part
// of the derivative, so the gradient below is that of the total chi2 as computed.
template <class T>
T kB_at(const Geo& g, const T& x, const T& y, const T& z) {
  if (g.fr == 0.0 && g.fz == 0.0) return T(g.kB);
  return g.kB * (1.0 + g.fr * (x * x + y * y) + g.fz * z * z);
}

Geo make_geo(const OGeom* g) {
  Geo o;
  o.nl = g->n_layers;
  o.kB = 0.299792458e-2 * g->B;
  o.srphi = g->sigma_rphi; o.sz = g->sigma_z; o.sr = g->sigma_r; o.mass = g->mass;
  for (int l = 0; l < 32; ++l) {
    o.radius[l] = g->radius[l];
    o.zhalf[l] = g->zhalf[l];
    o.disk_z[l] = g->disk_z[l];
    o.disk_rmin[l] = g->disk_rmin[l];
    o.disk_rmax[l] = g->disk_rmax[l];
    o.cyl_zmax[l] = g->cyl_zmax[l];
  }
  o.nphi = g->n_phi_bins; o.nz = g->n_z_bins;
  return o;
}

template <class T>
void make_layers(const Geo& g, const T* align /*[L][4]*/, const T* xX0, Layer<T>* lay) {
  using std::cos; using std::sin;
  for (int l = 0; l < g.nl; ++l) {
    lay[l].cx = align ? align[4 * l + 0] : T(0.0);
    lay[l].cy = align ? align[4 * l + 1] : T(0.0);
    lay[l].dz = align ? align[4 * l + 2] : T(0.0);
    T dphi = align ? align[4 * l + 3] : T(0.0);
    lay[l].cphi = cos(dphi);
    lay[l].sphi = sin(dphi);
    lay[l].xX0 = xX0 ? xX0[l] : T(0.0);
    lay[l].r = g.radius[l];
    lay[l].idx = l;
    lay[l].disk = g.disk_z[l] != 0.0;
    lay[l].zd = g.disk_z[l];
    lay[l].rmin = g.disk_rmin[l];
    lay[l].rmax = g.disk_rmax[l];
    lay[l].zmax = lay[l].disk ? 0.0 : g.cyl_zmax[l];
  }
}

// Nominal-frame hit -> the layer's actual position (rigid transform about its axis).
template <class T>
void place_hit(const Layer<T>& ly, double hx, double hy, double hz, T m[3]) {
  m[0] = ly.cx + ly.cphi * hx - ly.sphi * hy;
  m[1] = ly.cy + ly.sphi * hx + ly.cphi * hy;
  m[2] = ly.dz + hz;
}

// ------------------------------------------------------------------------------
// track model: helix in a uniform field along +z
// state (x, y, z, kappa = q/pT, phi, theta); omega = -k_B kappa is the turning rate
// per unit transverse arc length.
// ------------------------------------------------------------------------------

// Position and direction after a transverse arc s.
template <class T>
void helix_at(const T x[6], const T& s, const T& kB, T out[6]) {
  using std::cos; using std::sin;
  T w = -kB * x[3];
  T u = w * s;
  T A, Bn;  // displacement = s (A t + Bn n)
  if (std::fabs(val(u)) < 1e-4) {
    T u2 = u * u;
    A = 1.0 - u2 / 6.0 + u2 * u2 / 120.0;
    Bn = u * (0.5 - u2 / 24.0 + u2 * u2 / 720.0);
  } else {
    T sh = sin(0.5 * u);
    A = sin(u) / u;
    Bn = 2.0 * sh * sh / u;
  }
  T tx = cos(x[4]), ty = sin(x[4]);
  out[0] = x[0] + s * (A * tx - Bn * ty);
  out[1] = x[1] + s * (A * ty + Bn * tx);
  out[2] = x[2] + s * cos(x[5]) / sin(x[5]);
  out[3] = x[3];
  out[4] = wrap_pi(x[4] + u);
  out[5] = x[5];
}

// Transverse arc length to the first forward crossing with |p - c| = r, within the
// first half turn.  f(s) = |p(s) - c|^2 - r^2 is negative at s = 0 inside the cylinder
// (the crossing is the exit) and positive outside it (the entry, for a particle run
// inwards); march along the helix until it changes sign, bisect the bracket, then
// polish with Newton steps (which also settle the derivative parts of dual numbers).
template <class T>
T crossing_residual(const T x[6], const T& s, const T& cx, const T& cy, double r, const T& kB, T* fp) {
  using std::cos; using std::sin;
  T p[6];
  helix_at(x, s, kB, p);
  T dx = p[0] - cx, dy = p[1] - cy;
  if (fp) *fp = 2.0 * (dx * cos(p[4]) + dy * sin(p[4]));
  return dx * dx + dy * dy - r * r;
}

template <class T>
bool crossing_arc(const T x[6], const T& cx, const T& cy, double r, const T& kB, T& s) {
  T ex = x[0] - cx, ey = x[1] - cy;
  double c0 = val(ex * ex + ey * ey) - r * r;
  if (!(c0 != 0)) return false;
  const double sg = c0 < 0 ? 1.0 : -1.0;  // f * sg turns non-negative at the crossing
  double w = -val(kB) * val(x[3]);
  double smax = w != 0 ? kPi / std::fabs(w) : 4.0 * r;
  double h = 0.125 * r;
  if (w != 0) h = std::min(h, 0.125 / std::fabs(w));
  // Along the helix circle the squared distance to the layer axis is a sinusoid of
  // the turning angle, largest where the circle is farthest from the axis and smallest
  // opposite.  That point (the farthest for an exit, the nearest for an entry) is
  // always sampled, so a helix that only grazes the layer is bracketed too.
  double speak = -1.0;
  if (w != 0) {
    double tx = std::cos(val(x[4])), ty = std::sin(val(x[4]));
    double ccx = val(ex) - ty / w, ccy = val(ey) + tx / w;     // circle centre relative to the axis
    if (ccx * ccx + ccy * ccy > 0) {
      double psi_p = std::atan2(val(ey) - ccy, val(ex) - ccx);  // start, seen from the centre
      double psi_f = std::atan2(ccy, ccx);                      // farthest point, seen from the centre
      if (sg < 0) psi_f += kPi;                                 // nearest point
      double du = std::fmod((psi_f - psi_p) * (w > 0 ? 1.0 : -1.0), 2 * kPi);
      if (du < 0) du += 2 * kPi;
      speak = du / std::fabs(w);
    }
  }
  double lo = 0.0, hi = -1.0;
  bool peak_done = !(speak > 0 && speak < smax);
  for (double t = h; t < smax + h; t += h) {
    double tt = std::min(t, smax);
    if (!peak_done && speak <= tt) {
      peak_done = true;
      if (sg * val(crossing_residual<T>(x, T(speak), cx, cy, r, kB, nullptr)) >= 0) { hi = speak; break; }
      lo = speak;
    }
    double f = sg * val(crossing_residual<T>(x, T(tt), cx, cy, r, kB, nullptr));
    if (f >= 0) { hi = tt; break; }
    lo = tt;
    if (tt >= smax) break;
  }
  if (hi < 0) return false;
  for (int it = 0; it < 200 && hi - lo > 1e-14 * hi; ++it) {
    double mid = 0.5 * (lo + hi);
    if (sg * val(crossing_residual<T>(x, T(mid), cx, cy, r, kB, nullptr)) >= 0) hi = mid; else lo = mid;
  }
  s = T(0.5 * (lo + hi));
  for (int it = 0; it < 3; ++it) {
    T fp;
    T f = crossing_residual<T>(x, s, cx, cy, r, kB, &fp);
    if (val(fp) == 0) return false;
    s = s - f / fp;
  }
  if (!(val(s) > 0)) return false;
  if (w != 0 && std::fabs(w * val(s)) >= kPi) return false;
  return true;
}

// Transverse arc to the plane of a disk: z(s) = z + s cot(theta) = zp gives s = (zp - z)
// tan(theta).  The plane must lie ahead (s > 0) and be reached within half a turn.
template <class T>
bool plane_arc(const T x[6], const Layer<T>& ly, const T& kB, T& s) {
  using std::cos; using std::sin;
  const T ct = cos(x[5]);
  if (val(ct) == 0) return false;
  s = (ly.zd + ly.dz - x[2]) * sin(x[5]) / ct;
  if (!(val(s) > 0)) return false;
  const double w = -val(kB) * val(x[3]);
  return std::fabs(w * val(s)) < kPi;
}

// Transport Jacobian of the helix map at fixed transverse arc s (start state x,
// end state xe).  J = I plus six terms: d(x,y)/dphi, d(x,y)/dkappa, dz/dtheta,
// dphi/dkappa.
template <class T>
void transport_jacobian(const T x[6], const T xe[6], const T& s, const T& kB, T J[6][6]) {
  using std::cos; using std::sin;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) J[i][j] = T(i == j ? 1.0 : 0.0);
  T w = -kB * x[3];
  T u = w * s;
  T F1, F2;  // d(displacement)/d(omega) = s^2 (F1 t + F2 n)
  if (std::fabs(val(u)) < 1e-2) {
    T u2 = u * u;
    F1 = u * (-1.0 / 3.0 + u2 / 30.0 - u2 * u2 / 840.0);
    F2 = 0.5 - u2 / 8.0 + u2 * u2 / 144.0 - u2 * u2 * u2 / 5760.0;
  } else {
    F1 = (u * cos(u) - sin(u)) / (u * u);
    F2 = (u * sin(u) - 1.0 + cos(u)) / (u * u);
  }
  T tx = cos(x[4]), ty = sin(x[4]);
  T s2 = s * s;
  J[0][4] = -(xe[1] - x[1]);
  J[1][4] = xe[0] - x[0];
  J[0][3] = -kB * s2 * (F1 * tx - F2 * ty);
  J[1][3] = -kB * s2 * (F1 * ty + F2 * tx);
  T st = sin(x[5]);
  J[2][5] = -s / (st * st);
  J[4][3] = -kB * s;
}

template <class T>
void sandwich(const T J[6][6], T C[6][6]) {  // C <- J C J^T
  T JC[6][6], R[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T acc = 0.0;
      for (int k = 0; k < 6; ++k) acc += J[i][k] * C[k][j];
      JC[i][j] = acc;
    }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T acc = 0.0;
      for (int k = 0; k < 6; ++k) acc += JC[i][k] * J[j][k];
      R[i][j] = acc;
    }
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i][j] = 0.5 * (R[i][j] + R[j][i]);
}

// Multiple scattering of a thin layer at the predicted state: Highland's width with
// the 1/cos(psi) path-length factor, mapped to (kappa, phi, theta).
template <class T>
void add_scattering(const Geo& g, const Layer<T>& ly, const T x[6], T C[6][6]) {
  using std::cos; using std::sin; using std::sqrt; using std::log; using std::fabs;
  if (!(val(ly.xX0) > 0)) return;
  T ex = x[0] - ly.cx, ey = x[1] - ly.cy;
  T rho = sqrt(ex * ex + ey * ey);
  T st = sin(x[5]), ct = cos(x[5]);
  // cosine of the angle between the track and the surface normal: r_hat on a cylinder,
  // z on a disk
  T cpsi = ly.disk ? fabs(ct) : st * fabs((ex * cos(x[4]) + ey * sin(x[4])) / rho);
  T p = 1.0 / (fabs(x[3]) * st);
  T beta = p / sqrt(p * p + g.mass * g.mass);
  T xe = ly.xX0 / cpsi;
  T th0 = kHighlandA / (beta * p) * sqrt(xe) * (1.0 + kHighlandB * log(xe));
  T th2 = th0 * th0;
  T cot = ct / st;
  C[4][4] += th2 / (st * st);
  C[5][5] += th2;
  C[3][3] += x[3] * x[3] * cot * cot * th2;
  C[3][5] -= x[3] * cot * th2;
  C[5][3] -= x[3] * cot * th2;
}

// x/X0 of layer l at z (the layer's own frame) from the material map: linear
// interpolation between the centres of the map's equal z bins over [-Z_L, Z_L],
// constant beyond the outer centres.  (T: z may carry derivatives, which the
// interpolation's slope passes on.)
template <class T>
T map_xX0(const Geo& g, int l, const T& z) {
  const double* m = g.map + (int64_t)l * g.map_nz;
  const int nz = g.map_nz;
  if (nz == 1) return T(m[0]);
  const double Z = g.zhalf[l];
  const T u = (z + Z) / (2.0 * Z) * (double)nz - 0.5;
  if (val(u) <= 0.0) return T(m[0]);
  if (val(u) >= nz - 1) return T(m[nz - 1]);
  int k = (int)std::floor(val(u));
  if (k > nz - 2) k = nz - 2;
  const T t = u - (double)k;
  return m[k] + t * (m[k + 1] - m[k]);
}

// The mean ionisation loss of a thin layer as a map of kappa (Sec. 3): with
// p = 1 / (|kappa| sin(theta)), E = sqrt(p^2 + m^2) and c = eloss * x_eff, the energy
// drops by dE = c E^2 / p^2 (= c / beta^2) to E1 and kappa becomes kappa p / p1 (p1 the
// new momentum).  Returns false if E1 <= m.  With it, the derivatives of kappa1 in
// kappa and theta at fixed x_eff (the covariance's linearisation A: D = dkappa1/dkappa,
// Tt = dkappa1/dtheta), written out from those definitions: for p,
//   dE1/dp = p / E + 2 c m^2 / p^3,   dp1/dp = (E1 / p1) dE1/dp,
//   dkappa1/dp = kappa (p1 - p dp1/dp) / p1^2,
// and dp/dkappa = -p / kappa, dp/dtheta = -p cot(theta).
template <class T>
bool loss_map(const Geo& g, const T& kap, const T& th, const T& xe, T& k1, T& D, T& Tt) {
  using std::sin; using std::cos; using std::sqrt; using std::fabs;
  const double m2 = g.mass * g.mass;
  const T s = sin(th), ct = cos(th);
  const T p = 1.0 / (fabs(kap) * s);
  const T E = sqrt(p * p + m2);
  const T c = g.eloss * xe;
  const T E1 = E - c * (p * p + m2) / (p * p);
  if (!(val(E1) > g.mass)) return false;
  const T p1 = sqrt(E1 * E1 - m2);
  k1 = kap * p / p1;
  const T dE1 = p / E + 2.0 * c * m2 / (p * p * p);
  const T dp1 = E1 / p1 * dE1;
  const T dk1 = kap * (p1 - p * dp1) / (p1 * p1);
  D = p / p1 - dk1 * p / kap;
  Tt = -dk1 * p * ct / s;
  return true;
}

// The material of a thin layer at the predicted state (Sec. 3): multiple scattering
// with the layer's x/X0 there (the map plus its row's offset, else the layer's
// constant), then the mean ionisation loss dE = eloss * x_eff / beta^2 (x_eff the path
// length of the scattering term, beta at the incoming momentum): the energy drops to
// E - dE at fixed direction, so kappa becomes kappa * p / p' (loss_map).  The covariance
// follows kappa' as a function of (kappa, theta); the path-length factor enters the
// mean only.  False if the particle is left without kinetic energy.
template <class T>
bool material_step(const Geo& g, const Layer<T>& ly, T x[6], T C[6][6], double (*A_out)[6] = nullptr) {
  using std::cos; using std::sin; using std::sqrt; using std::fabs;
  if (A_out)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) A_out[i][j] = i == j ? 1.0 : 0.0;
  Layer<T> lm = ly;
  if (g.map && !ly.disk) lm.xX0 = map_xX0<T>(g, ly.idx, x[2] - ly.dz) + ly.moff;
  add_scattering(g, lm, x, C);
  if (!(g.eloss > 0.0) || !(val(lm.xX0) > 0.0)) return true;
  const T ex = x[0] - ly.cx, ey = x[1] - ly.cy;
  const T cpsi = ly.disk ? fabs(cos(x[5])) : sin(x[5]) * fabs((ex * cos(x[4]) + ey * sin(x[4])) / sqrt(ex * ex + ey * ey));
  const T xe = lm.xX0 / cpsi;
  T k1, D, Tt;
  if (!loss_map<T>(g, x[3], x[5], xe, k1, D, Tt)) return false;
  T A[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) A[i][j] = T(i == j ? 1.0 : 0.0);
  A[3][3] = D;
  A[3][5] = Tt;
  sandwich(A, C);
  x[3] = k1;
  if (A_out) {
    A_out[3][3] = val(D);
    A_out[3][5] = val(Tt);
  }
  return true;
}

// Gauss-Jordan inverse with partial pivoting (n <= 4); returns false if singular.
template <class T>
bool invert(int n, const T* A, T* Ai) {
  T M[4][8];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) M[i][j] = j < n ? A[i * n + j] : T(j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(val(M[r][c])) > std::fabs(val(M[piv][c]))) piv = r;
    if (val(M[piv][c]) == 0) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[c][j], M[piv][j]);
    T inv = 1.0 / M[c][c];
    for (int j = 0; j < 2 * n; ++j) M[c][j] = M[c][j] * inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      T f = M[r][c];
      for (int j = 0; j < 2 * n; ++j) M[r][j] = M[r][j] - f * M[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ai[i * n + j] = M[i][n + j];
  return true;
}

// Generic Kalman update for an n-dim state and m-dim measurement:
//   S = H C H^T + V, chi2 = r^T S^-1 r, K = C H^T S^-1, x += K r,
//   C <- (I - K H) C (I - K H)^T + K V K^T  (Joseph form), symmetrised.
template <class T>
bool kalman_update(int n, int m, T* x, T* C, const T* H, const T* V, const T* r, T& chi2, T* Sout = nullptr) {
  T HC[4 * 8], S[16], Si[16], K[8 * 4];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) {
      T acc = 0.0;
      for (int k = 0; k < n; ++k) acc += H[i * n + k] * C[k * n + j];
      HC[i * n + j] = acc;
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      T acc = V[i * m + j];
      for (int k = 0; k < n; ++k) acc += HC[i * n + k] * H[j * n + k];
      S[i * m + j] = acc;
    }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < i; ++j) { T a = 0.5 * (S[i * m + j] + S[j * m + i]); S[i * m + j] = a; S[j * m + i] = a; }
  if (Sout) for (int i = 0; i < m * m; ++i) Sout[i] = S[i];
  if (!invert(m, S, Si)) return false;
  chi2 = 0.0;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) chi2 += r[i] * Si[i * m + j] * r[j];
  for (int i = 0; i < n; ++i)  // K = (H C)^T S^-1
    for (int j = 0; j < m; ++j) {
      T acc = 0.0;
      for (int k = 0; k < m; ++k) acc += HC[k * n + i] * Si[k * m + j];
      K[i * m + j] = acc;
    }
  for (int i = 0; i < n; ++i) {
    T acc = 0.0;
    for (int j = 0; j < m; ++j) acc += K[i * m + j] * r[j];
    x[i] += acc;
  }
  T A[64], AC[64], N[64];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T acc = T(i == j ? 1.0 : 0.0);
      for (int k = 0; k < m; ++k) acc -= K[i * m + k] * H[k * n + j];
      A[i * n + j] = acc;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T acc = 0.0;
      for (int k = 0; k < n; ++k) acc += A[i * n + k] * C[k * n + j];
      AC[i * n + j] = acc;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T acc = 0.0;
      for (int k = 0; k < n; ++k) acc += AC[i * n + k] * A[j * n + k];
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) acc += K[i * m + a] * V[a * m + b] * K[j * m + b];
      N[i * n + j] = acc;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) C[i * n + j] = 0.5 * (N[i * n + j] + N[j * n + i]);
  return true;
}

// Measurement model at a predicted state on a cylindrical layer.
// Local frame about the layer axis at the prediction: (rho, rho*phi, z).
// Residual is cylindrical: (rho_m - rho_p, rho_p * wrap(phi_m - phi_p), z_m - z_p).
// H projects the state's position along its 3-D tangent onto the cylinder:
//   row 0 = 0, row 1 = phi_hat - tan(alpha) r_hat, row 2 = (-cot(theta)/cos(alpha) r_hat, 1),
// with cos(alpha) = r_hat . t and tan(alpha) = (phi_hat . t) / cos(alpha).
template <class T>
struct Meas {
  T H[3 * 6];
  T r[3];
  T rho, phip, cosa;
};

// On a disk the frame is the same about the disk's axis, with the plane's normal z:
// residual (z_m - z_p, rho_p * wrap(phi_m - phi_p), rho_m - rho_p) and H the projection
// along the state's tangent onto the plane (a position offset d moves to
// d - t3 d_z / cot(theta)): row 0 = 0 (the normal), row 1 = (phi_hat, -(phi_hat . t) /
// cot theta), row 2 = (r_hat, -(r_hat . t) / cot theta); cos alpha = cos theta.
template <class T>
void measurement_disk(const Layer<T>& ly, const T x[6], const T m[3], Meas<T>& o) {
  using std::atan2; using std::cos; using std::sin; using std::sqrt;
  T ex = x[0] - ly.cx, ey = x[1] - ly.cy;
  T rho = sqrt(ex * ex + ey * ey);
  T rx = ex / rho, ry = ey / rho;
  T fx = -ry, fy = rx;
  T tx = cos(x[4]), ty = sin(x[4]);
  T cot = cos(x[5]) / sin(x[5]);
  for (int i = 0; i < 18; ++i) o.H[i] = 0.0;
  o.H[6 + 0] = fx;
  o.H[6 + 1] = fy;
  o.H[6 + 2] = -(fx * tx + fy * ty) / cot;
  o.H[12 + 0] = rx;
  o.H[12 + 1] = ry;
  o.H[12 + 2] = -(rx * tx + ry * ty) / cot;
  T mx = m[0] - ly.cx, my = m[1] - ly.cy;
  T rhom = sqrt(mx * mx + my * my);
  T phim = atan2(my, mx), phip = atan2(ey, ex);
  o.r[0] = m[2] - x[2];
  o.r[1] = rho * wrap_pi(phim - phip);
  o.r[2] = rhom - rho;
  o.rho = rho;
  o.phip = phip;
  o.cosa = cos(x[5]);
}

template <class T>
void measurement(const Layer<T>& ly, const T x[6], const T m[3], Meas<T>& o) {
  using std::atan2; using std::cos; using std::sin; using std::sqrt;
  if (ly.disk) { measurement_disk(ly, x, m, o); return; }
  T ex = x[0] - ly.cx, ey = x[1] - ly.cy;
  T rho = sqrt(ex * ex + ey * ey);
  T rx = ex / rho, ry = ey / rho;
  T fx = -ry, fy = rx;
  T tx = cos(x[4]), ty = sin(x[4]);
  T cosa = rx * tx + ry * ty;
  T tana = (fx * tx + fy * ty) / cosa;
  T cot = cos(x[5]) / sin(x[5]);
  for (int i = 0; i < 18; ++i) o.H[i] = 0.0;
  o.H[6 + 0] = fx - tana * rx;
  o.H[6 + 1] = fy - tana * ry;
  o.H[12 + 0] = -cot / cosa * rx;
  o.H[12 + 1] = -cot / cosa * ry;
  o.H[12 + 2] = 1.0;
  T mx = m[0] - ly.cx, my = m[1] - ly.cy;
  T rhom = sqrt(mx * mx + my * my);
  T phim = atan2(my, mx), phip = atan2(ey, ex);
  o.r[0] = rhom - rho;
  o.r[1] = rho * wrap_pi(phim - phip);
  o.r[2] = m[2] - x[2];
  o.rho = rho;
  o.phip = phip;
  o.cosa = cosa;
}

template <class T>
double equilibrated_det(const T S[9]) {
  double d0 = val(S[0]), d1 = val(S[4]), d2 = val(S[8]);
  if (!(d0 > 0 && d1 > 0 && d2 > 0)) return 0.0;
  double a = val(S[1]) / std::sqrt(d0 * d1), b = val(S[2]) / std::sqrt(d0 * d2), c = val(S[5]) / std::sqrt(d1 * d2);
  return 1.0 + 2 * a * b * c - a * a - b * b - c * c;
}

template <class T>
struct Track {
  T x[6];
  T C[6][6];
  T chi2;
  int n;
  uint32_t status;
};

template <class T>
bool update_with_hit(const Geo& g, const Layer<T>& ly, Track<T>& tk, const T m[3], T* chi2_out = nullptr) {
  Meas<T> me;
  measurement(ly, tk.x, m, me);
  if (std::fabs(val(me.cosa)) < 0.3) tk.status |= ST_NEAR_TANGENT;
  T V[9] = {g.sr * g.sr, 0.0, 0.0, 0.0, g.srphi * g.srphi, 0.0, 0.0, 0.0, g.sz * g.sz};
  T S[9] = {};
  T chi2;
  if (!kalman_update(6, 3, tk.x, &tk.C[0][0], me.H, V, me.r, chi2, S)) { tk.status |= ST_NONFINITE; return false; }
  if (equilibrated_det(S) < kIllCond) tk.status |= ST_ILLCOND;
  if (val(chi2) < 0) chi2 = 0.0;
  tk.x[4] = wrap_pi(tk.x[4]);
  tk.chi2 += chi2;
  tk.n += 1;
  if (chi2_out) *chi2_out = chi2;
  return true;
}

// Propagate to layer L: crossing, C <- J C J^T, then + Q of the layer's material.
template <class T>
bool predict(const Geo& g, const Layer<T>& ly, Track<T>& tk, T (*J_out)[6] = nullptr) {
  T s;
  const T kB = kB_at<T>(g, tk.x[0], tk.x[1], tk.x[2]);  // the field at the step's start
  const bool crossed = ly.disk ? plane_arc(tk.x, ly, kB, s) : crossing_arc(tk.x, ly.cx, ly.cy, ly.r, kB, s);
  if (!crossed) { tk.status |= ST_PROP_FAIL; return false; }
  T xe[6];
  helix_at(tk.x, s, kB, xe);
  T J[6][6];
  transport_jacobian(tk.x, xe, s, kB, J);
  if (J_out)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) J_out[i][j] = J[i][j];
  sandwich(J, tk.C);
  for (int i = 0; i < 6; ++i) tk.x[i] = xe[i];
  {  // crossing angle: |cos alpha| = |r_hat . t| (a disk: |cos theta|) below 0.3 marks a
     // near-tangent crossing
    double ex = val(tk.x[0]) - val(ly.cx), ey = val(tk.x[1]) - val(ly.cy);
    double ca = ly.disk ? std::cos(val(tk.x[5]))
                        : (ex * std::cos(val(tk.x[4])) + ey * std::sin(val(tk.x[4]))) / std::sqrt(ex * ex + ey * ey);
    if (std::fabs(ca) < 0.3) tk.status |= ST_NEAR_TANGENT;
  }
  if (g.map || g.eloss > 0.0) {
    double A[6][6];
    if (!material_step(g, ly, tk.x, tk.C, A)) { tk.status |= ST_PROP_FAIL; return false; }
    if (J_out) {  // the step's linearisation is A J: the loss maps kappa after the transport
      T row[6];
      for (int j = 0; j < 6; ++j) row[j] = A[3][3] * J_out[3][j] + A[3][5] * J_out[5][j];
      for (int j = 0; j < 6; ++j) J_out[3][j] = row[j];
    }
  } else {
    add_scattering(g, ly, tk.x, tk.C);
  }
  return true;
}

// Three-hit helix seed at hit 0 (signed Menger curvature, chord angles), with the
// diagonal prior covariance inflated ten times in variance.  Curvature is turned into
// kappa with the field at hit 0.
template <class T>
void seed_from_hits(const Geo& g, const T m0[3], const T m1[3], const T m2[3], Track<T>& tk) {
  using std::asin; using std::atan2; using std::sqrt;
  T ax = m1[0] - m0[0], ay = m1[1] - m0[1];
  T bx = m2[0] - m1[0], by = m2[1] - m1[1];
  T cx = m2[0] - m0[0], cy = m2[1] - m0[1];
  T la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by), lc = sqrt(cx * cx + cy * cy);
  T w = 2.0 * (ax * by - ay * bx) / (la * lb * lc);
  T qa = 0.5 * w * la, qc = 0.5 * w * lc;
  if (val(qa) > 1) qa = 1.0;
  if (val(qa) < -1) qa = -1.0;
  if (val(qc) > 1) qc = 1.0;
  if (val(qc) < -1) qc = -1.0;
  T phi0 = atan2(ay, ax) - asin(qa);
  T s02;
  if (std::fabs(val(qc)) < 1e-4) s02 = lc * (1.0 + qc * qc / 6.0 + 0.075 * qc * qc * qc * qc);
  else s02 = lc * asin(qc) / qc;
  T theta = atan2(s02, m2[2] - m0[2]);
  tk.x[0] = m0[0]; tk.x[1] = m0[1]; tk.x[2] = m0[2];
  const T kB0 = kB_at<T>(g, m0[0], m0[1], m0[2]);
  tk.x[3] = -w / kB0;
  tk.x[4] = wrap_pi(phi0);
  tk.x[5] = theta;
  double dr = g.radius[2] - g.radius[0];
  double sphi = std::sqrt(2.0) * g.srphi / dr, sth = std::sqrt(2.0) * g.sz / dr;
  const T skap = 8.0 * std::sqrt(1.5) * g.srphi / (dr * dr * kB0);
  const T d[6] = {T(g.srphi * g.srphi), T(g.srphi * g.srphi), T(g.sz * g.sz), skap * skap, T(sphi * sphi),
                  T(sth * sth)};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) tk.C[i][j] = i == j ? 10.0 * d[i] : T(0.0);
  tk.chi2 = 0.0;
  tk.n = 0;
  tk.status = 0;
}


inline int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// The fit of one track: seed at layer 0, update on hit 0, then for every later layer
// up to the last hit: predict (crossing, transport, scattering) and, where the layer
// has a hit, update.  m[l] are the placed hits, mask bit l marks a hit on layer l.
// rec (optional) receives the state and covariance after each processed layer, [L][27]
// (after the update, or the prediction where the layer has no hit).
template <class T>
Track<T> fit_core(const Geo& g, const Layer<T>* lay, const T (*m)[3], uint32_t mask, bool from_hits,
                  const double* seed_x, const double* seed_C, double* rec) {
  Track<T> tk;
  for (int i = 0; i < 6; ++i) { tk.x[i] = 0.0; for (int j = 0; j < 6; ++j) tk.C[i][j] = 0.0; }
  tk.chi2 = 0.0; tk.n = 0; tk.status = 0;
  uint32_t need = from_hits ? 7u : 1u;
  if ((mask & need) != need) { tk.status = ST_BAD_INPUT; return tk; }
  if (from_hits) {
    seed_from_hits(g, m[0], m[1], m[2], tk);
  } else {
    for (int i = 0; i < 6; ++i) tk.x[i] = seed_x[i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) tk.C[i][j] = seed_C[i * 6 + j];
  }
  auto record = [&](int l) {
    if (!rec) return;
    for (int i = 0; i < 6; ++i) rec[(int64_t)l * 27 + i] = val(tk.x[i]);
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j <= i; ++j) rec[(int64_t)l * 27 + 6 + tri(i, j)] = val(tk.C[i][j]);
  };
  if (!update_with_hit(g, lay[0], tk, m[0])) return tk;
  record(0);
  int last = 31 - __builtin_clz(mask);
  if (last >= g.nl) last = g.nl - 1;
  for (int l = 1; l <= last; ++l) {
    // a bounded surface (a disk, or a cylinder of finite length) without a hit is one
    // the track did not cross: it is passed over (no material); one with a hit was
    // crossed.  Unbounded cylinders are crossed in turn, with or without a hit.
    if (lay[l].bounded() && !(mask >> l & 1u)) { record(l); continue; }
    if (!predict(g, lay[l], tk)) break;
    if (mask >> l & 1u)
      if (!update_with_hit(g, lay[l], tk, m[l])) break;
    record(l);
  }
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(val(tk.x[i]))) tk.status |= ST_NONFINITE;
  return tk;
}

// Gather and place the hits of track i from the [L][3][n] layout.
template <class T, class HT>
void gather_hits(const Geo& g, const Layer<T>* lay, const HT* hits, int64_t n, int64_t i, uint32_t mask, T (*m)[3]) {
  for (int l = 0; l < g.nl; ++l) {
    if (!(mask >> l & 1u)) { m[l][0] = 0.0; m[l][1] = 0.0; m[l][2] = 0.0; continue; }
    const HT* h = hits + (int64_t)l * 3 * n;
    place_hit(lay[l], (double)h[i], (double)h[n + i], (double)h[2 * n + i], m[l]);
  }
}

template <class T, class HT>
Track<T> fit_track_i(const Geo& g, const Layer<T>* lay, const HT* hits, int64_t n, int64_t i, uint32_t mask,
                     bool from_hits, const HT* seed_state, const HT* seed_cov, double* rec) {
  T m[32][3];
  gather_hits(g, lay, hits, n, i, mask, m);
  double sx[6], sC[36];
  if (!from_hits) {
    for (int k = 0; k < 6; ++k) sx[k] = (double)seed_state[(int64_t)k * n + i];
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b < 6; ++b) sC[a * 6 + b] = (double)seed_cov[(int64_t)tri(a, b) * n + i];
  }
  return fit_core<T>(g, lay, m, mask, from_hits, sx, sC, rec);
}

}  // namespace

// ==============================================================================
// C entry points (called from Python through ctypes)
// ==============================================================================
extern "C" {

// Threads the OpenMP loops of the batch entries use, and a setter (for the CPU
// scaling study; n < 1 restores the default).
int oracle_num_threads() { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : omp_get_num_procs()); }

// Crossing of one state with the cylinder |p - c| = r: writes the propagated state
// and the transverse arc; returns 1 on success, 0 if the layer is not reached.
int oracle_propagate(const double* state, double cx, double cy, double r, double B, double* out, double* s_out) {
  double kB = 0.299792458e-2 * B;
  double s;
  if (!crossing_arc<double>(state, cx, cy, r, kB, s)) return 0;
  helix_at<double>(state, s, kB, out);
  *s_out = s;
  return 1;
}

// Fixed-s transport Jacobian (row-major 6x6) of the state at arc s.
void oracle_transport_jacobian(const double* state, double s, double B, double* J) {
  double kB = 0.299792458e-2 * B;
  double xe[6], Jm[6][6];
  helix_at<double>(state, s, kB, xe);
  transport_jacobian<double>(state, xe, s, kB, Jm);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) J[i * 6 + j] = Jm[i][j];
}

// Helix map at fixed arc s (for finite-difference checks of the Jacobian).
void oracle_helix_at(const double* state, double s, double B, double* out) {
  helix_at<double>(state, s, 0.299792458e-2 * B, out);
}

// Measurement model of a state against a placed hit on a cylinder centred at
// (cx, cy): H (row-major 3x6) and the residual r (3).
void oracle_measurement(const double* state, double cx, double cy, const double* m, double* H, double* r) {
  Layer<double> ly{cx, cy, 0.0, 1.0, 0.0, 0.0, 0.0};
  Meas<double> me;
  measurement(ly, state, m, me);
  for (int i = 0; i < 18; ++i) H[i] = me.H[i];
  for (int i = 0; i < 3; ++i) r[i] = me.r[i];
}

// The same on the plane z = zd of a disk centred at (cx, cy): H and the residual
// (z_m - z_p, rho_p dphi, rho_m - rho_p).
void oracle_measurement_disk(const double* state, double cx, double cy, double zd, const double* m, double* H,
                             double* r) {
  Layer<double> ly{cx, cy, 0.0, 1.0, 0.0, 0.0, 0.0};
  ly.disk = true;
  ly.zd = zd;
  Meas<double> me;
  measurement(ly, state, m, me);
  for (int i = 0; i < 18; ++i) H[i] = me.H[i];
  for (int i = 0; i < 3; ++i) r[i] = me.r[i];
}

// Crossing of one state with the plane z = zd: the propagated state and the transverse
// arc; 1 on success, 0 if the plane is behind or beyond half a turn.
int oracle_propagate_disk(const double* state, double zd, double B, double* out, double* s_out) {
  const double kB = 0.299792458e-2 * B;
  Layer<double> ly{0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0};
  ly.disk = true;
  ly.zd = zd;
  double s;
  if (!plane_arc<double>(state, ly, kB, s)) return 0;
  helix_at<double>(state, s, kB, out);
  *s_out = s;
  return 1;
}

// Multiple-scattering covariance Q (row-major 6x6) at a state on a layer: a cylinder
// centred at (cx, cy), or (zd != 0) the disk in the plane z = zd.
void oracle_scattering(const OGeom* og, const double* state, double cx, double cy, double xX0, double zd,
                       double* Q) {
  Geo g = make_geo(og);
  Layer<double> ly{cx, cy, 0.0, 1.0, 0.0, xX0, 0.0};
  ly.disk = zd != 0.0;
  ly.zd = zd;
  double C[6][6] = {};
  add_scattering(g, ly, state, C);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Q[i * 6 + j] = C[i][j];
}

// Generic Kalman update (n <= 8, m <= 4), row-major matrices, in place on x and C.
int oracle_kalman_update(int n, int m, double* x, double* C, const double* H, const double* V, const double* r, double* chi2) {
  double c2;
  if (!kalman_update<double>(n, m, x, C, H, V, r, c2)) return 0;
  *chi2 = c2;
  return 1;
}

// The energy loss's map of kappa (loss_map): out = (kappa1, dkappa1/dkappa,
// dkappa1/dtheta) at path length xe; returns 0 if the particle stops.
int oracle_loss_map(const OGeom* og, double eloss, double kap, double th, double xe, double* out) {
  Geo g = make_geo(og);
  g.eloss = eloss;
  double k1, D, Tt;
  if (!loss_map<double>(g, kap, th, xe, k1, D, Tt)) return 0;
  out[0] = k1;
  out[1] = D;
  out[2] = Tt;
  return 1;
}

// Three-hit seed (state 6, covariance row-major 6x6) from three placed hits.
void oracle_seed(const OGeom* og, const double* m0, const double* m1, const double* m2, double* state, double* cov) {
  Geo g = make_geo(og);
  Track<double> tk;
  seed_from_hits(g, m0, m1, m2, tk);
  for (int i = 0; i < 6; ++i) state[i] = tk.x[i];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) cov[i * 6 + j] = tk.C[i][j];
}

// Batched fit.  hits [L][3][n] float32 in each layer's nominal frame; align [L][4]
// and xX0 [L] (either may be null: zero).  seed_from_hits != 0 builds each seed from
// hits 0-2; otherwise seed_state [6][n] and seed_cov [21][n] are used.  Outputs in
// float64: state [6][n], cov [21][n] (packed lower triangle, index i(i+1)/2 + j),
// chi2 [n], ndf [n] = 2 n_hits - 5, status [n]; rec (optional) [n][L][27] state and
// covariance after each processed layer (NaN elsewhere).
}  // extern "C"

namespace {
template <class HT>
void fit_batch(const OGeom* og, const double* align, const double* xX0, int64_t n, const HT* hits,
               const uint32_t* mask, int seed_from_hits_flag, const HT* seed_state, const HT* seed_cov,
               double* state, double* cov, double* chi2, int32_t* ndf, uint32_t* status, double* rec,
               const double* map = nullptr, int map_nz = 0, double eloss = 0.0, double fr = 0.0,
               double fz = 0.0) {
  Geo g = make_geo(og);
  g.map = map;
  g.map_nz = map_nz;
  g.eloss = eloss;
  g.fr = fr;
  g.fz = fz;
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double* r = nullptr;
    if (rec) {
      r = rec + i * (int64_t)g.nl * 27;
      for (int64_t k = 0; k < (int64_t)g.nl * 27; ++k) r[k] = std::numeric_limits<double>::quiet_NaN();
    }
    Track<double> tk = fit_track_i<double, HT>(g, lay, hits, n, i, mask[i], seed_from_hits_flag != 0, seed_state, seed_cov, r);
    for (int k = 0; k < 6; ++k) state[k * n + i] = tk.x[k];
    for (int a = 0; a < 6; ++a)
      for (int b = 0; b <= a; ++b) cov[(int64_t)tri(a, b) * n + i] = tk.C[a][b];
    chi2[i] = tk.chi2;
    ndf[i] = 2 * tk.n - 5;
    status[i] = tk.status;
  }
}
}  // namespace

extern "C" {

void oracle_fit(const OGeom* og, const double* align, const double* xX0, int64_t n, const float* hits,
                const uint32_t* mask, int seed_from_hits_flag, const float* seed_state, const float* seed_cov,
                double* state, double* cov, double* chi2, int32_t* ndf, uint32_t* status, double* rec) {
  fit_batch<float>(og, align, xX0, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, state, cov, chi2, ndf,
                   status, rec);
}

// As oracle_fit with the detector model of Sec. 3: map [L][map_nz] of x/X0 (null: the
// per-layer xX0), the mean ionisation loss per radiation length eloss (0: none) and
// the field B_z(r, z) = B (1 + fr r^2 + fz z^2) (0, 0: uniform).
void oracle_fit_model(const OGeom* og, const double* align, const double* xX0, const double* map, int map_nz,
                      double eloss, double fr, double fz, int64_t n, const float* hits, const uint32_t* mask,
                      int seed_from_hits_flag, const float* seed_state, const float* seed_cov, double* state,
                      double* cov, double* chi2, int32_t* ndf, uint32_t* status, double* rec) {
  fit_batch<float>(og, align, xX0, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, state, cov, chi2, ndf,
                   status, rec, map, map_nz, eloss, fr, fz);
}

// The same with float64 hits and seeds (noiseless checks finer than float32).
void oracle_fit_model_f64(const OGeom* og, const double* align, const double* xX0, const double* map, int map_nz,
                          double eloss, double fr, double fz, int64_t n, const double* hits, const uint32_t* mask,
                          int seed_from_hits_flag, const double* seed_state, const double* seed_cov, double* state,
                          double* cov, double* chi2, int32_t* ndf, uint32_t* status, double* rec) {
  fit_batch<double>(og, align, xX0, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, state, cov, chi2, ndf,
                    status, rec, map, map_nz, eloss, fr, fz);
}

// One material step on a state at its crossing with layer l (align [4] and xX0 of
// that layer, either may be null): x [6] and C [36] in, updated in place.  Returns 0
// if the particle stops.
int oracle_material_step(const OGeom* og, int l, const double* align, double xX0, const double* map, int map_nz,
                         double eloss, double* x, double* C) {
  Geo g = make_geo(og);
  g.map = map;
  g.map_nz = map_nz;
  g.eloss = eloss;
  Layer<double> lay[32];
  double al[32 * 4] = {};
  double xx[32] = {};
  if (align)
    for (int q = 0; q < 4; ++q) al[4 * l + q] = align[q];
  xx[l] = xX0;
  make_layers<double>(g, al, xx, lay);
  double Cm[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Cm[i][j] = C[i * 6 + j];
  const bool ok = material_step(g, lay[l], x, Cm);
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i * 6 + j] = Cm[i][j];
  return ok ? 1 : 0;
}

// As oracle_fit with float64 hits and seeds (for noiseless checks finer than float32).
void oracle_fit_f64(const OGeom* og, const double* align, const double* xX0, int64_t n, const double* hits,
                    const uint32_t* mask, int seed_from_hits_flag, const double* seed_state, const double* seed_cov,
                    double* state, double* cov, double* chi2, int32_t* ndf, uint32_t* status, double* rec) {
  fit_batch<double>(og, align, xX0, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, state, cov, chi2, ndf,
                    status, rec);
}

// Weighted total chi2, sum_i weight[i] * chi2_i (weight may be null: all ones),
// summed in track order, seeds built from hits.  For central finite differences.
double oracle_total_chi2(const OGeom* og, const double* align, const double* xX0, int64_t n, const float* hits,
                         const uint32_t* mask, const double* weight, double fr, double fz, const double* map,
                         int32_t map_nz, double eloss) {
  Geo g = make_geo(og);
  g.fr = fr;
  g.fz = fz;
  g.map = map;
  g.map_nz = map ? map_nz : 0;
  g.eloss = eloss;
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  std::vector<double> c(n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    Track<double> tk = fit_track_i<double, float>(g, lay, hits, n, i, mask[i], true, nullptr, nullptr, nullptr);
    c[i] = tk.chi2;
  }
  double acc = 0;
  for (int64_t i = 0; i < n; ++i) acc += (weight ? weight[i] : 1.0) * c[i];
  return acc;
}

// Gradient of sum_i weight[i] chi2_i with respect to align [L][4] and xX0 [L], by
// forward-mode dual numbers through the whole fit (seeds built from the placed
// hits), one layer's five parameters per pass.
// fr, fz: the parameterised field B_z(r, z) = B (1 + fr r^2 + fz z^2).  Each step's field
// is taken at its start and the seed's at hit 0, points that move with the parameters;
// the dual numbers carry that dependence, so this is the exact derivative of the total
// chi2 that oracle_total_chi2 evaluates.
// The material model (map [L][nz] or null, eloss) enters as in the fit; with a map,
// g_xX0[l] is the derivative with respect to an additive offset of the map's row l (the
// per-layer xX0 is then not used).
void oracle_fit_grad(const OGeom* og, const double* align, const double* xX0, int64_t n, const float* hits,
                     const uint32_t* mask, const double* weight, double* g_align, double* g_xX0, double fr,
                     double fz, const double* map, int32_t map_nz, double eloss) {
  using D = Dual<5>;
  Geo g = make_geo(og);
  g.fr = fr;
  g.fz = fz;
  g.map = map;
  g.map_nz = map ? map_nz : 0;
  g.eloss = eloss;
  for (int pl = 0; pl < g.nl; ++pl) {
    D al[32 * 4], xx[32];
    for (int l = 0; l < g.nl; ++l) {
      for (int k = 0; k < 4; ++k) al[4 * l + k] = D(align ? align[4 * l + k] : 0.0);
      xx[l] = D(xX0 ? xX0[l] : 0.0);
    }
    for (int k = 0; k < 4; ++k) al[4 * pl + k].d[k] = 1.0;
    if (!map) xx[pl].d[4] = 1.0;
    Layer<D> lay[32];
    make_layers<D>(g, al, xx, lay);
    if (map) lay[pl].moff.d[4] = 1.0;
    std::vector<double> part((size_t)n * 5);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      Track<D> tk = fit_track_i<D, float>(g, lay, hits, n, i, mask[i], true, nullptr, nullptr, nullptr);
      double w = weight ? weight[i] : 1.0;
      for (int k = 0; k < 5; ++k) part[(size_t)i * 5 + k] = w * tk.chi2.d[k];
    }
    double acc[5] = {0, 0, 0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < 5; ++k) acc[k] += part[(size_t)i * 5 + k];
    for (int k = 0; k < 4; ++k) g_align[4 * pl + k] = acc[k];
    g_xX0[pl] = acc[4];
  }
}

}  // extern "C"

// ==============================================================================
// combinatorial track finder
// ==============================================================================
namespace {

struct BinnedLayer {
  std::vector<double> phi, z;   // azimuth about the layer axis and z of each binned hit
  std::vector<int64_t> idx;     // global hit index, in bin order
  std::vector<int64_t> off;     // [nphi * nz + 1]
  int64_t begin = 0, end = 0;   // the layer's slice of the global hit arrays
};

int64_t bin_floor(double v, double lo, double span, int nb) {
  return (int64_t)std::floor((v - lo) * nb / span);
}
int clamp_bin(int64_t b, int nb) { return (int)(b < 0 ? 0 : (b > nb - 1 ? nb - 1 : b)); }

struct Cand {
  Track<double> tk;
  int nmiss = 0;
  bool term = false;
  std::vector<int32_t> hist;
};

struct Branch {
  int parent;
  int kind;      // 0 hit, 1 miss, 2 carry (terminated parent), 3 pass (a bounded surface not crossed)
  int64_t hit;
  int nhits;
  double chi2tot, chi2h;
};

// Candidate score: more hits first, then smaller total chi2, then the parent's
// rank, then the hit's index (the miss branch after every hit branch).
bool branch_less(const Branch& a, const Branch& b) {
  if (a.nhits != b.nhits) return a.nhits > b.nhits;
  if (a.chi2tot != b.chi2tot) return a.chi2tot < b.chi2tot;
  if (a.parent != b.parent) return a.parent < b.parent;
  int64_t ha = a.kind == 0 ? a.hit : std::numeric_limits<int64_t>::max();
  int64_t hb = b.kind == 0 ? b.hit : std::numeric_limits<int64_t>::max();
  return ha < hb;
}

struct FindCfg {
  double chi2_cut, nsigma, tol_abs, tol_rel, tol_win;
  int keep, max_miss;
  bool brute;
};

// Relative margin by which the helix of state x clears (> 0) or misses (< 0) the
// cylinder of layer ly: its circle reaches |centre - axis| + R from the axis.
double reach_margin(const Geo& g, const Layer<double>& ly, const double x[6]) {
  double w = -kB_at<double>(g, x[0], x[1], x[2]) * x[3];
  if (w == 0) return 1.0;
  double R = 1.0 / std::fabs(w);
  double cx = x[0] - std::sin(x[4]) / w - ly.cx, cy = x[1] + std::cos(x[4]) / w - ly.cy;
  return (std::sqrt(cx * cx + cy * cy) + R - ly.r) / ly.r;
}

struct EventView {
  const float* hits;  // [3][H]
  int64_t H;
  const int64_t* off;  // [L+1] of this event
};

void place_global(const Layer<double>& ly, const EventView& ev, int64_t j, double m[3]) {
  place_hit(ly, (double)ev.hits[j], (double)ev.hits[ev.H + j], (double)ev.hits[2 * ev.H + j], m);
}

// phi/z bins of one layer of one event: counting sort, stable in hit index.
void bin_layer(const Geo& g, const Layer<double>& ly, int l, const EventView& ev, BinnedLayer& B) {
  const int nphi = g.nphi, nz = g.nz, nb = nphi * nz;
  B.begin = ev.off[l];
  B.end = ev.off[l + 1];
  int64_t nh = B.end - B.begin;
  std::vector<int> bin(nh);
  std::vector<double> ph(nh), zz(nh);
  for (int64_t j = 0; j < nh; ++j) {
    double m[3];
    place_global(ly, ev, B.begin + j, m);
    ph[j] = std::atan2(m[1] - val(ly.cy), m[0] - val(ly.cx));
    // the bins' second coordinate: z on a cylinder, the radius about the axis on a disk
    zz[j] = ly.disk ? std::hypot(m[0] - val(ly.cx), m[1] - val(ly.cy)) : m[2];
    const double lo2 = ly.disk ? ly.rmin : -g.zhalf[l], span2 = ly.disk ? ly.rmax - ly.rmin : 2 * g.zhalf[l];
    int bp = clamp_bin(bin_floor(ph[j], -kPi, 2 * kPi, nphi), nphi);
    int bz = clamp_bin(bin_floor(zz[j], lo2, span2, nz), nz);
    bin[j] = bp * nz + bz;
  }
  B.off.assign(nb + 1, 0);
  for (int64_t j = 0; j < nh; ++j) B.off[bin[j] + 1]++;
  for (int b = 0; b < nb; ++b) B.off[b + 1] += B.off[b];
  std::vector<int64_t> cur(B.off.begin(), B.off.end() - 1);
  B.phi.resize(nh); B.z.resize(nh); B.idx.resize(nh);
  for (int64_t j = 0; j < nh; ++j) {
    int64_t p = cur[bin[j]]++;
    B.phi[p] = ph[j]; B.z[p] = zz[j]; B.idx[p] = B.begin + j;
  }
}

// chi2 of a placed hit against a prediction whose S^-1 is known.
double hit_chi2(const Layer<double>& ly, const double x[6], const double Si[9], const double m[3]) {
  Meas<double> me;
  measurement(ly, x, m, me);
  double c = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) c += me.r[i] * Si[i * 3 + j] * me.r[j];
  return c < 0 ? 0 : c;
}

// One seed through layers 3 .. L-1.  Returns the candidates in rank order; ambig gets
// bit L set when some decision on layer L that can change the set of surviving
// candidates lies within the FP32 tolerance of its threshold: a helix grazing the
// layer (reach margin below 1e-4), a chi2 near the cut, a hit near a window edge, or
// the last kept and first dropped branch scores near a tie.
// work (optional) counts what the search does for the seed: [0] predictions that reach
// their layer, [1] hits inside a window (each gets a chi2), [2] updates of surviving
// hit branches, [3] the seed refit (1 per seed).
std::vector<Cand> find_seed(const Geo& g, const Layer<double>* lay, const FindCfg& o, const EventView& ev,
                            const std::vector<BinnedLayer>& bl, const int32_t sh[3], uint32_t& ambig,
                            int64_t* work = nullptr) {
  ambig = 0;
  int64_t wk[4] = {0, 0, 0, 1};
  std::vector<Cand> cands;
  Cand c0;
  c0.hist.assign(g.nl, -2);
  double m[3][3];
  for (int l = 0; l < 3; ++l) { place_global(lay[l], ev, sh[l], m[l]); c0.hist[l] = sh[l]; }
  seed_from_hits(g, m[0], m[1], m[2], c0.tk);
  bool ok = update_with_hit(g, lay[0], c0.tk, m[0]);
  for (int l = 1; ok && l < 3; ++l) {
    ok = predict(g, lay[l], c0.tk);
    if (ok) ok = update_with_hit(g, lay[l], c0.tk, m[l]);
  }
  if (!ok) c0.term = true;
  cands.push_back(c0);
  const int nphi = g.nphi, nz = g.nz;
  auto tol = [&](double c) { return o.tol_abs + o.tol_rel * std::fabs(c); };
  for (int L = 3; L < g.nl; ++L) {
    const Layer<double>& ly = lay[L];
    const BinnedLayer& B = bl[L];
    std::vector<Branch> br;
    std::vector<Track<double>> pred(cands.size());
    for (size_t k = 0; k < cands.size(); ++k) {
      Cand& cd = cands[k];
      if (cd.term) { br.push_back({(int)k, 2, -1, cd.tk.n, cd.tk.chi2, 0.0}); continue; }
      // reaching the layer at all is FP32-sensitive for a helix that grazes it
      if (!ly.disk && std::fabs(reach_margin(g, ly, cd.tk.x)) < 1e-4) ambig |= 1u << L;
      Track<double> p = cd.tk;
      if (ly.bounded()) {
        // a bounded surface that the candidate does not reach, or reaches outside its
        // active area, is passed over: the candidate goes on unchanged (no miss).  A
        // crossing within 0.01 cm of the area's edge is an FP32-sensitive decision.
        bool cross = predict(g, ly, p);
        if (cross) {
          const double c2 = ly.disk ? std::hypot(p.x[0] - ly.cx, p.x[1] - ly.cy) : std::fabs(p.x[2] - ly.dz);
          const double lo = ly.disk ? ly.rmin : -1.0, hi = ly.disk ? ly.rmax : ly.zmax;
          if (std::fabs(c2 - hi) < 0.01 || (ly.disk && std::fabs(c2 - lo) < 0.01)) ambig |= 1u << L;
          cross = c2 <= hi && (!ly.disk || c2 >= lo);
        } else if (ly.disk && std::fabs(std::cos(cd.tk.x[5])) < 1e-6) {
          ambig |= 1u << L;  // a track along the plane: which side it heads to is FP32-sensitive
        }
        if (!cross) {
          br.push_back({(int)k, 3, -1, cd.tk.n, cd.tk.chi2, 0.0});
          continue;
        }
      } else if (!predict(g, ly, p)) {
        // no crossing (the state is untouched), or the particle stops in the layer's
        // material (it ends with the prediction transported to the layer)
        cd.tk = p;
        cd.term = true;
        cd.tk.status |= ST_PROP_FAIL;
        br.push_back({(int)k, 2, -1, cd.tk.n, cd.tk.chi2, 0.0});
        continue;
      }
      pred[k] = p;
      ++wk[0];
      // S at the prediction: the frame and H belong to the prediction, so S is shared
      // by every hit of the window.
      Meas<double> me;
      double self[3] = {p.x[0], p.x[1], p.x[2]};
      measurement(ly, p.x, self, me);
      double HC[18], S[9], Si[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 6; ++j) {
          double a = 0;
          for (int q = 0; q < 6; ++q) a += me.H[i * 6 + q] * p.C[q][j];
          HC[i * 6 + j] = a;
        }
      double V[3] = {g.sr * g.sr, g.srphi * g.srphi, g.sz * g.sz};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double a = i == j ? V[i] : 0.0;
          for (int q = 0; q < 6; ++q) a += HC[i * 6 + q] * me.H[j * 6 + q];
          S[i * 3 + j] = a;
        }
      if (!invert(3, S, Si)) {
        cd.term = true;
        cd.tk.status |= ST_NONFINITE;
        br.push_back({(int)k, 2, -1, cd.tk.n, cd.tk.chi2, 0.0});
        continue;
      }
      double wphi = o.nsigma * std::sqrt(S[4]) / me.rho;
      double wz = o.nsigma * std::sqrt(S[8]);
      // the window's second coordinate: z on a cylinder, the radius on a disk
      double phip = me.phip, zp = ly.disk ? me.rho : p.x[2];
      auto consider = [&](int64_t j, double phih, double zh) {
        double dphi = wrap_pi(phih - phip), dz = zh - zp;
        double ephi = std::fabs(dphi) - wphi, ez = std::fabs(dz) - wz;
        bool inside = ephi <= 0 && ez <= 0;
        bool near_edge = (std::fabs(ephi) <= o.tol_win * wphi && ez <= o.tol_win * wz) ||
                         (std::fabs(ez) <= o.tol_win * wz && ephi <= o.tol_win * wphi);
        if (!inside && !near_edge) return;
        double mh[3];
        place_global(ly, ev, j, mh);
        double c = hit_chi2(ly, p.x, Si, mh);
        if (near_edge && c < o.chi2_cut + tol(o.chi2_cut)) ambig |= 1u << L;
        if (!inside) return;
        ++wk[1];
        if (std::fabs(c - o.chi2_cut) <= tol(o.chi2_cut)) ambig |= 1u << L;
        if (c < o.chi2_cut) br.push_back({(int)k, 0, j, cd.tk.n + 1, cd.tk.chi2 + c, c});
      };
      if (o.brute) {
        for (int64_t j = B.begin; j < B.end; ++j) {
          double mh[3];
          place_global(ly, ev, j, mh);
          consider(j, std::atan2(mh[1] - ly.cy, mh[0] - ly.cx),
                   ly.disk ? std::hypot(mh[0] - ly.cx, mh[1] - ly.cy) : mh[2]);
        }
      } else {
        // every bin that can hold a hit within (1 + tol_win) of the window, and more
        double wq = (1.0 + 2 * o.tol_win) * wphi + 1e-6;
        double zq = (1.0 + 2 * o.tol_win) * wz + 1e-6;
        const double lo2 = ly.disk ? ly.rmin : -g.zhalf[L], span2 = ly.disk ? ly.rmax - ly.rmin : 2 * g.zhalf[L];
        int zlo = clamp_bin(bin_floor(zp - zq, lo2, span2, nz), nz);
        int zhi = clamp_bin(bin_floor(zp + zq, lo2, span2, nz), nz);
        int64_t blo = 0, bhi = nphi - 1;
        if (wq < kPi) {
          blo = bin_floor(phip - wq, -kPi, 2 * kPi, nphi);
          bhi = bin_floor(phip + wq, -kPi, 2 * kPi, nphi);
          if (bhi - blo + 1 >= nphi) { blo = 0; bhi = nphi - 1; }
        }
        for (int64_t b = blo; b <= bhi; ++b) {
          int pb = (int)(((b % nphi) + nphi) % nphi);
          for (int64_t q = B.off[pb * nz + zlo]; q < B.off[pb * nz + zhi + 1]; ++q) consider(B.idx[q], B.phi[q], B.z[q]);
        }
      }
      br.push_back({(int)k, 1, -1, cd.tk.n, cd.tk.chi2, 0.0});
    }
    std::sort(br.begin(), br.end(), branch_less);
    size_t nk = std::min<size_t>((size_t)o.keep, br.size());
    // Which branches survive is decided at the boundary between the last kept and the
    // first dropped branch; near-ties among kept branches only relabel ranks.
    if (br.size() > nk) {
      const Branch& a = br[nk - 1];
      const Branch& b = br[nk];
      if (a.nhits == b.nhits && std::fabs(a.chi2tot - b.chi2tot) <= tol(std::max(a.chi2tot, b.chi2tot)))
        ambig |= 1u << L;
    }
    std::vector<Cand> next;
    for (size_t i = 0; i < nk; ++i) {
      const Branch& b = br[i];
      Cand nc = cands[b.parent];
      if (b.kind == 1) {
        nc.tk = pred[b.parent];
        nc.nmiss += 1;
        nc.hist[L] = -1;
        if (nc.nmiss >= o.max_miss) { nc.term = true; nc.tk.status |= ST_TERM_MISSES; }
      } else if (b.kind == 3) {
        nc.hist[L] = -2;  // a bounded surface passed over: unchanged, no miss
      } else if (b.kind == 0) {
        nc.tk = pred[b.parent];
        double mh[3];
        place_global(ly, ev, b.hit, mh);
        if (!update_with_hit(g, ly, nc.tk, mh)) nc.term = true;
        ++wk[2];
        nc.tk.chi2 = b.chi2tot;
        nc.hist[L] = (int32_t)b.hit;
      }
      next.push_back(std::move(nc));
    }
    cands.swap(next);
  }
  if (work)
    for (int q = 0; q < 4; ++q) work[q] += wk[q];
  return cands;
}

}  // namespace

extern "C" {

// Combinatorial search of every seed of every event, then (refit != 0) a fit of each
// seed's rank-0 candidate from its own hits.
//   hit_off [E][L+1] slices of the global hits [3][H] per event and layer;
//   seed_event [S], seed_hits [3][S] global indices of the seed's hits on layers 0-2;
//   brute != 0 tests every hit of a layer instead of the phi/z bins.
// Outputs (k < keep slots per seed, unused slots zero / -2):
//   n_cand [S]; hit_idx [keep][L][S] (global index, -1 missing layer, -2 not reached);
//   n_hits, n_miss [keep][S]; chi2 [keep][S]; state [keep][6][S]; cov [keep][21][S];
//   status [keep][S]; ambig [S] (bit L: an FP32-sensitive decision on layer L);
//   rf_* [S]: refit of rank 0 (may be null).
// The detector model of Sec. 3 for the finder (null: one x/X0 per layer, uniform field).
struct OModel {
  const double* map;  // [L][nz] x/X0 at z-bin centres, or null
  int32_t nz, pad;
  double eloss, fr, fz;
};

}  // extern "C"

namespace {
void set_model(Geo& g, const OModel* model) {
  if (!model) return;
  g.map = model->map;
  g.map_nz = model->nz;
  g.eloss = model->eloss;
  g.fr = model->fr;
  g.fz = model->fz;
}
}  // namespace

extern "C" {

void oracle_find(const OGeom* og, const double* align, const double* xX0, const OModel* model, int32_t n_events,
                 const int64_t* hit_off,
                 int64_t n_hits_total, const float* hits, int64_t n_seeds, const int32_t* seed_event,
                 const int32_t* seed_hits, double chi2_cut, double nsigma, int32_t keep, int32_t max_miss,
                 int32_t brute, double tol_abs, double tol_rel, double tol_win, int32_t* n_cand, int32_t* hit_idx,
                 int32_t* n_hits, int32_t* n_miss, double* chi2, double* state, double* cov, uint32_t* status,
                 uint32_t* ambig, double* rf_state, double* rf_cov, double* rf_chi2, int32_t* rf_ndf,
                 uint32_t* rf_status, int64_t* work) {
  Geo g = make_geo(og);
  set_model(g, model);
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  const int L = g.nl;
  std::vector<std::vector<BinnedLayer>> bins(n_events, std::vector<BinnedLayer>(L));
#pragma omp parallel for schedule(dynamic)
  for (int e = 0; e < n_events; ++e) {
    EventView ev{hits, n_hits_total, hit_off + (int64_t)e * (L + 1)};
    for (int l = 0; l < L; ++l) bin_layer(g, lay[l], l, ev, bins[e][l]);
  }
  FindCfg o{chi2_cut, nsigma, tol_abs, tol_rel, tol_win, keep, max_miss, brute != 0};
  const int64_t S = n_seeds;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t s = 0; s < S; ++s) {
    int e = seed_event[s];
    EventView ev{hits, n_hits_total, hit_off + (int64_t)e * (L + 1)};
    int32_t sh[3] = {seed_hits[s], seed_hits[S + s], seed_hits[2 * S + s]};
    uint32_t amb = 0;
    int64_t wk[4] = {0, 0, 0, 0};
    std::vector<Cand> cs = find_seed(g, lay, o, ev, bins[e], sh, amb, work ? wk : nullptr);
    if (work)
      for (int q = 0; q < 4; ++q) {
#pragma omp atomic
        work[q] += wk[q];
      }
    ambig[s] = amb;
    n_cand[s] = (int32_t)cs.size();
    for (int k = 0; k < keep; ++k) {
      bool have = k < (int)cs.size();
      for (int l = 0; l < L; ++l) hit_idx[((int64_t)k * L + l) * S + s] = have ? cs[k].hist[l] : -2;
      n_hits[(int64_t)k * S + s] = have ? cs[k].tk.n : 0;
      n_miss[(int64_t)k * S + s] = have ? cs[k].nmiss : 0;
      chi2[(int64_t)k * S + s] = have ? cs[k].tk.chi2 : 0.0;
      status[(int64_t)k * S + s] = have ? cs[k].tk.status : 0u;
      for (int i = 0; i < 6; ++i) state[((int64_t)k * 6 + i) * S + s] = have ? cs[k].tk.x[i] : 0.0;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b <= a; ++b) cov[((int64_t)k * 21 + tri(a, b)) * S + s] = have ? cs[k].tk.C[a][b] : 0.0;
    }
    if (rf_state) {
      double m[32][3];
      uint32_t mask = 0;
      for (int l = 0; l < L; ++l) {
        int32_t h = cs[0].hist[l];
        if (h >= 0) { mask |= 1u << l; place_global(lay[l], ev, h, m[l]); }
        else { m[l][0] = m[l][1] = m[l][2] = 0.0; }
      }
      Track<double> tk = fit_core<double>(g, lay, m, mask, true, nullptr, nullptr, nullptr);
      for (int i = 0; i < 6; ++i) rf_state[(int64_t)i * S + s] = tk.x[i];
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b <= a; ++b) rf_cov[(int64_t)tri(a, b) * S + s] = tk.C[a][b];
      rf_chi2[s] = tk.chi2;
      rf_ndf[s] = 2 * tk.n - 5;
      rf_status[s] = tk.status;
    }
  }
}

}  // extern "C"

// ==============================================================================
// Fixed-interval smoother (Rauch-Tung-Striebel) over the forward fit
// ==============================================================================
// The paper's chain ends with a backward pass and a final fit of the built tracks
// (Sec. 4.2, Sec. 5).  Read here as the textbook RTS smoother on the filter's own
// linearisation: with the filtered state x_f(l), C_f(l) after layer l, the
// prediction x_p(l+1), C_p(l+1) = J C_f(l) J^T + Q at layer l+1 (J the fixed-arc
// transport Jacobian of that step) and the smoothed x_s(l+1), C_s(l+1),
//   G      = C_f(l) J^T C_p(l+1)^-1,
//   x_s(l) = x_f(l) + G (x_s(l+1) - x_p(l+1))      (azimuth difference wrapped),
//   C_s(l) = C_f(l) + G (C_s(l+1) - C_p(l+1)) G^T,
// from the last layer with a hit (x_s = x_f there) down to layer 0.  Layers without
// a hit inside that range take part with their prediction as the filtered state.

namespace {

// Gauss-Jordan inverse with partial pivoting for n <= 6 (dense, row-major).
bool invert_dense(int n, const double* A, double* Ai) {
  double M[6][12];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) M[i][j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(M[c][j], M[piv][j]);
    double inv = 1.0 / M[c][c];
    for (int j = 0; j < 2 * n; ++j) M[c][j] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = M[r][c];
      for (int j = 0; j < 2 * n; ++j) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ai[i * n + j] = M[i][n + j];
  return true;
}

// One RTS step for an n-dim state (n <= 6), dense row-major matrices.  wrap_idx >= 0
// names a state component that is an angle (its difference is wrapped to (-pi, pi]).
bool rts_step(int n, const double* xf, const double* Cf, const double* J, const double* xp, const double* Cp,
              const double* xs1, const double* Cs1, double* xs, double* Cs, int wrap_idx) {
  double Cpi[36], CJt[36], G[36], E[36], GE[36];
  if (!invert_dense(n, Cp, Cpi)) return false;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double a = 0;
      for (int k = 0; k < n; ++k) a += Cf[i * n + k] * J[j * n + k];
      CJt[i * n + j] = a;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double a = 0;
      for (int k = 0; k < n; ++k) a += CJt[i * n + k] * Cpi[k * n + j];
      G[i * n + j] = a;
    }
  double d[6];
  for (int i = 0; i < n; ++i) d[i] = xs1[i] - xp[i];
  if (wrap_idx >= 0) d[wrap_idx] = wrap_pi(d[wrap_idx]);
  for (int i = 0; i < n; ++i) {
    double a = xf[i];
    for (int k = 0; k < n; ++k) a += G[i * n + k] * d[k];
    xs[i] = a;
  }
  if (wrap_idx >= 0) xs[wrap_idx] = wrap_pi(xs[wrap_idx]);
  for (int i = 0; i < n * n; ++i) E[i] = Cs1[i] - Cp[i];
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double a = 0;
      for (int k = 0; k < n; ++k) a += G[i * n + k] * E[k * n + j];
      GE[i * n + j] = a;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double a = Cf[i * n + j];
      for (int k = 0; k < n; ++k) a += GE[i * n + k] * G[j * n + k];
      Cs[i * n + j] = a;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) { double a = 0.5 * (Cs[i * n + j] + Cs[j * n + i]); Cs[i * n + j] = a; Cs[j * n + i] = a; }
  return true;
}

// Forward fit of one track keeping, for every processed layer, the filtered state
// and covariance and (from layer 1) the Jacobian and the prediction; then the RTS
// pass.  Writes smoothed states/covariances for layers 0..lend (lend = last layer
// with an update, -1 if none) and returns the forward status.
uint32_t smooth_track(const Geo& g, const Layer<double>* lay, const double (*m)[3], uint32_t mask, bool from_hits,
                      const double* seed_x, const double* seed_C, double (*xs)[6], double (*Cs)[36], int& lend) {
  static thread_local double xf[32][6], Cf[32][36], xp[32][6], Cp[32][36], Jl[32][36];
  Track<double> tk;
  for (int i = 0; i < 6; ++i) { tk.x[i] = 0.0; for (int j = 0; j < 6; ++j) tk.C[i][j] = 0.0; }
  tk.chi2 = 0.0; tk.n = 0; tk.status = 0;
  lend = -1;
  uint32_t need = from_hits ? 7u : 1u;
  if ((mask & need) != need) return ST_BAD_INPUT;
  if (from_hits) {
    seed_from_hits(g, m[0], m[1], m[2], tk);
  } else {
    for (int i = 0; i < 6; ++i) tk.x[i] = seed_x[i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) tk.C[i][j] = seed_C[i * 6 + j];
  }
  auto keep = [&](double (*xo)[6], double (*Co)[36], int l) {
    for (int i = 0; i < 6; ++i) xo[l][i] = tk.x[i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) Co[l][i * 6 + j] = tk.C[i][j];
  };
  if (!update_with_hit(g, lay[0], tk, m[0])) return tk.status;
  keep(xf, Cf, 0);
  lend = 0;
  int last = 31 - __builtin_clz(mask);
  if (last >= g.nl) last = g.nl - 1;
  for (int l = 1; l <= last; ++l) {
    double J[6][6];
    if (!predict(g, lay[l], tk, J)) break;
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) Jl[l][i * 6 + j] = J[i][j];
    keep(xp, Cp, l);
    if (mask >> l & 1u) {
      if (!update_with_hit(g, lay[l], tk, m[l])) break;
      lend = l;
    }
    keep(xf, Cf, l);
  }
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(tk.x[i])) tk.status |= ST_NONFINITE;
  if (lend < 0) return tk.status;
  for (int i = 0; i < 6; ++i) xs[lend][i] = xf[lend][i];
  for (int i = 0; i < 36; ++i) Cs[lend][i] = Cf[lend][i];
  for (int l = lend - 1; l >= 0; --l)
    if (!rts_step(6, xf[l], Cf[l], Jl[l + 1], xp[l + 1], Cp[l + 1], xs[l + 1], Cs[l + 1], xs[l], Cs[l], 4)) {
      tk.status |= ST_NONFINITE;
      break;
    }
  return tk.status;
}

// The RTS pass alone over filtered estimates supplied by the caller (x_f, C_f at
// layers 0..lend, for instance another implementation's forward fit): the
// prediction of layer l+1 from x_f(l), C_f(l) is made as in the forward fit, then the
// step above.  Returns the lowest layer reached (lend if layer lend's predecessor
// already fails, -1 if lend < 0).
int smooth_from_filtered(const Geo& g, const Layer<double>* lay, int lend, const double (*xf)[6],
                         const double (*Cf)[36], double (*xs)[6], double (*Cs)[36]) {
  if (lend < 0) return -1;
  for (int i = 0; i < 6; ++i) xs[lend][i] = xf[lend][i];
  for (int i = 0; i < 36; ++i) Cs[lend][i] = Cf[lend][i];
  int first = lend;
  for (int l = lend - 1; l >= 0; --l) {
    Track<double> tk;
    for (int i = 0; i < 6; ++i) tk.x[i] = xf[l][i];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) tk.C[i][j] = Cf[l][i * 6 + j];
    tk.chi2 = 0.0; tk.n = 0; tk.status = 0;
    double J[6][6];
    if (!predict(g, lay[l + 1], tk, J)) break;
    double Cp[36];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) Cp[i * 6 + j] = tk.C[i][j];
    if (!rts_step(6, xf[l], Cf[l], &J[0][0], tk.x, Cp, xs[l + 1], Cs[l + 1], xs[l], Cs[l], 4)) break;
    first = l;
  }
  return first;
}

}  // namespace

extern "C" {

// The RTS pass alone (smooth_from_filtered) for a batch: xf [L][6][n] and Cf
// [L][21][n] (packed lower triangle) hold the filtered estimates after each layer,
// lend [n] the last updated layer (-1: none).  Outputs as oracle_smooth for layers
// first[i]..lend[i] (zero elsewhere) and first [n] (-1 if lend < 0).
void oracle_smooth_filtered(const OGeom* og, const double* align, const double* xX0, const OModel* model, int64_t n,
                            const int32_t* lend, const double* xf, const double* Cf, double* xs_out,
                            double* Cs_out, int32_t* first_out) {
  Geo g = make_geo(og);
  set_model(g, model);
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  const int L = g.nl;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double x[32][6], C[32][36], xs[32][6], Cs[32][36];
    const int le = lend[i] < L ? lend[i] : L - 1;
    for (int l = 0; l <= le; ++l) {
      for (int k = 0; k < 6; ++k) x[l][k] = xf[((int64_t)l * 6 + k) * n + i];
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) C[l][a * 6 + b] = Cf[((int64_t)l * 21 + tri(a, b)) * n + i];
    }
    const int first = smooth_from_filtered(g, lay, le, x, C, xs, Cs);
    first_out[i] = first;
    for (int l = 0; l < L; ++l) {
      const bool have = first >= 0 && l >= first && l <= le;
      for (int k = 0; k < 6; ++k) xs_out[((int64_t)l * 6 + k) * n + i] = have ? xs[l][k] : 0.0;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b <= a; ++b) Cs_out[((int64_t)l * 21 + tri(a, b)) * n + i] = have ? Cs[l][a * 6 + b] : 0.0;
    }
  }
}

// One RTS step for an n-dim state (n <= 6), dense row-major; returns 0 if C_p is
// singular.  wrap_idx: index of an angle component or -1.
int oracle_rts_step(int n, const double* xf, const double* Cf, const double* J, const double* xp, const double* Cp,
                    const double* xs1, const double* Cs1, double* xs, double* Cs, int wrap_idx) {
  return rts_step(n, xf, Cf, J, xp, Cp, xs1, Cs1, xs, Cs, wrap_idx) ? 1 : 0;
}

}  // extern "C"

namespace {
template <class HT>
void smooth_batch(const OGeom* og, const double* align, const double* xX0, const OModel* model, int64_t n,
                  const HT* hits, const uint32_t* mask, int seed_from_hits_flag, const HT* seed_state,
                  const HT* seed_cov, double* xs_out, double* Cs_out, int32_t* lend_out, uint32_t* status) {
  Geo g = make_geo(og);
  set_model(g, model);
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  const int L = g.nl;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double m[32][3];
    gather_hits(g, lay, hits, n, i, mask[i], m);
    double sx[6], sC[36];
    if (!seed_from_hits_flag) {
      for (int k = 0; k < 6; ++k) sx[k] = (double)seed_state[(int64_t)k * n + i];
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) sC[a * 6 + b] = (double)seed_cov[(int64_t)tri(a, b) * n + i];
    }
    double xs[32][6], Cs[32][36];
    int lend;
    status[i] = smooth_track(g, lay, m, mask[i], seed_from_hits_flag != 0, sx, sC, xs, Cs, lend);
    lend_out[i] = lend;
    for (int l = 0; l < L; ++l) {
      const bool have = l <= lend;
      for (int k = 0; k < 6; ++k) xs_out[((int64_t)l * 6 + k) * n + i] = have ? xs[l][k] : 0.0;
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b <= a; ++b) Cs_out[((int64_t)l * 21 + tri(a, b)) * n + i] = have ? Cs[l][a * 6 + b] : 0.0;
    }
  }
}
}  // namespace

extern "C" {

// Batched smoother.  Inputs as oracle_fit.  Outputs in float64: xs [L][6][n],
// Cs [L][21][n] (packed lower triangle) for layers 0..lend[i] (zero elsewhere),
// lend [n] (last layer with an update, -1 if none), status [n] (the forward fit's).
void oracle_smooth(const OGeom* og, const double* align, const double* xX0, const OModel* model, int64_t n,
                   const float* hits, const uint32_t* mask, int seed_from_hits_flag, const float* seed_state,
                   const float* seed_cov, double* xs_out, double* Cs_out, int32_t* lend_out, uint32_t* status) {
  smooth_batch<float>(og, align, xX0, model, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, xs_out,
                      Cs_out, lend_out, status);
}

// As oracle_smooth with float64 hits and seeds.
void oracle_smooth_f64(const OGeom* og, const double* align, const double* xX0, const OModel* model, int64_t n,
                       const double* hits, const uint32_t* mask, int seed_from_hits_flag, const double* seed_state,
                       const double* seed_cov, double* xs_out, double* Cs_out, int32_t* lend_out,
                       uint32_t* status) {
  smooth_batch<double>(og, align, xX0, model, n, hits, mask, seed_from_hits_flag, seed_state, seed_cov, xs_out,
                       Cs_out, lend_out, status);
}

}  // extern "C"


// ==============================================================================
// Duplicate handling (Sec. 4.2): seed cleaning before building, duplicate removal
// after it.  The paper names the quantities (pT, eta and phi of the seeds or tracks,
// and shared hits) but gives no cuts.  Read here as a pairwise duplicate relation
// between two items of one event plus a priority order: an item is removed when an
// item of higher priority in its event is its duplicate.  The relation is not made
// transitive (an item that is itself removed still removes the ones below it), so the
// result does not depend on the order in which pairs are examined.  Every relation
// also requires |psi_i - psi_j| <= psi_window, psi the azimuth of the item's first
// hit, which bounds the search.  Written brute force: every pair of an event.
//
// A decision is flagged float-sensitive when one of its comparisons lies within a
// small margin of its cut and flipping that comparison alone would flip the decision.
// ==============================================================================

namespace {

struct Cmp {
  bool ok, near;
};

Cmp cmp_le(double a, double cut, double margin) { return {a <= cut, std::fabs(a - cut) <= margin}; }

// c[0] && ... && c[n-1], and whether one near comparison could flip it
Cmp all_of(const Cmp* c, int n) {
  Cmp r{true, false};
  int n_fail = 0;
  for (int k = 0; k < n; ++k) n_fail += !c[k].ok;
  r.ok = n_fail == 0;
  for (int k = 0; k < n; ++k)
    if (c[k].near && (n_fail == 0 || (n_fail == 1 && !c[k].ok))) r.near = true;
  return r;
}

struct SeedPar {
  double psi, z, kap, phi, theta;
  int32_t h[3];
  bool valid;
};

}  // namespace

extern "C" {

// Seed cleaning.  Seeds as for oracle_find (hit triplets on layers 0-2, global indices
// into hits [3][H]; seed_event [S]).  A seed's kinematics are the three-hit helix at
// its first hit (the fit's seed, on the placed hits).  Seeds i, j of one event are
// duplicates when |dpsi| <= psi_window and either they share >= min_shared hits, or
// they share >= min_shared_kin hits and |dkappa| <= kap_rel max|kappa| + kap_abs,
// |dtheta|, |dphi| and |dz| (z at the first hit) are within their cuts.  Priority:
// the lower index.  keep [S] = 1 / 0; sens [S] = 1 where a decision against a
// higher-priority seed is float-sensitive; invalid seeds (event or hit index out of
// range) are kept and take no part.
void oracle_clean_seeds(const OGeom* og, const double* align, const double* xX0, int32_t n_events, const float* hits,
                        int64_t H, const int64_t* hit_off, int64_t n_seeds, const int32_t* seed_event,
                        const int32_t* seed_hits, double psi_window, int32_t min_shared, int32_t min_shared_kin,
                        double kap_rel, double kap_abs, double theta_cut, double phi_cut, double z_cut, int32_t* keep,
                        uint8_t* sens) {
  Geo g = make_geo(og);
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  std::vector<SeedPar> P(n_seeds);
  std::vector<std::vector<int64_t>> by_event(n_events > 0 ? n_events : 0);
  for (int64_t i = 0; i < n_seeds; ++i) {
    SeedPar& p = P[i];
    keep[i] = 1;
    sens[i] = 0;
    p.valid = seed_event[i] >= 0 && seed_event[i] < n_events;
    double m[3][3];
    for (int l = 0; l < 3 && p.valid; ++l) {
      const int32_t j = seed_hits[(int64_t)l * n_seeds + i];
      p.h[l] = j;
      const int64_t* off = hit_off + (int64_t)seed_event[i] * (g.nl + 1);
      if (j < 0 || j >= H || j < off[l] || j >= off[l + 1]) {
        p.valid = false;
        break;
      }
      place_hit(lay[l], (double)hits[j], (double)hits[H + j], (double)hits[2 * H + j], m[l]);
    }
    if (!p.valid) continue;
    Track<double> tk;
    seed_from_hits(g, m[0], m[1], m[2], tk);
    p.psi = std::atan2(m[0][1], m[0][0]);
    p.z = tk.x[2];
    p.kap = tk.x[3];
    p.phi = tk.x[4];
    p.theta = tk.x[5];
    by_event[seed_event[i]].push_back(i);
  }
#pragma omp parallel for schedule(dynamic)
  for (int64_t e = 0; e < (int64_t)by_event.size(); ++e) {
    const std::vector<int64_t>& ev = by_event[e];
    for (size_t a = 0; a < ev.size(); ++a) {
      const int64_t i = ev[a];
      const SeedPar& pi = P[i];
      for (size_t b = 0; b < a; ++b) {  // j < i: higher priority
        const int64_t j = ev[b];
        const SeedPar& pj = P[j];
        const Cmp w = cmp_le(std::fabs(wrap_pi(pi.psi - pj.psi)), psi_window, 1e-5);
        int shared = 0;
        for (int l = 0; l < 3; ++l) shared += pi.h[l] == pj.h[l];
        Cmp d{shared >= min_shared, false};
        if (!d.ok && shared >= min_shared_kin) {
          const double kcut = kap_rel * std::max(std::fabs(pi.kap), std::fabs(pj.kap)) + kap_abs;
          const Cmp c[4] = {cmp_le(std::fabs(pi.kap - pj.kap), kcut, 1e-3 * kcut),
                            cmp_le(std::fabs(pi.theta - pj.theta), theta_cut, 1e-5),
                            cmp_le(std::fabs(wrap_pi(pi.phi - pj.phi)), phi_cut, 1e-5),
                            cmp_le(std::fabs(pi.z - pj.z), z_cut, 1e-4)};
          d = all_of(c, 4);
        }
        const Cmp both[2] = {w, d};
        const Cmp r = all_of(both, 2);
        if (r.near) sens[i] = 1;
        if (r.ok) keep[i] = 0;
      }
    }
  }
}

// Duplicate removal over built tracks (for instance each seed's best finder candidate).
// Item i: event [i], hits hit_idx [L][n] (global index, < 0 none), n_hits [i], chi2 [i],
// kappa = state[3][i], theta = state[5][i] (state [6][n]).  psi: azimuth of the placed
// hit on the item's lowest layer with a hit.  i, j are duplicates when |dpsi| <=
// psi_window, they share at least shared_frac * min(n_hits) hits (the same hit on the
// same layer) and |dkappa| <= kap_rel max|kappa| + kap_abs and |dtheta| <= theta_cut.
// Priority: more hits, then lower chi2, then the lower index.  Items without hits are
// kept and remove nothing.
void oracle_remove_duplicates(const OGeom* og, const double* align, const double* xX0, int32_t n_events,
                              const float* hits, int64_t H, int64_t n, const int32_t* event, const int32_t* hit_idx,
                              const int32_t* n_hits, const float* chi2, const float* state, double psi_window,
                              double shared_frac, double kap_rel, double kap_abs, double theta_cut, int32_t* keep,
                              uint8_t* sens) {
  Geo g = make_geo(og);
  Layer<double> lay[32];
  make_layers<double>(g, align, xX0, lay);
  const int L = g.nl;
  std::vector<double> psi(n, 0.0);
  std::vector<std::vector<int64_t>> by_event(n_events > 0 ? n_events : 0);
  for (int64_t i = 0; i < n; ++i) {
    keep[i] = 1;
    sens[i] = 0;
    if (event[i] < 0 || event[i] >= n_events || n_hits[i] <= 0) continue;
    int first = -1;
    for (int l = 0; l < L && first < 0; ++l) {
      const int32_t j = hit_idx[(int64_t)l * n + i];
      if (j >= 0 && j < H) first = l;
    }
    if (first < 0) continue;
    const int32_t j = hit_idx[(int64_t)first * n + i];
    double m[3];
    place_hit(lay[first], (double)hits[j], (double)hits[H + j], (double)hits[2 * H + j], m);
    psi[i] = std::atan2(m[1], m[0]);
    by_event[event[i]].push_back(i);
  }
  auto higher = [&](int64_t j, int64_t i) {  // priority of j above i
    if (n_hits[j] != n_hits[i]) return n_hits[j] > n_hits[i];
    if (chi2[j] != chi2[i]) return chi2[j] < chi2[i];
    return j < i;
  };
#pragma omp parallel for schedule(dynamic)
  for (int64_t e = 0; e < (int64_t)by_event.size(); ++e)
    for (int64_t i : by_event[e])
      for (int64_t j : by_event[e]) {
        if (j == i || !higher(j, i)) continue;
        int shared = 0;
        for (int l = 0; l < L; ++l) {
          const int32_t a = hit_idx[(int64_t)l * n + i];
          shared += a >= 0 && a == hit_idx[(int64_t)l * n + j];
        }
        const double need = shared_frac * std::min(n_hits[i], n_hits[j]);
        const double ki = state[3 * n + i], kj = state[3 * n + j];
        const double kcut = kap_rel * std::max(std::fabs(ki), std::fabs(kj)) + kap_abs;
        const Cmp c[4] = {cmp_le(std::fabs(wrap_pi(psi[i] - psi[j])), psi_window, 1e-5),
                          {shared >= need, std::fabs(shared - need) < 1e-5},
                          cmp_le(std::fabs(ki - kj), kcut, 1e-5 * kcut),
                          cmp_le(std::fabs((double)state[5 * n + i] - (double)state[5 * n + j]), theta_cut, 1e-6)};
        const Cmp r = all_of(c, 4);
        if (r.near) sens[i] = 1;
        if (r.ok) keep[i] = 0;
      }
}

}  // extern "C"
