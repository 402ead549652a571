// Per-particle decode and per-sub-pixel forward / adjoint math of the lens model.
//
// Forward model (Gu et al. 2022, Sec. 2.1.1): deflection by an elliptical power law (EPL,
// deflection through the Gauss hypergeometric series of Tessore & Metcalf 2015) or its
// slope-2 case the SIE (closed form), plus external shear; ray trace beta = x - alpha;
// elliptical Sersic source plus Cartesian shapelets at beta; elliptical Sersic lens light
// at x.
//
// Everything is written in complex image-plane variables that are smooth in the
// eccentricities (eps1, eps2), so the gradient has no 0/0 at a round lens:
//   z = (x - x_c) + i (y - y_c),  eps = eps1 + i eps2,  w = z - eps conj(z),
//   B = theta_E sqrt(1 - |eps|^2),  X = conj(eps) w^2 / |w|^2,
//   alpha = B^t |w|^-t w S_t(X),  S_t(X) = sum_n c_n(t) (-X)^n,
//   c_0 = 1,  c_n = c_{n-1} (2n - 2 + t) / (2n + 2 - t),  t = gamma_epl - 1.
// This is the paper's (q, phi) form rewritten: with q = (1-|eps|)/(1+|eps|),
// q x_l + i y_l = ((1+q)/2) e^{-i phi} w, the elliptical radius R = |w| / (1 + |eps|), the
// prefactor 2b/(1+q) (b/R)^(t-1) = B^t |w|^(1-t) and (1-q)/(1+q) e^{-2i phi} = conj(eps).
// For t = 1 the series sums to S_1(X) = atan(sqrt X) / sqrt X, the SIE closed form.
//
// Precision: sub-pixel positions, the deflection and the ray trace run in FP64 (on CDNA4 a
// double FMA issues at the rate of an unpacked float FMA), so the source offset
// beta - x_s keeps full FP32 relative precision even where the source has a cusp; the light
// profiles and all derivative terms run in FP32 on offsets from their centres.
//
// Sersic light uses the rotation-free quadratic form of the elliptical radius,
//   q x_l^2 + y_l^2 / q = [(1+|e|^2-2e1) dx^2 - 4 e2 dx dy + (1+|e|^2+2e1) dy^2] / (1-|e|^2),
// which is the same quantity without the position angle.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "glens_types.h"

#define GL_HD __host__ __device__ __forceinline__

namespace glens {

constexpr float kInvSqrtPi = 0.56418958354775628f;

// System of a Group that owns block b of a grouped launch.
__device__ __forceinline__ int find_sys(const Group& g, int b) {
  int i = 0;
  while (i + 1 < g.nsys && b >= g.block0[i + 1]) ++i;
  return i;
}

// ------------------------------------------------------------------------------------------
// Per-particle decode (prologue). Double precision: it runs once per particle.
// ------------------------------------------------------------------------------------------

// Rescale |eps| onto eps_max when above it; returns the clamp Jacobian (symmetric).
GL_HD void clamp_eps(double e1, double e2, double emax, double& c1, double& c2, double& j11,
                     double& j12, double& j22) {
  const double r = sqrt(e1 * e1 + e2 * e2);
  if (r > emax) {
    const double s = emax / r, u1 = e1 / r, u2 = e2 / r;
    c1 = e1 * s;
    c2 = e2 * s;
    j11 = s * (1.0 - u1 * u1);
    j12 = -s * u1 * u2;
    j22 = s * (1.0 - u2 * u2);
  } else {
    c1 = e1;
    c2 = e2;
    j11 = 1.0;
    j12 = 0.0;
    j22 = 1.0;
  }
}

// r_n = sqrt(2^n / n!) for n = 0 .. kMaxNmax; r_n1 r_n2 scales coefficient (n1, n2).
constexpr double kHermR[kMaxNmax + 1] = {
    1.0, 1.4142135623730951, 1.4142135623730951, 1.1547005383792515, 0.816496580927726,
    0.5163977794943222, 0.29814239699997197, 0.15936381457791915, 0.07968190728895957};
GL_HD inline double hermite_scale(int n1, int n2) { return kHermR[n1] * kHermR[n2]; }

GL_HD void decode_light(const float* th, LightC& L) {
  const double re = th[0], n = th[1];
  double e1, e2, j11, j12, j22;
  clamp_eps(th[2], th[3], kLightEpsMax, e1, e2, j11, j12, j22);
  const double ee = e1 * e1 + e2 * e2, den = 1.0 / (1.0 - ee);
  L.i0 = th[6];
  L.qa = float((1.0 + ee - 2.0 * e1) * den);
  L.qb = float(-4.0 * e2 * den);
  L.qc = float((1.0 + ee + 2.0 * e1) * den);
  L.qbh = float(-2.0 * e2 * den);
  L.kq = float(-(1.9992 * n - 0.3271) / n);
  L.inv2n = float(0.5 / n);
  L.l2re_n = float(log2(re) / n);
  L.bn = float(1.9992 * n - 0.3271);
  L.bnl = float((1.9992 * n - 0.3271) * 1.4426950408889634);
  L.n = float(n);
  L.re = float(re);
  L.e1 = float(e1);
  L.e2 = float(e2);
  L.inv1me2 = float(den);
  L.j11 = float(j11);
  L.j12 = float(j12);
  L.j22 = float(j22);
}

// Number of parameters of the mass model (lens mass + external shear) in the gl.h layout.
GL_HD int mass_param_count(int mass, int shear) { return 5 + (mass == 1) + 2 * shear; }

// Mass constants of one parameter vector (layout of gl.h): everything but the series
// coefficients, whose term counts it sets.
GL_HD void decode_mass(const float* th, int mass, int shear, PConst& c) {
  int p = 0;
  const double theta_e = th[p++];
  const double t = (mass == 1) ? double(th[p++]) - 1.0 : 1.0;
  double e1, e2, j11, j12, j22;
  clamp_eps(th[p], th[p + 1], kMassEpsMax, e1, e2, j11, j12, j22);
  p += 2;
  c.xc = th[p++];
  c.yc = th[p++];
  if (shear) {
    c.g1 = th[p++];
    c.g2 = th[p++];
  } else {
    c.g1 = 0.0;
    c.g2 = 0.0;
  }
  const double ee = e1 * e1 + e2 * e2, eabs = sqrt(ee);
  const double B = theta_e * sqrt(1.0 - ee);
  c.t = t;
  c.e1 = e1;
  c.e2 = e2;
  c.tlnb = t * log(B);
  c.bmass = B;
  c.w2floor = 1e-12 * (1.0 + eabs) * (1.0 + eabs);
  c.epsabs = eabs;
  c.theta_e = float(theta_e);
  c.tf = float(t);
  c.hp = float(1.0 - 0.5 * t);
  c.hm = float(-0.5 * t);
  c.e1f = float(e1);
  c.e2f = float(e2);
  c.lnb = float(log(B));
  c.xcf = float(c.xc);
  c.ycf = float(c.yc);
  c.w2floorf = float(c.w2floor);
  c.tlnb2 = float(c.tlnb * 1.4426950408889634);
  c.tfac = float(t / (2.0 * (1.0 - ee)));
  c.mj11 = float(j11);
  c.mj12 = float(j12);
  c.mj22 = float(j22);
  // series: terms until the tail bound |eps|^N / (1 - |eps|) drops below the tolerance
  // (FP64 value series), and below the looser derivative tolerance (adjoint series)
  int nt = 1, ntd = 1;
  if (eabs > 1e-30) {
    nt = int(ceil(log(kSeriesTol * (1.0 - eabs)) / log(eabs)));
    nt = nt < 1 ? 1 : (nt > kMaxTerms ? kMaxTerms : nt);
    ntd = int(ceil(log(kSeriesTolDeriv * (1.0 - eabs)) / log(eabs))) + 1;
    ntd = ntd < 1 ? 1 : (ntd > nt ? nt : ntd);
  }
  c.nterms = nt;
  c.nterms_d = ntd;
  // SIE closed form: s = sqrt(conj(eps)), S_1(X) = atan(s u) / (s u), u = w / |w|
  c.sie_closed = (mass == 0 && eabs >= kSieClosedMin) ? 1 : 0;
  if (c.sie_closed) {
    const double ang = -0.5 * atan2(e2, e1), rs = sqrt(eabs);
    c.sr = rs * cos(ang);
    c.si = rs * sin(ang);
  } else {
    c.sr = c.si = 0.0;
  }
  c.iebr = eabs >= kSxClosedMin ? float(e1 / ee) : 0.f;
  c.iebi = eabs >= kSxClosedMin ? float(e2 / ee) : 0.f;
}

// Series ratio c_n / c_{n-1} = (2n - 2 + t) / (2n + 2 - t) and the increment of
// d log c_n / dt, 1 / (2n - 2 + t) + 1 / (2n + 2 - t), for n >= 1.
GL_HD void series_step(int n, double t, double& ratio, double& dlog) {
  const double a = 2.0 * n - 2.0 + t, b = 2.0 * n + 2.0 - t;
  ratio = a / b;
  dlog = 1.0 / a + 1.0 / b;
}

// Stores term n of the value series (c_n), of the derivative series n c_n (at n - 1) and
// of dc_n / dt = c_n sum_k dlog_k, given the running product and sum.
GL_HD void series_store(PConst& c, int n, double cn, double dsum) {
  c.c[n] = n < c.nterms ? cn : 0.0;
  c.dc[n] = n < c.nterms_d ? float(cn * dsum) : 0.f;
  if (n > 0) c.nc[n - 1] = n < c.nterms_d ? float(n * cn) : 0.f;
  if (n == kMaxTerms - 1) c.nc[kMaxTerms - 1] = 0.f;
}

// ------------------------------------------------------------------------------------------
// The floored sub-pixel. The elliptical mass radius R is kept >= 1e-6 arcsec (R^2 >= 1e-12);
// below that the deflection is the formula with R frozen at 1e-6, a function of the remaining
// variables whose derivatives the per-lane FP32 adjoint does not carry (the frozen radius on
// |w| is 1e-12 (1 + |eps|)^2, which depends on eps, and the SIE's closed form with a frozen
// radius is not its series with one). The prologue finds that sub-pixel (at most one per
// particle) and evaluates the frozen-radius deflection and its derivatives exactly, by
// forward-mode dual numbers in FP64 over (t, eps1, eps2, x_c, y_c).
// ------------------------------------------------------------------------------------------
struct D5 {
  double v;
  double d[5];
};
GL_HD D5 d5(double v, int k = -1) {
  D5 r;
  r.v = v;
#pragma unroll
  for (int i = 0; i < 5; ++i) r.d[i] = i == k ? 1.0 : 0.0;
  return r;
}
GL_HD D5 operator+(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v + b.v;
  for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
GL_HD D5 operator-(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v - b.v;
  for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
GL_HD D5 operator*(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v * b.v;
  for (int i = 0; i < 5; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
GL_HD D5 operator*(double s, const D5& a) {
  D5 r;
  r.v = s * a.v;
  for (int i = 0; i < 5; ++i) r.d[i] = s * a.d[i];
  return r;
}
GL_HD D5 operator/(const D5& a, const D5& b) {
  D5 r;
  r.v = a.v / b.v;
  for (int i = 0; i < 5; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r;
}
// f(a) given f(a.v) and f'(a.v)
GL_HD D5 d5_chain(const D5& a, double f, double df) {
  D5 r;
  r.v = f;
  for (int i = 0; i < 5; ++i) r.d[i] = df * a.d[i];
  return r;
}
GL_HD D5 d5_exp(const D5& a) { const double e = exp(a.v); return d5_chain(a, e, e); }
GL_HD D5 d5_log(const D5& a) { return d5_chain(a, log(a.v), 1.0 / a.v); }
GL_HD D5 d5_sqrt(const D5& a) { const double r = sqrt(a.v); return d5_chain(a, r, 0.5 / r); }
GL_HD D5 d5_atan(const D5& a) { return d5_chain(a, atan(a.v), 1.0 / (1.0 + a.v * a.v)); }
GL_HD D5 d5_atanh(const D5& a) { return d5_chain(a, atanh(a.v), 1.0 / (1.0 - a.v * a.v)); }
GL_HD D5 d5_cos(const D5& a) { return d5_chain(a, cos(a.v), -sin(a.v)); }
GL_HD D5 d5_sin(const D5& a) { return d5_chain(a, sin(a.v), cos(a.v)); }
GL_HD D5 d5_atan2(const D5& y, const D5& x) {
  D5 r;
  r.v = atan2(y.v, x.v);
  const double n = x.v * x.v + y.v * y.v;
  for (int i = 0; i < 5; ++i) r.d[i] = (x.v * y.d[i] - y.v * x.d[i]) / n;
  return r;
}

// Centre of sub-pixel column (or row) n of the system's grid: x0 + n dxs, one rounding.
GL_HD double subpix_coord(double x0, int n, double dxs) { return fma(double(n), dxs, x0); }

// Deflection at image position (x, y) with the elliptical radius frozen at its floor
// R_f = 1e-6 arcsec, as dual numbers over (t, eps1, eps2, x_c, y_c).
//   EPL (and the SIE's series): alpha = A w S_t(X) with A = (theta_E sqrt(q) / R_f)^t,
//     q = (1 - |eps|)/(1 + |eps|), w = z - eps conj(z), X = conj(eps) w^2 / |w_f|^2,
//     |w_f| = R_f (1 + |eps|): the series form in which |w| only enters through R;
//   SIE: the closed form with the radius frozen, in the lens frame (rotation by
//     phi = atan2(eps2, eps1) / 2): alpha_l = b / q' (atan(q' x_l / R_f), atanh(q' y_l / R_f)),
//     b = theta_E sqrt(q), q' = sqrt(1 - q^2); at |eps| = 0 the SIS limit b z / R_f.
// |eps| has no derivative at eps = 0: there the eps-derivatives of |eps| are taken as 0.
GL_HD void floored_deflection(const PConst& c, int mass, double x, double y, D5& ar, D5& ai) {
  const double rf = 1e-6;
  const D5 e1 = d5(c.e1, 1), e2 = d5(c.e2, 2);
  const D5 zr = d5(x) - d5(c.xc, 3), zi = d5(y) - d5(c.yc, 4);
  const D5 ee = e1 * e1 + e2 * e2;
  const D5 ea = ee.v > 0.0 ? d5_sqrt(ee) : d5(0.0);
  const D5 one = d5(1.0);
  const D5 q = (one - ea) / (one + ea);
  const double the = double(c.theta_e);
  if (mass == 1) {
    const D5 t = d5(c.t, 0);
    const D5 A = d5_exp(t * (d5(log(the / rf)) + 0.5 * d5_log(q)));
    const D5 wr = zr - e1 * zr - e2 * zi, wi = zi - e2 * zr + e1 * zi;
    const D5 wf2 = (rf * rf) * ((one + ea) * (one + ea));
    const D5 w2r = wr * wr - wi * wi, w2i = 2.0 * (wr * wi);
    const D5 Xr = (e1 * w2r + e2 * w2i) / wf2, Xi = (e1 * w2i - e2 * w2r) / wf2;
    D5 Sr = one, Si = d5(0.0), cn = one, pr = one, pi = d5(0.0);
    for (int n = 1; n < c.nterms; ++n) {
      cn = cn * (d5(2.0 * n - 2.0) + t) / (d5(2.0 * n + 2.0) - t);
      const D5 nr = d5(0.0) - (pr * Xr - pi * Xi), ni = d5(0.0) - (pr * Xi + pi * Xr);
      pr = nr;
      pi = ni;
      Sr = Sr + cn * pr;
      Si = Si + cn * pi;
    }
    ar = A * (wr * Sr - wi * Si);
    ai = A * (wr * Si + wi * Sr);
    return;
  }
  const D5 b = the * d5_sqrt(q);
  if (ea.v == 0.0) {  // circular: the SIS with its radius frozen
    ar = (1.0 / rf) * (b * zr);
    ai = (1.0 / rf) * (b * zi);
    return;
  }
  const D5 phi = 0.5 * d5_atan2(e2, e1);
  const D5 cp = d5_cos(phi), sp = d5_sin(phi);
  const D5 xl = cp * zr + sp * zi, yl = sp * (d5(0.0) - zr) + cp * zi;
  const D5 qp = d5_sqrt(one - q * q);
  const D5 axl = b / qp * d5_atan((1.0 / rf) * (qp * xl));
  const D5 ayl = b / qp * d5_atanh((1.0 / rf) * (qp * yl));
  ar = cp * axl - sp * ayl;
  ai = sp * axl + cp * ayl;
}

// Finds the floored sub-pixel of one particle (fills c.fl_*; after decode_mass). Only the
// sub-pixel nearest the lens centre can have R below the floor.
GL_HD void decode_floor(const SysDesc& s, PConst& c) {
  c.fl_i = c.fl_j = -1;
  c.fl_a[0] = c.fl_a[1] = 0.0;
  const double fj = rint((c.xc - s.x0) / s.dxs), fi = rint((c.yc - s.y0) / s.dxs);
  if (!(fj >= 0.0 && fj < double(s.W * s.k) && fi >= 0.0 && fi < double(s.H * s.k))) return;
  const int jj = int(fj), ii = int(fi);
  const double x = subpix_coord(s.x0, jj, s.dxs), y = subpix_coord(s.y0, ii, s.dxs);
  const double zr = x - c.xc, zi = y - c.yc;
  const double wr = zr - c.e1 * zr - c.e2 * zi, wi = zi - c.e2 * zr + c.e1 * zi;
  if (!(wr * wr + wi * wi < c.w2floor)) return;
  D5 ar, ai;
  floored_deflection(c, s.mass, x, y, ar, ai);
  c.fl_i = ii;
  c.fl_j = jj;
  c.fl_a[0] = ar.v;
  c.fl_a[1] = ai.v;
  for (int k = 0; k < 5; ++k) {
    c.fl_d[k][0] = ar.d[k];
    c.fl_d[k][1] = ai.d[k];
  }
}

// Orders (n1, n2) of shapelet coefficient q: q runs over n = n1 + n2 = 0, 1, ... and, within
// one n, over n2 = 0 .. n.
GL_HD void shapelet_orders(int q, int& n1, int& n2) {
  int n = 0;
  while ((n + 1) * (n + 2) / 2 <= q) ++n;
  n2 = q - n * (n + 1) / 2;
  n1 = n - n2;
}

// Light constants (lens light, source Sersic, shapelet coefficients) of one vector, spread
// over the lanes of the prologue: lane 1 the lens light, lane 2 the source, lane 3 the
// shapelet scale, lanes 3 .. 3 + M - 1 one shapelet coefficient each (M = (n_max + 1)
// (n_max + 2) / 2 <= 45). Every field is written by exactly one lane.
GL_HD void decode_lights_lane(const float* th, int mass, int shear, int lens_light, int nmax,
                              PConst& c, int lane) {
  const int pl = mass_param_count(mass, shear);        // lens light
  const int ps = pl + (lens_light ? 7 : 0);            // source Sersic
  const int pb = ps + 7;                               // shapelet scale, then coefficients
  if (lane == 1) {
    c.lxs = c.lys = 0.0;
    if (lens_light) {
      decode_light(th + pl, c.lens);
      c.lxs = th[pl + 4];
      c.lys = th[pl + 5];
    }
  } else if (lane == 2) {
    decode_light(th + ps, c.src);
    c.sxs = th[ps + 4];
    c.sys = th[ps + 5];
  }
  if (nmax < 0) return;
  const int q = lane - 3, M = (nmax + 1) * (nmax + 2) / 2;
  if (q < 0 || q >= M) return;
  const double beta = th[pb];
  if (q == 0) {
    c.beta = float(beta);
    c.inv_beta = float(1.0 / beta);
  }
  const double f = 0.56418958354775628 / beta;  // 1 / (beta sqrt(pi))
  int n1, n2;
  shapelet_orders(q, n1, n2);
  c.shp[q] = float(double(th[pb + 1 + q]) * (f * hermite_scale(n1, n2)));
}

// ------------------------------------------------------------------------------------------
// Double-precision helpers for the ray trace, for the argument ranges met there (normal,
// finite, positive arguments). Written from the mathematics:
//   rcp: hardware estimate (relative error about 2^-23) refined by one Newton step
//        r <- r + r (1 - x r), which squares the error (about 1e-14);
//   the power B^t |w|^-t: per-particle tables (pow_from_table, after these helpers).
// The targets sit below the 1e-10 relative tolerance of the deflection series: the ray
// trace needs |alpha| to ~1e-9 arcsec, far below FP32 resolution but far above FP64's.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double rcp_f64(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(fma(-x, r, 1.0), r, r);
}
__host__ inline double rcp_f64(double x) { return 1.0 / x; }

// Single-precision hardware transcendentals in base 2 (about 1 ulp), for normal, finite
// arguments; callers fold log2(e) into their per-particle constants.
__device__ __forceinline__ float exp2_f32(float x) { return __builtin_amdgcn_exp2f(x); }
__host__ inline float exp2_f32(float x) { return exp2f(x); }
__device__ __forceinline__ float log2_f32(float x) { return __builtin_amdgcn_logf(x); }
__host__ inline float log2_f32(float x) { return log2f(x); }
__device__ __forceinline__ float rcp_f32(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ inline float rcp_f32(float x) { return 1.0f / x; }
constexpr float kLn2f = 0.69314718055994531f;
constexpr float kLog2e = 1.44269504088896341f;

constexpr double kLn2 = 0.6931471805599453;  // nearest double to ln 2

// Entries of the power tables (PConst::pw) at table index i: i < kPowExp gives B^t 2^(-t e/2)
// for e = i - kPowExp/2; i = kPowExp + 8 j + k the Taylor coefficient k of m^(-t/2) about
// m_j = 1 + (j + 1/2)/16: a_0 = m_j^(-t/2), a_k = a_(k-1) (-t/2 - k + 1) / (k m_j).
GL_HD double pow_table_entry(double t, double log2B, int i) {
  if (i < kPowExp) return exp2(t * (log2B - 0.5 * (i - kPowExp / 2)));
  const int j = (i - kPowExp) / 8, k = (i - kPowExp) % 8;
  if (k > kPowDeg) return 0.0;
  const double mj = 1.0 + (j + 0.5) / kPowSeg;
  double a = exp2(-0.5 * t * log2(mj));
  for (int q = 1; q <= k; ++q) a *= (-0.5 * t - (q - 1)) / (q * mj);
  return a;
}

// The power tables shared by `nl` lanes (this one is lane l of them): the exponent entries
// round-robin, and the sixteen segments' Taylor coefficients one segment per lane on the last
// kPowSeg lanes (each segment's coefficients by the recursion of pow_table_entry, the same
// operations in the same order).
GL_HD void pow_tables_lane(double t, double log2B, int l, int nl, double* pw) {
  for (int i = l; i < kPowExp; i += nl) pw[i] = pow_table_entry(t, log2B, i);
  const int j = l - (nl - kPowSeg);
  if (j < 0) return;
  double* seg = pw + kPowExp + 8 * j;
  const double mj = 1.0 + (j + 0.5) / kPowSeg;
  double a = exp2(-0.5 * t * log2(mj));
  seg[0] = a;
  for (int q = 1; q < 8; ++q) {
    if (q <= kPowDeg) a *= (-0.5 * t - (q - 1)) / (q * mj);
    seg[q] = q <= kPowDeg ? a : 0.0;
  }
}

// A = B^t |w|^-t = B^t (|w|^2)^(-t/2) from the particle's power tables (staged in LDS): with
// |w|^2 = 2^e m, m in [1, 2), the four leading mantissa bits pick the sixteenth j of [1, 2)
// and the remaining ones give x = m - m_j exactly, so that A = T[e] P_j(x) (about 3e-11
// relative; no logarithm or exponential). |w|^2 is at least the 1e-12 floor, so e >= -40; an
// exponent beyond the table (|w| above 2^31 arcsec) is clamped.
GL_HD double pow_from_table(const double* __restrict__ pw, double w2) {
  const uint64_t b = __builtin_bit_cast(uint64_t, w2);
  const int e = int((b >> 52) & 0x7ffu) - 1023;
  const int j = int((b >> 48) & 15u);
  const double m = __builtin_bit_cast(double, (b & 0x0000ffffffffffffull) | 0x3ff0000000000000ull);
  const double x = m - (1.0 + 0.5 / kPowSeg);
  const double* a = pw + kPowExp + 8 * j;
  double p = fma(a[6], x, a[5]);
  p = fma(p, x, a[4]);
  p = fma(p, x, a[3]);
  p = fma(p, x, a[2]);
  p = fma(p, x, a[1]);
  p = fma(p, x, a[0]);
  const int ie = e + kPowExp / 2;
  return pw[ie < 0 ? 0 : (ie >= kPowExp ? kPowExp - 1 : ie)] * p;
}

// ------------------------------------------------------------------------------------------
// Sub-pixel math
// ------------------------------------------------------------------------------------------

struct Cx {
  float r, i;
};
GL_HD Cx cmul(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
GL_HD Cx cadd(Cx a, Cx b) { return {a.r + b.r, a.i + b.i}; }
GL_HD Cx csub(Cx a, Cx b) { return {a.r - b.r, a.i - b.i}; }
GL_HD Cx cscale(Cx a, float s) { return {a.r * s, a.i * s}; }
GL_HD Cx cconj(Cx a) { return {a.r, -a.i}; }
GL_HD Cx cmuli(Cx a) { return {-a.i, a.r}; }  // i a
GL_HD float cdot(Cx g, Cx v) { return g.r * v.r + g.i * v.i; }  // real dot product

// The lens quantities of one sub-pixel that the adjoint uses (FP32).
struct MassState {
  float sdx, sdy;     // beta - x_s (source offset)
  Cx z, w, u2, X;     // z, w, w^2/|w|^2, X = conj(eps) u2
  float lnw2;         // ln |w|^2 (floored)
  float A;            // B^t |w|^-t
  Cx S, XSX, U2SX, St;  // S_t(X), X dS/dX, u2 dS/dX, dS/dt
  Cx alpha;
};

// EPL / SIE deflection plus shear at image position (x, y), in FP64: returns beta - x_s with
// beta = x - alpha - alpha_ext. cs: the particle's series coefficients c.c (the kernels pass
// a copy staged in LDS).
// at_floor: this is the particle's floored sub-pixel (c.fl_*); the SIE then takes the
// frozen-radius closed form the prologue evaluated (the EPL's value there is this formula's).
// cs / pw: the particle's series coefficients c.c and power tables c.pw (staged in LDS).
template <int MASS>
GL_HD void ray_trace(const PConst& c, const double* __restrict__ cs,
                     const double* __restrict__ pw, double x, double y, bool at_floor,
                     float& sdx, float& sdy) {
  const double zr = x - c.xc, zi = y - c.yc;
  const double e1 = c.e1, e2 = c.e2;
  const double wr = zr - e1 * zr - e2 * zi, wi = zi - e2 * zr + e1 * zi;
  const double w2 = fmax(wr * wr + wi * wi, c.w2floor);
  const double inv_w2 = rcp_f64(w2);
  const double u2r = (wr * wr - wi * wi) * inv_w2, u2i = 2.0 * wr * wi * inv_w2;
  const double Xr = e1 * u2r + e2 * u2i, Xi = e1 * u2i - e2 * u2r;
  double Sr, Si, A;
  if (MASS == 0 && c.sie_closed) {
    // S_1(X) = atan(zeta) / zeta, zeta = s w / |w|; atan of |zeta| < 1 in closed form
    const double rinv = sqrt(inv_w2);
    const double ur = wr * rinv, ui = wi * rinv;
    const double a = c.sr * ur - c.si * ui, b = c.sr * ui + c.si * ur;
    const double aa = a * a;
    const double atr = 0.5 * atan(2.0 * a / (1.0 - c.epsabs));
    const double ati = 0.25 * log(((1.0 + b) * (1.0 + b) + aa) / ((1.0 - b) * (1.0 - b) + aa));
    const double ie = 1.0 / c.epsabs;  // S = atan(zeta) conj(zeta) / |eps|
    Sr = (atr * a + ati * b) * ie;
    Si = (ati * a - atr * b) * ie;
    A = c.bmass * rinv;
  } else {
    // The coefficients are real, so the series is evaluated at the complex point y = -X by
    // synthetic division by the real quadratic (v - y)(v - conj y) = v^2 - 2 Re(y) v + |y|^2
    // (Knuth, TAOCP vol. 2, sec. 4.6.4): b_n = c_n + 2 Re(y) b_(n+1) - |y|^2 b_(n+2) from the
    // top down to n = 0, and the sum is b_0 - Re(y) b_1 + i Im(y) b_1. That is two real FMAs
    // per term where complex Horner takes four. |y| = |eps| < 1, so rounding errors made
    // early are damped as the recurrence runs down. Terms are taken two per trip (so that the
    // two carried values need no register moves); coefficients past the series length are
    // zero, so rounding the length up to an even number is exact.
    const double yr = -Xr, yi = -Xi;
    const double r2 = 2.0 * yr, yy = fma(yr, yr, yi * yi);
    double b1 = 0.0, b2 = 0.0;  // b_(n+1), b_(n+2)
    const int nt2 = (c.nterms + 1) & ~1;
    for (int n0 = nt2 - 2; n0 >= 0; n0 -= 2) {  // leaves b_n0 in b1 and b_(n0+1) in b2
      b2 = fma(r2, b1, fma(-yy, b2, cs[n0 + 1]));
      b1 = fma(r2, b2, fma(-yy, b1, cs[n0]));
    }
    Sr = fma(-yr, b2, b1);
    Si = yi * b2;
    A = pow_from_table(pw, w2);
  }
  double ar = A * (wr * Sr - wi * Si), ai = A * (wr * Si + wi * Sr);
  if (MASS == 0 && at_floor) {
    ar = c.fl_a[0];
    ai = c.fl_a[1];
  }
  // beta - x_s = x - alpha - alpha_ext - x_s
  sdx = float(x - ar - (c.g1 * x + c.g2 * y) - c.sxs);
  sdy = float(y - ai - (c.g2 * x - c.g1 * y) - c.sys);
}

// The lens quantities the adjoint needs, in FP32: z, w, u2, X, ln|w|^2, A, S, X dS/dX,
// u2 dS/dX, dS/dt, alpha. (sdx, sdy) is beta - x_s of the forward pass's FP64 ray trace (SysDesc::beta): the
// light profiles and their derivatives are evaluated there (an FP32 ray trace moves it by
// ~3e-7 arcsec, which shows at 2e-3 in the gradient of a vector far from the posterior). The
// rest only enters the Jacobian d(beta)/d(theta) and the local derivatives, whose tolerance
// (a relative 1e-3 on the gradient) is far above FP32 rounding:
//   alpha = x - alpha_ext - x_s - (beta - x_s), formed from the kept offset (FP64 up to the
//         last subtraction), and S = alpha / (A w), so the value series is not run again
//         (a sub-pixel whose |w|^2 hit the floor, where alpha carries no S, sums it);
//   dS/dX by the closed form of the identity below for |eps| >= kSxClosedMin (its numerator
//         cancels like |eps|, costing at most a relative 1e-6 / 0.02), by its series below;
//   dS/dt (EPL) by its series; the series run over the FP32-resolution length nterms_d;
//   log and exp are the hardware ones.
// |w|^2 is kept at or above the floor so that every quantity stays finite; the particle's
// floored sub-pixel itself (c.fl_*) takes its mass terms from the prologue's exact
// derivatives instead (the caller passes a zero weight here).
// ncs / dcs: the particle's c.nc / c.dc (staged in LDS). SXS = false: the caller has checked
// that |eps| >= kSxClosedMin, so dS/dX takes the closed form without a test.
template <int MASS, bool SXS = true>
__device__ __forceinline__ void mass_jacobian_f32(const PConst& c, const float* __restrict__ ncs,
                                                  const float* __restrict__ dcs, double x,
                                                  double y, float sdx, float sdy, MassState& m) {
  const float zr = float(x) - c.xcf, zi = float(y) - c.ycf;
  const float e1 = c.e1f, e2 = c.e2f;
  const float wr = zr - e1 * zr - e2 * zi, wi = zi - e2 * zr + e1 * zi;
  const float w2 = fmaxf(wr * wr + wi * wi, c.w2floorf);
  const float inv_w2 = rcp_f32(w2);
  const float u2r = (wr * wr - wi * wi) * inv_w2, u2i = 2.0f * wr * wi * inv_w2;
  const float Xr = e1 * u2r + e2 * u2i, Xi = e1 * u2i - e2 * u2r;
  const float l2w2 = log2_f32(w2);
  m.sdx = sdx;
  m.sdy = sdy;
  m.z = {zr, zi};
  m.w = {wr, wi};
  m.u2 = {u2r, u2i};
  m.X = {Xr, Xi};
  m.lnw2 = kLn2f * l2w2;
  // A = B^t |w|^-t = 2^(t log2 B - (t/2) log2 |w|^2) (SIE: t = 1)
  const float A = exp2_f32(fmaf(-0.5f * c.tf, l2w2, c.tlnb2));
  const float ar = float(x - (c.g1 * x + c.g2 * y) - c.sxs) - sdx;
  const float ai = float(y - (c.g2 * x - c.g1 * y) - c.sys) - sdy;
  // series by synthetic division at y = -X (ray_trace): dS/dt (EPL) and, for small |eps|,
  // dS/dy
  const float yr = -Xr, yi = -Xi, r2 = 2.0f * yr, yy = yr * yr + yi * yi;
  const bool sx_series = SXS && c.epsabs < kSxClosedMin;
  // four terms per trip, the length rounded up to a multiple of four (the padding
  // coefficients are zero): the LDS reads of a trip go out together, which at this kernel's
  // three waves per SIMD was measured faster than two terms per trip. dS/dt (EPL) here, dS/dy
  // (small |eps| only) below in a loop of its own, so that the common path carries no state
  // of the other.
  const int nd4 = (c.nterms_d + 3) & ~3;
  float t1 = 0.f, t2 = 0.f;
  if (MASS == 1) {
    for (int n0 = nd4 - 4; n0 >= 0; n0 -= 4) {
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        const float t0 = fmaf(r2, t1, fmaf(-yy, t2, dcs[n0 + q]));
        t2 = t1;
        t1 = t0;
      }
    }
  }
  // S = alpha conj(w) / (A |w|^2)
  const float r = rcp_f32(A * w2);
  const float Sr = (ar * wr + ai * wi) * r;
  const float Si = (ai * wr - ar * wi) * r;
  if (sx_series) {
    float d1 = 0.f, d2 = 0.f;
    for (int n0 = nd4 - 4; n0 >= 0; n0 -= 4) {
#pragma unroll
      for (int q = 3; q >= 0; --q) {
        const float d0 = fmaf(r2, d1, fmaf(-yy, d2, ncs[n0 + q]));
        d2 = d1;
        d1 = d0;
      }
    }
    const Cx SX = {-fmaf(-yr, d2, d1), -yi * d2};  // dS/dX = -dS/dy
    m.XSX = cmul(m.X, SX);
    m.U2SX = cmul(m.u2, SX);
  } else {
    // S = sum c_n (-X)^n with c_n / c_(n-1) = (2n - 2 + t) / (2n + 2 - t) obeys
    //   X (1 + X) dS/dX = (1 - t/2)(1 - S) - (t/2) X S
    // (as series: the coefficient of (-X)^n on both sides agrees for every n; for the SIE,
    // t = 1, it is S_X = (1/(1+X) - S) / (2X), which the closed form atan(zeta)/zeta obeys),
    // so X dS/dX is the right side over 1 + X, and u2 dS/dX = X dS/dX / conj(eps), as
    // X = conj(eps) u2. The numerator cancels like |X| = |eps|, so this is used for
    // |eps| >= kSxClosedMin only.
    const float xsr = Xr * Sr - Xi * Si, xsi = Xr * Si + Xi * Sr;
    const float numr = c.hp * (1.0f - Sr) + c.hm * xsr;
    const float numi = -c.hp * Si + c.hm * xsi;
    const float opr = 1.0f + Xr, inv = rcp_f32(opr * opr + Xi * Xi);
    m.XSX = {(numr * opr + numi * Xi) * inv, (numi * opr - numr * Xi) * inv};
    m.U2SX = cmul(m.XSX, Cx{c.iebr, c.iebi});
  }
  m.St = MASS == 1 ? Cx{fmaf(-yr, t2, t1), yi * t2} : Cx{0.f, 0.f};
  m.A = A;
  m.S = {Sr, Si};
  m.alpha = {ar, ai};
}

// Adds the mass-parameter terms g . d alpha/d(theta) to acc, with g = d s / d beta (already
// weighted by the pixel adjoint); beta = x - alpha - alpha_ext, so the signs are applied at
// the mapping. For a complex derivative D, g . D = Re(gb D) with gb = conj(g), and every
// derivative is contracted with gb as soon as it is formed:
//   with aw = d alpha/dw = A P1 and awb = d alpha/d conj(w) = A u2 P2 (eps fixed),
//   U = gb aw, V = gb awb;
//   d alpha/dz = aw - conj(eps) awb, d alpha/d conj(z) = awb - eps aw, and with x = z +
//   conj z, y = i (z - conj z):
//     g . d alpha/dx = Re((1 - eps) U + (1 - conj eps) V) = (1 - e1) Sp + e2 Dm,
//     g . d alpha/dy = -Im((1 + eps) U - (1 + conj eps) V) = -(1 + e1) Dm - e2 Sp,
//   Sp = Re U + Re V, Dm = Im U - Im V;
//   d alpha/d eps = -tfac conj(eps) alpha - conj(z) aw,
//   d alpha/d conj(eps) = -tfac eps alpha - z awb + A w u2 S_X (A depends on |eps|^2, X on
//   conj(eps)); with eps = e1 + i e2 and W = gb A w u2 S_X:
//     g . d alpha/de1 = -2 tfac e1 Re(gb alpha) - Re(z) Sp - Im(z) Dm + Re W,
//     g . d alpha/de2 = -2 tfac e2 Re(gb alpha) + Re(z) Dm - Im(z) Sp + Im W;
//   d alpha/dt = alpha (ln B - ln|w|^2 / 2) + A w S_t.
template <int MASS>
GL_HD void mass_adjoint(const PConst& c, const MassState& m, float x, float y, Cx g, float* acc) {
  const Cx XSX = m.XSX;
  const Cx P1 = cadd(cscale(m.S, c.hp), XSX);  // (1 - t/2) S + X S_X
  const Cx P2 = csub(cscale(m.S, c.hm), XSX);  // -(t/2) S - X S_X
  const Cx gA = {g.r * m.A, -g.i * m.A};  // A gb
  const Cx U = cmul(gA, P1);
  const Cx V = cmul(gA, cmul(m.u2, P2));
  const float Sp = U.r + V.r, Dm = U.i - V.i;
  const float e1 = c.e1f, e2 = c.e2f;
  const float ga = cdot(g, m.alpha);  // Re(gb alpha)
  const Cx gAw = cmul(gA, m.w);
  const Cx W = cmul(gAw, m.U2SX);
  acc[A_M_ALPHA] += ga;
  if (MASS == 1) {
    const float lt = fmaf(-0.5f, m.lnw2, c.lnb);  // ln B - ln|w|^2 / 2
    acc[A_M_T] += fmaf(lt, ga, gAw.r * m.St.r - gAw.i * m.St.i);
  }
  const float k = -2.0f * c.tfac;
  acc[A_M_E1] += fmaf(k * e1, ga, W.r - m.z.r * Sp - m.z.i * Dm);
  acc[A_M_E2] += fmaf(k * e2, ga, W.i + m.z.r * Dm - m.z.i * Sp);
  acc[A_M_X] += fmaf(1.0f - e1, Sp, e2 * Dm);
  acc[A_M_Y] -= fmaf(1.0f + e1, Dm, e2 * Sp);
  acc[A_M_G1] += g.r * x - g.i * y;
  acc[A_M_G2] += g.r * y + g.i * x;
}

// Elliptical Sersic intensity at offset (dx, dy) from its centre.
GL_HD float sersic_fwd(const LightC& L, float dx, float dy) {
  // R^2 = dx (qa dx + qb dy) + qc dy^2
  float q = fmaf(dx, fmaf(L.qb, dy, L.qa * dx), L.qc * dy * dy);
  q = q < kR2Floor ? kR2Floor : q;  // a select, not fmaxf: a NaN offset stays NaN
  // rho = (R / R_eff)^(1/n) = 2^(log2(R^2) / (2n) - log2(R_eff) / n);  I = I0 e^(b_n (1 - rho))
  const float rho = exp2_f32(fmaf(log2_f32(q), L.inv2n, -L.l2re_n));
  return L.i0 * exp2_f32(fmaf(-L.bnl, rho, L.bnl));
}

// Accumulator terms (weight sb) and the weighted sb dI/d(dx, dy). With the half gradient of
// R^2, (px, py) = (qa dx + qb dy / 2, qb dx / 2 + qc dy), R^2 = dx px + dy py and
// dR^2/d(dx, dy) = 2 (px, py); dI/dR^2 = -I b_n rho / (2 n R^2), so
// 2 sb dI/dR^2 = sb I rho (-b_n / n) / R^2 =: sIQ2 and sb dI/d(dx, dy) = sIQ2 (px, py).
// Slots: L_E: sb E; L_RHO: sb I rho; L_RHO1: sb I (rho - 1); L_RHOLN: sb I rho log2(rho)
// (ln 2 is applied at the mapping); L_Q1, L_Q2: the two eccentricity terms times
// 2 sb dI/dR^2 (the 1/2 is applied at the mapping).
GL_HD void sersic_adj(const LightC& L, float dx, float dy, float sb, float* acc, float& gdx,
                      float& gdy) {
  const float px = fmaf(L.qa, dx, L.qbh * dy), py = fmaf(L.qc, dy, L.qbh * dx);
  float q = fmaf(dx, px, dy * py);
  const bool fl = q < kR2Floor;
  q = fl ? kR2Floor : q;
  const float l2rho = fmaf(log2_f32(q), L.inv2n, -L.l2re_n);
  const float rho = exp2_f32(l2rho);
  const float sE = sb * exp2_f32(fmaf(-L.bnl, rho, L.bnl));
  const float sI = L.i0 * sE, sIr = sI * rho;
  const float sIQ2 = fl ? 0.0f : sIr * L.kq * rcp_f32(q);
  gdx = sIQ2 * px;
  gdy = sIQ2 * py;
  const float r2q = fmaf(dx, dx, fmaf(dy, dy, q));
  acc[L_E] += sE;
  acc[L_RHO] += sIr;
  acc[L_RHO1] += sIr - sI;
  acc[L_RHOLN] = fmaf(sIr, l2rho, acc[L_RHOLN]);
  acc[L_Q1] = fmaf(sIQ2, fmaf(L.e1, r2q, fmaf(dy, dy, -dx * dx)), acc[L_Q1]);
  acc[L_Q2] = fmaf(sIQ2, fmaf(L.e2, r2q, -2.0f * dx * dy), acc[L_Q2]);
}

// Scaled Hermite polynomials g_n(u) = H_n(u) / 2^n (H_n the physicists' polynomials):
// g_0 = 1, g_1 = u, g_(n+1) = u g_n - (n/2) g_(n-1), two operations per step, and
// g_n' = n g_(n-1). The Hermite functions are phi_n = (2^n n! sqrt(pi))^(-1/2) H_n e^(-u^2/2)
// = pi^(-1/4) r_n g_n e^(-u^2/2) with r_n = sqrt(2^n / n!); the coefficients carry r_n1 r_n2
// (hermite_scale) so that the sums run over the g_n directly.
// Started from h0 instead of 1 the recurrence gives h0 g_n(u) (it is linear).
template <int NMAX>
GL_HD void hermite(float u, float* h, float h0 = 1.0f) {
  h[0] = h0;
  if (NMAX >= 1) h[1] = h0 * u;
#pragma unroll
  for (int n = 1; n < NMAX; ++n) h[n + 1] = fmaf(u, h[n], -(0.5f * n) * h[n - 1]);
}

// Index of coefficient (n1, n2) in the order n = 0..NMAX, n1 = n..0, n2 = n - n1.
__host__ __device__ constexpr int shp_index(int n1, int n2) {
  return (n1 + n2) * (n1 + n2 + 1) / 2 + n2;
}

// Shapelet intensity at offset (sdx, sdy) from the source centre:
// G(u, v) sum_k c'_k g_n1(u) g_n2(v), c'_k = c_k r_n1 r_n2 / (beta sqrt(pi)),
// G = exp(-(u^2+v^2)/2), summed as U = sum_n1 g_n1(u) T_n1 with
// T_n1 = sum_n2 c'_(n1,n2) g_n2(v).
template <int NMAX>
GL_HD float shapelet_fwd(const PConst& c, float sdx, float sdy, const float* shp) {
  const float u = sdx * c.inv_beta, v = sdy * c.inv_beta;
  float hu[NMAX + 1], hv[NMAX + 1];
  hermite<NMAX>(u, hu);
  hermite<NMAX>(v, hv);
  // g_0 = 1: every sum starts from its n = 0 term (no addition of a zero, which the
  // compiler must keep for signed zeros)
  float U = 0.f;
#pragma unroll
  for (int n1 = 0; n1 <= NMAX; ++n1) {
    float T = shp[shp_index(n1, 0)];
#pragma unroll
    for (int n2 = 1; n2 <= NMAX - n1; ++n2) T = fmaf(shp[shp_index(n1, n2)], hv[n2], T);
    U = n1 == 0 ? T : fmaf(hu[n1], T, U);
  }
  return exp2_f32(-0.5f * kLog2e * (u * u + v * v)) * U;
}

// Shapelet accumulator terms and the weighted derivatives sb dI/d(beta_x, beta_y), using
// g_n' = n g_(n-1) for the scaled Hermite polynomials:
//   dI/du = G (sum_n1 n1 g_(n1-1)(u) T_n1 - u U),
//   dI/dv = G (sum_n1 g_n1(u) Tv_n1 - v U),  Tv_n1 = sum_n2 c'_(n1,n2) n2 g_(n2-1)(v),
//   dI/dc_k = G g_n1(u) g_n2(v) r_n1 r_n2 / (beta sqrt(pi)) (the factor r_n1 r_n2 /
//   (beta sqrt(pi)) is applied when the accumulators are mapped onto the gradient).
// The u-polynomials are taken times sg = sb G, so every sum over them carries the weight:
// U, Uu and Uv below are sb G times the sums above, and sb I = U.
template <int NMAX>
GL_HD void shapelet_adj(const PConst& c, float sdx, float sdy, const float* shp, float sb,
                        float* acc, float& gbx, float& gby) {
  const float ib = c.inv_beta;
  const float u = sdx * ib, v = sdy * ib;
  const float sg = sb * exp2_f32(-0.5f * kLog2e * (u * u + v * v));
  float hu[NMAX + 1], hv[NMAX + 1];
  hermite<NMAX>(u, hu, sg);
  hermite<NMAX>(v, hv);
  float U = 0.f, Uu = 0.f, Uv = 0.f;
#pragma unroll
  for (int n1 = 0; n1 <= NMAX; ++n1) {
    // g_0(v) = 1: T starts from its n2 = 0 term (no addition of a zero)
    float T = shp[shp_index(n1, 0)], Tv = 0.f;
#pragma unroll
    for (int n2 = 1; n2 <= NMAX - n1; ++n2) {
      const float ck = shp[shp_index(n1, n2)];
      T = fmaf(ck, hv[n2], T);
      Tv = n2 == 1 ? ck : fmaf(ck, float(n2) * hv[n2 - 1], Tv);
    }
    U = n1 == 0 ? hu[0] * T : fmaf(hu[n1], T, U);
    if (n1 < NMAX) Uv = n1 == 0 ? hu[0] * Tv : fmaf(hu[n1], Tv, Uv);
    if (n1 > 0) Uu = n1 == 1 ? hu[0] * T : fmaf(float(n1) * hu[n1 - 1], T, Uu);
  }
#pragma unroll
  for (int n1 = 0; n1 <= NMAX; ++n1)
#pragma unroll
    for (int n2 = 0; n2 <= NMAX - n1; ++n2)
      acc[A_SHP_C + shp_index(n1, n2)] = fmaf(hu[n1], hv[n2], acc[A_SHP_C + shp_index(n1, n2)]);
  const float Iu = Uu - u * U, Iv = Uv - v * U;  // sb dI/du, sb dI/dv
  acc[A_SHP_BETA] += (-U - u * Iu - v * Iv) * ib;
  gbx = Iu * ib;
  gby = Iv * ib;
}

// d(source Sersic + shapelets)/d(beta) at offset (sdx, sdy) from the source centre, in FP64
// (the floored sub-pixel's weight g of the mass terms, formed once per particle):
//   Sersic: dI/dR^2 = -I b_n rho / (2 n R^2), rho = (R / R_eff)^(1/n), dR^2 = 2 (px, py);
//   shapelets: as shapelet_adj, with g_n' = n g_(n-1).
GL_HD void source_light_grad(const PConst& c, int nmax, double sdx, double sdy, double& gx,
                             double& gy) {
  const LightC& L = c.src;
  const double px = L.qa * sdx + 0.5 * double(L.qb) * sdy;
  const double py = L.qc * sdy + 0.5 * double(L.qb) * sdx;
  const double r2 = sdx * px + sdy * py;
  gx = gy = 0.0;
  if (r2 >= kR2FloorD) {
    const double n = L.n, rho = exp(log(r2) / (2.0 * n) - log(double(L.re)) / n);
    const double I = double(L.i0) * exp(double(L.bn) * (1.0 - rho));
    const double dIdr2 = -I * double(L.bn) * rho / (2.0 * n * r2);
    gx = 2.0 * dIdr2 * px;
    gy = 2.0 * dIdr2 * py;
  }
  if (nmax < 0) return;
  const double ib = c.inv_beta, u = sdx * ib, v = sdy * ib;
  double hu[kMaxNmax + 1], hv[kMaxNmax + 1];
  hu[0] = hv[0] = 1.0;
  hu[1] = u;
  hv[1] = v;
  for (int k = 1; k < nmax; ++k) {
    hu[k + 1] = u * hu[k] - 0.5 * k * hu[k - 1];
    hv[k + 1] = v * hv[k] - 0.5 * k * hv[k - 1];
  }
  double U = 0.0, Uu = 0.0, Uv = 0.0;
  for (int n1 = 0; n1 <= nmax; ++n1)
    for (int n2 = 0; n1 + n2 <= nmax; ++n2) {
      const double ck = c.shp[shp_index(n1, n2)];
      U += ck * hu[n1] * hv[n2];
      if (n1 > 0) Uu += ck * n1 * hu[n1 - 1] * hv[n2];
      if (n2 > 0) Uv += ck * n2 * hu[n1] * hv[n2 - 1];
    }
  const double G = exp(-0.5 * (u * u + v * v));
  gx += G * (Uu - u * U) * ib;
  gy += G * (Uv - v * U) * ib;
}

// ------------------------------------------------------------------------------------------
// Accumulators -> d logL / d theta in the parameter order of gl.h. Returns d.
// ------------------------------------------------------------------------------------------
GL_HD void light_grad(const LightC& L, const double* a, float* g) {
  g[0] = float(a[L_RHO] * L.bn / (double(L.n) * L.re));                 // R_eff
  g[1] = float(-1.9992 * a[L_RHO1] + L.bn / double(L.n) * kLn2 * a[L_RHOLN]);  // n
  const double ge1 = L.inv1me2 * a[L_Q1], ge2 = L.inv1me2 * a[L_Q2];
  g[2] = float(L.j11 * ge1 + L.j12 * ge2);                               // eps1
  g[3] = float(L.j12 * ge1 + L.j22 * ge2);                               // eps2
  g[4] = float(-a[L_DX]);                                                // x
  g[5] = float(-a[L_DY]);                                                // y
  g[6] = float(a[L_E]);                                                  // I0
}

GL_HD int map_gradient(const PConst& c, const double* a, int mass, int shear, int lens_light,
                       int nmax, float* gr) {
  int j = 0;
  gr[j++] = float(-double(c.t) / c.theta_e * a[A_M_ALPHA]);
  if (mass == 1) gr[j++] = float(-a[A_M_T]);
  gr[j++] = float(-(c.mj11 * a[A_M_E1] + c.mj12 * a[A_M_E2]));
  gr[j++] = float(-(c.mj12 * a[A_M_E1] + c.mj22 * a[A_M_E2]));
  gr[j++] = float(a[A_M_X]);
  gr[j++] = float(a[A_M_Y]);
  if (shear) {
    gr[j++] = float(-a[A_M_G1]);
    gr[j++] = float(-a[A_M_G2]);
  }
  if (lens_light) {
    light_grad(c.lens, a + A_LENS, gr + j);
    j += 7;
  }
  light_grad(c.src, a + A_SRC, gr + j);
  j += 7;
  if (nmax >= 0) gr[j++] = float(a[A_SHP_BETA]);
  return j;
}

// Gradient component of shapelet coefficient q (0 <= q < M), whose slot in the gradient
// follows those of map_gradient.
GL_HD float shapelet_coef_grad(const PConst& c, const double* a, int q) {
  int n1, n2;
  shapelet_orders(q, n1, n2);
  return float(a[A_SHP_C + q] * (double(c.inv_beta) * kInvSqrtPi) * hermite_scale(n1, n2));
}

}  // namespace glens
