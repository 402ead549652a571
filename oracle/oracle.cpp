// FP64 CPU oracle for the GIGA-Lens lens model (Gu et al. 2022, arXiv:2202.07663).
//
// TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the CPU-baseline leg of the
// benchmark call this code; the product library never does, and the two share no code.
//
// What it computes, in the order the paper states it (Sec. 2.1.1 "Physical Model" and
// Sec. 2.1.2 "Probabilistic Model"):
//   1. pixel and supersampled grid (Sec. 2.1.1, last paragraph);
//   2. eccentricities -> (q, phi) (eq. for (eps1, eps2)) and the frame rotation
//      (eq. coord-trans);
//   3. EPL deflection through the Gauss hypergeometric function, summed as its defining
//      power series (Sec. 2.1.1, citing Tessore & Metcalf 2015); SIE closed form (the
//      slope-2 case); external shear (eq. alpha_ext);
//   4. ray trace beta = x - alpha and elliptical Sersic light (eq. Sersic), plus Cartesian
//      shapelets (Refregier 2003; the paper names shapelets in Sec. 4 but prints no
//      formula);
//   5. k x k mean downsampling, then the PSF convolution ("finally convolving");
//   6. the Gaussian log-likelihood with model-dependent variance (eq. model-def).
// The gradient is exact forward-mode differentiation (dual numbers) of the same code.
//
// Plain and slow on purpose: every pixel and sub-pixel is evaluated on its own, sums are
// plain FP64 loops, no blocking, fusion or reordering.
//
// Readings where the paper is silent (each is listed in the design notes):
//   * pixel (i, j) has centre ((j - (W-1)/2) s, (i - (H-1)/2) s); sub-pixel (a, b) of it is
//     offset by (((b + 1/2)/k - 1/2) s, ((a + 1/2)/k - 1/2) s);
//   * |eps| is clamped by rescaling (eps1, eps2) onto radius 0.6 (mass) or 0.9 (light);
//   * R^2 >= 1e-12 arcsec^2 in the EPL, SIE and Sersic radii;
//   * the PSF acts after downsampling, as a zero-padded "same" convolution;
//   * sigma_tot^2 uses max(I_model, 0);
//   * shapelets: circular Cartesian basis, centre tied to the source Sersic centre, order
//     n = 0..n_max, n1 = n..0, n2 = n - n1.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------------------------------
// Forward-mode dual numbers: value plus D partial derivatives.
// ---------------------------------------------------------------------------------------
template <int D>
struct Dual {
  double v;
  double g[D];
  Dual() : v(0.0) { std::memset(g, 0, sizeof(g)); }
  Dual(double x) : v(x) { std::memset(g, 0, sizeof(g)); }  // NOLINT: implicit on purpose
};

template <int D> Dual<D> operator+(const Dual<D>& a, const Dual<D>& b) {
  Dual<D> r; r.v = a.v + b.v;
  for (int i = 0; i < D; ++i) r.g[i] = a.g[i] + b.g[i];
  return r;
}
template <int D> Dual<D> operator-(const Dual<D>& a, const Dual<D>& b) {
  Dual<D> r; r.v = a.v - b.v;
  for (int i = 0; i < D; ++i) r.g[i] = a.g[i] - b.g[i];
  return r;
}
template <int D> Dual<D> operator-(const Dual<D>& a) {
  Dual<D> r; r.v = -a.v;
  for (int i = 0; i < D; ++i) r.g[i] = -a.g[i];
  return r;
}
template <int D> Dual<D> operator*(const Dual<D>& a, const Dual<D>& b) {
  Dual<D> r; r.v = a.v * b.v;
  for (int i = 0; i < D; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
  return r;
}
template <int D> Dual<D> operator/(const Dual<D>& a, const Dual<D>& b) {
  Dual<D> r; r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
  for (int i = 0; i < D; ++i) r.g[i] = (a.g[i] - r.v * b.g[i]) * ib;
  return r;
}
template <int D> Dual<D> operator+(const Dual<D>& a, double b) { return a + Dual<D>(b); }
template <int D> Dual<D> operator+(double a, const Dual<D>& b) { return Dual<D>(a) + b; }
template <int D> Dual<D> operator-(const Dual<D>& a, double b) { return a - Dual<D>(b); }
template <int D> Dual<D> operator-(double a, const Dual<D>& b) { return Dual<D>(a) - b; }
template <int D> Dual<D> operator*(const Dual<D>& a, double b) {
  Dual<D> r; r.v = a.v * b;
  for (int i = 0; i < D; ++i) r.g[i] = a.g[i] * b;
  return r;
}
template <int D> Dual<D> operator*(double a, const Dual<D>& b) { return b * a; }
template <int D> Dual<D> operator/(const Dual<D>& a, double b) { return a * (1.0 / b); }
template <int D> Dual<D> operator/(double a, const Dual<D>& b) { return Dual<D>(a) / b; }
template <int D> Dual<D>& operator+=(Dual<D>& a, const Dual<D>& b) { a = a + b; return a; }
template <int D> Dual<D>& operator-=(Dual<D>& a, const Dual<D>& b) { a = a - b; return a; }
template <int D> Dual<D>& operator*=(Dual<D>& a, const Dual<D>& b) { a = a * b; return a; }

// Chain rule for a scalar function f with value fv and derivative df at a.v.
template <int D> Dual<D> chain(const Dual<D>& a, double fv, double df) {
  Dual<D> r; r.v = fv;
  for (int i = 0; i < D; ++i) r.g[i] = df * a.g[i];
  return r;
}
template <int D> Dual<D> sqrt(const Dual<D>& a) {
  const double s = std::sqrt(a.v);
  return chain(a, s, 0.5 / s);
}
template <int D> Dual<D> exp(const Dual<D>& a) {
  const double e = std::exp(a.v);
  return chain(a, e, e);
}
template <int D> Dual<D> log(const Dual<D>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int D> Dual<D> sin(const Dual<D>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int D> Dual<D> cos(const Dual<D>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int D> Dual<D> atan(const Dual<D>& a) {
  return chain(a, std::atan(a.v), 1.0 / (1.0 + a.v * a.v));
}
template <int D> Dual<D> atanh(const Dual<D>& a) {
  return chain(a, std::atanh(a.v), 1.0 / (1.0 - a.v * a.v));
}
template <int D> Dual<D> atan2(const Dual<D>& y, const Dual<D>& x) {
  // d atan2(y, x) = (x dy - y dx) / (x^2 + y^2)
  Dual<D> r; r.v = std::atan2(y.v, x.v);
  const double n = x.v * x.v + y.v * y.v;
  for (int i = 0; i < D; ++i) r.g[i] = (x.v * y.g[i] - y.v * x.g[i]) / n;
  return r;
}
// a^p for a > 0 and a dual exponent p.
template <int D> Dual<D> pow(const Dual<D>& a, const Dual<D>& p) { return exp(p * log(a)); }

inline double value(double x) { return x; }
template <int D> double value(const Dual<D>& x) { return x.v; }

using std::atan;
using std::atan2;
using std::atanh;
using std::cos;
using std::exp;
using std::log;
using std::pow;
using std::sin;
using std::sqrt;

template <class T> T sq(const T& x) { return x * x; }

// max(x, floor) with the derivative of whichever branch is taken.
template <class T> T floor_at(const T& x, double floor) { return value(x) < floor ? T(floor) : x; }

constexpr double kPi = 3.14159265358979323846;
constexpr double kR2Floor = 1e-12;      // arcsec^2, floor on every elliptical radius^2
constexpr double kMassEpsMax = 0.6;     // |eps| clamp for the lens mass
constexpr double kLightEpsMax = 0.9;    // |eps| clamp for light profiles

// ---------------------------------------------------------------------------------------
// Model description. Parameter layout (rows of theta):
//   mass:       theta_E, [gamma_epl if EPL], eps1, eps2, x, y, [gamma_ext1, gamma_ext2]
//   lens light: R, n, eps1, eps2, x, y, I0                       (if lens_light)
//   source:     R, n, eps1, eps2, x, y, I0
//   shapelets:  beta, c_0 .. c_{M-1}, M = (nmax+1)(nmax+2)/2     (if nmax >= 0)
// ---------------------------------------------------------------------------------------
struct Model {
  int H, W, k;
  double pix;        // arcsec per pixel
  int epl;           // 0 = SIE, 1 = EPL
  int shear;         // 0/1
  int lens_light;    // 0/1
  int nmax;          // -1 = no shapelets
  int K;             // PSF side (odd)
  const double* psf; // K*K row-major
  double sigma_bkg, t_exp, gain;
};

int n_mass(const Model& m) { return (m.epl ? 6 : 5) + (m.shear ? 2 : 0); }
int n_shapelet_coeffs(int nmax) { return nmax < 0 ? 0 : (nmax + 1) * (nmax + 2) / 2; }
int n_params(const Model& m) {
  return n_mass(m) + (m.lens_light ? 7 : 0) + 7 + (m.nmax >= 0 ? 1 + n_shapelet_coeffs(m.nmax) : 0);
}

// ---------------------------------------------------------------------------------------
// Eccentricities and frames (Sec. 2.1.1, eq. for (eps1, eps2) and eq. coord-trans).
// ---------------------------------------------------------------------------------------

// (eps1, eps2) = (1-q)/(1+q) (cos 2phi, sin 2phi) inverted: q = (1-|eps|)/(1+|eps|),
// phi = atan2(eps2, eps1)/2. |eps| above eps_max is rescaled onto eps_max.
template <class T> void axis_ratio_angle(T e1, T e2, double eps_max, T& q, T& phi) {
  T eps = sqrt(e1 * e1 + e2 * e2);
  if (value(eps) > eps_max) {
    e1 = e1 * (eps_max / eps);
    e2 = e2 * (eps_max / eps);
    eps = sqrt(e1 * e1 + e2 * e2);
  }
  q = (1.0 - eps) / (1.0 + eps);
  phi = 0.5 * atan2(e2, e1);
}

// [x_l, y_l] = [[cos phi, sin phi], [-sin phi, cos phi]] [x - x_c, y - y_c]
template <class T> void to_frame(const T& dx, const T& dy, const T& phi, T& xl, T& yl) {
  const T c = cos(phi), s = sin(phi);
  xl = c * dx + s * dy;
  yl = -s * dx + c * dy;
}

// Inverse rotation, for vectors (deflections) computed in the lens frame.
template <class T> void from_frame(const T& vx, const T& vy, const T& phi, T& ox, T& oy) {
  const T c = cos(phi), s = sin(phi);
  ox = c * vx - s * vy;
  oy = s * vx + c * vy;
}

// ---------------------------------------------------------------------------------------
// Gauss hypergeometric 2F1(1, t/2; 2 - t/2; z) for complex |z| < 1, summed as its
// defining power series sum_n (1)_n (t/2)_n / ((2 - t/2)_n n!) z^n. With a = 1 the
// Pochhammer ratio (1)_n / n! is 1, so consecutive coefficients differ by the factor
// (t/2 + n - 1) / (2 - t/2 + n - 1). Terms are added until the coefficient falls below
// 1e-17 (the paper quotes < 1e-16 truncation error within 35 terms for q >~ 0.5), with a
// cap of 400 terms.
// ---------------------------------------------------------------------------------------
template <class T> void hyp2f1_series(const T& t, const T& zr, const T& zi, T& fr, T& fi) {
  T coef(1.0);             // (t/2)_n / (2 - t/2)_n
  T pr(1.0), pi(0.0);      // z^n
  fr = T(1.0);
  fi = T(0.0);
  const T a = 0.5 * t, c = 2.0 - 0.5 * t;
  for (int n = 1; n < 400; ++n) {
    coef = coef * (a + (n - 1)) / (c + (n - 1));
    const T nr = pr * zr - pi * zi;
    const T ni = pr * zi + pi * zr;
    pr = nr;
    pi = ni;
    fr += coef * pr;
    fi += coef * pi;
    const double bound = std::fabs(value(coef)) * std::sqrt(sq(value(pr)) + sq(value(pi)));
    if (bound < 1e-17) break;
  }
}

// ---------------------------------------------------------------------------------------
// EPL deflection (Sec. 2.1.1: kappa = (3-g)/2 (theta_E / sqrt(q x^2 + y^2/q))^(g-1);
// deflection from Tessore & Metcalf 2015). In their variables b = theta_E sqrt(q),
// t = g - 1, R = sqrt(q^2 x_l^2 + y_l^2) and elliptical angle (q x_l, y_l) = R (cos v, sin v):
//   alpha_l = 2b/(1+q) (b/R)^(t-1) e^{iv} 2F1(1, t/2; 2 - t/2; -(1-q)/(1+q) e^{2iv}).
// ---------------------------------------------------------------------------------------
template <class T>
void epl_deflection(const T& x, const T& y, const T& theta_e, const T& gamma, const T& e1,
                    const T& e2, const T& xc, const T& yc, T& ax, T& ay) {
  T q, phi;
  axis_ratio_angle(e1, e2, kMassEpsMax, q, phi);
  T xl, yl;
  to_frame(x - xc, y - yc, phi, xl, yl);
  const T t = gamma - 1.0;
  const T b = theta_e * sqrt(q);
  const T r2 = floor_at(q * q * xl * xl + yl * yl, kR2Floor);
  const T r = sqrt(r2);
  const T cv = q * xl / r, sv = yl / r;                 // e^{iv}
  const T f = (1.0 - q) / (1.0 + q);
  const T zr = -f * (cv * cv - sv * sv), zi = -f * (2.0 * cv * sv);  // -f e^{2iv}
  T fr, fi;
  hyp2f1_series(t, zr, zi, fr, fi);
  const T pref = 2.0 * b / (1.0 + q) * pow(b / r, t - 1.0);
  const T axl = pref * (cv * fr - sv * fi);
  const T ayl = pref * (cv * fi + sv * fr);
  from_frame(axl, ayl, phi, ax, ay);
}

// SIE (EPL with slope 2, t = 1): closed form with q' = sqrt(1 - q^2),
// psi = sqrt(q^2 x_l^2 + y_l^2): alpha_l = b/q' (atan(q' x_l/psi), atanh(q' y_l/psi)).
template <class T>
void sie_deflection(const T& x, const T& y, const T& theta_e, const T& e1, const T& e2,
                    const T& xc, const T& yc, T& ax, T& ay) {
  T q, phi;
  axis_ratio_angle(e1, e2, kMassEpsMax, q, phi);
  T xl, yl;
  to_frame(x - xc, y - yc, phi, xl, yl);
  const T b = theta_e * sqrt(q);
  const T psi = sqrt(floor_at(q * q * xl * xl + yl * yl, kR2Floor));
  T axl, ayl;
  if (value(q) >= 1.0) {  // circular: the singular isothermal sphere
    axl = b * xl / psi;
    ayl = b * yl / psi;
  } else {
    const T qp = sqrt(1.0 - q * q);
    axl = b / qp * atan(qp * xl / psi);
    ayl = b / qp * atanh(qp * yl / psi);
  }
  from_frame(axl, ayl, phi, ax, ay);
}

// EPL convergence exactly as printed (Sec. 2.1.1).
template <class T>
T epl_kappa(const T& x, const T& y, const T& theta_e, const T& gamma, const T& e1, const T& e2,
            const T& xc, const T& yc) {
  T q, phi;
  axis_ratio_angle(e1, e2, kMassEpsMax, q, phi);
  T xl, yl;
  to_frame(x - xc, y - yc, phi, xl, yl);
  return (3.0 - gamma) / 2.0 * pow(theta_e / sqrt(q * xl * xl + yl * yl / q), gamma - 1.0);
}

// External shear (eq. alpha_ext), origin at the image centre.
template <class T>
void shear_deflection(const T& x, const T& y, const T& g1, const T& g2, T& ax, T& ay) {
  ax = g1 * x + g2 * y;
  ay = g2 * x - g1 * y;
}

// ---------------------------------------------------------------------------------------
// Elliptical Sersic (eq. Sersic): I = I0 exp(-b_n ((sqrt(q x_l^2 + y_l^2/q)/R_eff)^(1/n) - 1)),
// b_n = 1.9992 n - 0.3271 as printed.
// ---------------------------------------------------------------------------------------
template <class T>
T sersic(const T& x, const T& y, const T& r_eff, const T& n, const T& e1, const T& e2,
         const T& xc, const T& yc, const T& i0) {
  T q, phi;
  axis_ratio_angle(e1, e2, kLightEpsMax, q, phi);
  T xl, yl;
  to_frame(x - xc, y - yc, phi, xl, yl);
  const T r = sqrt(floor_at(q * xl * xl + yl * yl / q, kR2Floor));
  const T bn = 1.9992 * n - 0.3271;
  return i0 * exp(-bn * (pow(r / r_eff, 1.0 / n) - 1.0));
}

// ---------------------------------------------------------------------------------------
// Cartesian shapelets (Refregier 2003): phi_n(u) = [2^n sqrt(pi) n!]^(-1/2) H_n(u) e^(-u^2/2)
// with physicists' Hermite polynomials H_0 = 1, H_1 = 2u, H_{n+1} = 2u H_n - 2n H_{n-1};
// B_{n1 n2}(x, y; beta) = beta^-1 phi_n1(x/beta) phi_n2(y/beta).
// ---------------------------------------------------------------------------------------
template <class T> void hermite_functions(const T& u, int nmax, T* out) {
  std::vector<T> h(nmax + 2);
  h[0] = T(1.0);
  if (nmax >= 1) h[1] = 2.0 * u;
  for (int n = 1; n < nmax; ++n) h[n + 1] = 2.0 * u * h[n] - (2.0 * n) * h[n - 1];
  const T g = exp(-0.5 * u * u);
  double fact = 1.0;
  for (int n = 0; n <= nmax; ++n) {
    if (n > 0) fact *= n;
    const double norm = 1.0 / std::sqrt(std::ldexp(1.0, n) * std::sqrt(kPi) * fact);
    out[n] = norm * h[n] * g;
  }
}

template <class T>
T shapelets(const T& x, const T& y, const T& xc, const T& yc, const T& beta, const T* coeffs,
            int nmax) {
  std::vector<T> pu(nmax + 1), pv(nmax + 1);
  hermite_functions((x - xc) / beta, nmax, pu.data());
  hermite_functions((y - yc) / beta, nmax, pv.data());
  T s(0.0);
  int k = 0;
  for (int n = 0; n <= nmax; ++n)
    for (int n1 = n; n1 >= 0; --n1, ++k) s += coeffs[k] * pu[n1] * pv[n - n1];
  return s / beta;
}

// ---------------------------------------------------------------------------------------
// Surface brightness at one image-plane point: deflect, ray trace, evaluate the source at
// beta (surface-brightness conservation) and add the lens light at x (Sec. 2.1.1).
// ---------------------------------------------------------------------------------------
template <class T> T surface_brightness(const Model& m, const T* th, double xd, double yd) {
  const T x(xd), y(yd);
  int p = 0;
  T ax, ay;
  if (m.epl) {
    epl_deflection(x, y, th[0], th[1], th[2], th[3], th[4], th[5], ax, ay);
    p = 6;
  } else {
    sie_deflection(x, y, th[0], th[1], th[2], th[3], th[4], ax, ay);
    p = 5;
  }
  if (m.shear) {
    T sx, sy;
    shear_deflection(x, y, th[p], th[p + 1], sx, sy);
    ax += sx;
    ay += sy;
    p += 2;
  }
  T lens(0.0);
  if (m.lens_light) {
    lens = sersic(x, y, th[p], th[p + 1], th[p + 2], th[p + 3], th[p + 4], th[p + 5], th[p + 6]);
    p += 7;
  }
  const T bx = x - ax, by = y - ay;  // ray trace to the source plane
  const int ps = p;
  T src = sersic(bx, by, th[p], th[p + 1], th[p + 2], th[p + 3], th[p + 4], th[p + 5], th[p + 6]);
  p += 7;
  if (m.nmax >= 0) src += shapelets(bx, by, th[ps + 4], th[ps + 5], th[p], th + p + 1, m.nmax);
  return src + lens;
}

double pixel_centre(int idx, int n, double pix) { return (idx - 0.5 * (n - 1)) * pix; }

// Noiseless model image: supersample, downsample by the k x k mean, then convolve with the
// PSF (zero padding, output the same size as the image).
template <class T> void model_image(const Model& m, const T* th, T* img) {
  const int H = m.H, W = m.W, k = m.k;
  std::vector<T> low(static_cast<size_t>(H) * W);
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      T acc(0.0);
      for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) {
          const double x = pixel_centre(j, W, m.pix) + ((b + 0.5) / k - 0.5) * m.pix;
          const double y = pixel_centre(i, H, m.pix) + ((a + 0.5) / k - 0.5) * m.pix;
          acc += surface_brightness(m, th, x, y);
        }
      low[static_cast<size_t>(i) * W + j] = acc / double(k * k);
    }
  const int K = m.K, c = (K - 1) / 2;
  for (int i = 0; i < H; ++i)
    for (int j = 0; j < W; ++j) {
      T acc(0.0);
      for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) {
          const int ii = i + c - a, jj = j + c - b;
          if (ii < 0 || ii >= H || jj < 0 || jj >= W) continue;
          acc += m.psf[a * K + b] * low[static_cast<size_t>(ii) * W + jj];
        }
      img[static_cast<size_t>(i) * W + j] = acc;
    }
}

// eq. model-def: log L = -1/2 sum [ (I_obs - I_model)^2 / s2 + log(2 pi s2) ],
// s2 = sigma_bkg^2 + max(I_model, 0) / (G t_exp).
template <class T> T log_likelihood(const Model& m, const T* img, const double* obs) {
  T acc(0.0);
  const double s2b = m.sigma_bkg * m.sigma_bkg, inv_gt = 1.0 / (m.gain * m.t_exp);
  for (int p = 0; p < m.H * m.W; ++p) {
    const T mod = img[p];
    const T pos = value(mod) > 0.0 ? mod : T(0.0);
    const T s2 = s2b + pos * inv_gt;
    const T r = obs[p] - mod;
    acc += r * r / s2 + log(2.0 * kPi * s2);
  }
  return -0.5 * acc;
}

template <int D>
void loglik_grad_one(const Model& m, const double* th, const double* obs, double* logl,
                     double* grad) {
  const int d = n_params(m);
  std::vector<Dual<D>> t(d);
  for (int i = 0; i < d; ++i) {
    t[i] = Dual<D>(th[i]);
    t[i].g[i] = 1.0;
  }
  std::vector<Dual<D>> img(static_cast<size_t>(m.H) * m.W);
  model_image(m, t.data(), img.data());
  const Dual<D> ll = log_likelihood(m, img.data(), obs);
  *logl = ll.v;
  for (int i = 0; i < d; ++i) grad[i] = ll.g[i];
}

}  // namespace

// =======================================================================================
// C interface (ctypes). All arrays are host FP64, row-major.
// =======================================================================================
extern "C" {

struct or_model_desc {
  int H, W, k;
  double pix;
  int epl, shear, lens_light, nmax;
  int K;
  const double* psf;
  double sigma_bkg, t_exp, gain;
};

static Model to_model(const or_model_desc* d) {
  Model m;
  m.H = d->H; m.W = d->W; m.k = d->k; m.pix = d->pix;
  m.epl = d->epl; m.shear = d->shear; m.lens_light = d->lens_light; m.nmax = d->nmax;
  m.K = d->K; m.psf = d->psf;
  m.sigma_bkg = d->sigma_bkg; m.t_exp = d->t_exp; m.gain = d->gain;
  return m;
}

int or_nparams(const or_model_desc* d) { return n_params(to_model(d)); }

// Threads the parallel loops below use.
void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Noiseless model images, img[P][H][W].
void or_simulate(const or_model_desc* d, const double* theta, int P, double* img) {
  const Model m = to_model(d);
  const int np = n_params(m);
  const size_t hw = static_cast<size_t>(m.H) * m.W;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; ++p) model_image(m, theta + static_cast<size_t>(p) * np, img + p * hw);
}

void or_loglik(const or_model_desc* d, const double* theta, int P, const double* obs,
               double* logl) {
  const Model m = to_model(d);
  const int np = n_params(m);
  const size_t hw = static_cast<size_t>(m.H) * m.W;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; ++p) {
    std::vector<double> img(hw);
    model_image(m, theta + static_cast<size_t>(p) * np, img.data());
    logl[p] = log_likelihood(m, img.data(), obs);
  }
}

// log L and its exact gradient (forward-mode duals). Returns -1 if d exceeds 72.
int or_loglik_grad(const or_model_desc* d, const double* theta, int P, const double* obs,
                   double* logl, double* grad) {
  const Model m = to_model(d);
  const int np = n_params(m);
  if (np > 72) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int p = 0; p < P; ++p) {
    const double* th = theta + static_cast<size_t>(p) * np;
    double* g = grad + static_cast<size_t>(p) * np;
    if (np <= 16) loglik_grad_one<16>(m, th, obs, logl + p, g);
    else if (np <= 32) loglik_grad_one<32>(m, th, obs, logl + p, g);
    else if (np <= 56) loglik_grad_one<56>(m, th, obs, logl + p, g);
    else loglik_grad_one<72>(m, th, obs, logl + p, g);
  }
  return 0;
}

// ---- component evaluators for the closed-form pins ----

void or_epl_deflection(int n, const double* x, const double* y, double theta_e, double gamma,
                       double e1, double e2, double xc, double yc, double* ax, double* ay) {
  for (int i = 0; i < n; ++i)
    epl_deflection(x[i], y[i], theta_e, gamma, e1, e2, xc, yc, ax[i], ay[i]);
}

void or_sie_deflection(int n, const double* x, const double* y, double theta_e, double e1,
                       double e2, double xc, double yc, double* ax, double* ay) {
  for (int i = 0; i < n; ++i) sie_deflection(x[i], y[i], theta_e, e1, e2, xc, yc, ax[i], ay[i]);
}

void or_epl_kappa(int n, const double* x, const double* y, double theta_e, double gamma,
                  double e1, double e2, double xc, double yc, double* out) {
  for (int i = 0; i < n; ++i) out[i] = epl_kappa(x[i], y[i], theta_e, gamma, e1, e2, xc, yc);
}

void or_hyp2f1(int n, double t, const double* zr, const double* zi, double* fr, double* fi) {
  for (int i = 0; i < n; ++i) hyp2f1_series(t, zr[i], zi[i], fr[i], fi[i]);
}

void or_shear_deflection(int n, const double* x, const double* y, double g1, double g2,
                         double* ax, double* ay) {
  for (int i = 0; i < n; ++i) shear_deflection(x[i], y[i], g1, g2, ax[i], ay[i]);
}

void or_sersic(int n, const double* x, const double* y, double r_eff, double nn, double e1,
               double e2, double xc, double yc, double i0, double* out) {
  for (int i = 0; i < n; ++i) out[i] = sersic(x[i], y[i], r_eff, nn, e1, e2, xc, yc, i0);
}

// out[i][0..nmax] = phi_0..phi_nmax at u[i]
void or_hermite_functions(int n, const double* u, int nmax, double* out) {
  for (int i = 0; i < n; ++i) hermite_functions(u[i], nmax, out + static_cast<size_t>(i) * (nmax + 1));
}

void or_shapelets(int n, const double* x, const double* y, double xc, double yc, double beta,
                  const double* coeffs, int nmax, double* out) {
  for (int i = 0; i < n; ++i) out[i] = shapelets(x[i], y[i], xc, yc, beta, coeffs, nmax);
}

// Surface brightness (before downsampling and PSF) at arbitrary points.
void or_surface_brightness(const or_model_desc* d, const double* theta, int n, const double* x,
                           const double* y, double* out) {
  const Model m = to_model(d);
  for (int i = 0; i < n; ++i) out[i] = surface_brightness(m, theta, x[i], y[i]);
}

double or_log_likelihood_image(const or_model_desc* d, const double* img, const double* obs) {
  const Model m = to_model(d);
  return log_likelihood(m, img, obs);
}

}  // extern "C"
