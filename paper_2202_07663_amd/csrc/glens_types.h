// Internal data layout shared by the host launchers and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace glens {

constexpr int kMaxTerms = 48;      // EPL series terms (|eps| <= 0.6 needs 47 at the tolerance)
// Power tables of the ray trace's A = B^t |w|^-t (PConst::pw): exponents e of |w|^2 = 2^e m
// from -kPowExp/2 to kPowExp/2 - 1, and kPowSeg polynomial segments of m in [1, 2).
constexpr int kPowExp = 128;
constexpr int kPowSeg = 16;
constexpr int kPowDeg = 6;
constexpr int kMaxNmax = 8;        // shapelet order
constexpr int kMaxShp = (kMaxNmax + 1) * (kMaxNmax + 2) / 2;  // 45
constexpr int kMaxParams = 68;
constexpr int kNAcc = 72;          // adjoint accumulator slots per (particle, tile)
constexpr float kR2Floor = 1e-12f; // arcsec^2 floor on elliptical radii
constexpr double kR2FloorD = 1e-12;
// Smallest sub-pixel pitch (arcsec): a mass radius below the floor needs the sub-pixel within
// 4e-6 arcsec of the lens centre (|eps| <= 0.6), so at most one sub-pixel can be floored.
constexpr double kMinPitch = 1e-4;
constexpr float kMassEpsMax = 0.6f;
constexpr float kLightEpsMax = 0.9f;
constexpr float kSieClosedMin = 0.1f;  // SIE closed form for |eps| >= this, series below
constexpr double kSeriesTol = 1e-10;   // EPL series truncation, relative (far below FP32)
constexpr double kSeriesTolDeriv = 1e-7;  // truncation of the derivative series (adjoint)
// dS/dX from S by the first-order identity of the series for |eps| >= this (its cancellation
// costs 1e-10 / |eps| relative: below 1e-8 here); the derivative series below
constexpr double kSxClosedMin = 0.02;

// Accumulator slots of the adjoint (per particle, summed over sub-pixels).
enum AccSlot {
  A_M_ALPHA = 0,  // sum g.alpha                      -> theta_E (and SIE)
  A_M_T = 1,      // sum g.(d alpha / d t)             -> gamma_epl
  A_M_E1 = 2, A_M_E2 = 3,   // sum g.(d alpha / d eps_k) (clamped eps)
  A_M_X = 4, A_M_Y = 5,     // sum g.(d alpha / d x), g.(d alpha / d y)
  A_M_G1 = 6, A_M_G2 = 7,   // sum g.(x, -y), g.(y, x)
  A_LENS = 8,     // 8 slots, see LightSlot
  A_SRC = 16,     // 8 slots; the centre slots also collect the shapelet beta-gradient
  A_SHP_BETA = 24,
  A_SHP_C = 25,   // kMaxShp slots
};
enum LightSlot { L_E = 0, L_RHO = 1, L_RHO1 = 2, L_RHOLN = 3, L_Q1 = 4, L_Q2 = 5, L_DX = 6, L_DY = 7 };
static_assert(A_SHP_C + kMaxShp <= kNAcc, "accumulator slots");

// Elliptical Sersic constants of one particle.
struct LightC {
  float qa, qb, qc;    // R^2 = qa dx^2 + qb dx dy + qc dy^2
  float qbh;           // qb / 2
  float kq;            // -b_n / n
  float inv2n;         // 1 / (2n)
  float l2re_n;        // log2(R_eff) / n
  float bn, i0;        // b_n = 1.9992 n - 0.3271, I0
  float bnl;           // b_n log2(e)
  float n, re;         // Sersic index, R_eff
  float e1, e2;        // clamped eccentricities
  float inv1me2;       // 1 / (1 - |eps|^2)
  float j11, j12, j22; // d eps_clamped / d eps (symmetric)
};

// Per-particle constants written by the prologue and read (uniformly) by every sub-pixel
// lane of that particle.
struct PConst {
  int nterms;          // EPL / SIE series terms
  int nterms_d;        // terms of the derivative series (adjoint), <= nterms
  int sie_closed;      // SIE: 1 = closed form, 0 = series
  // FP64 part: positions and the deflection are evaluated in double precision, because the
  // ray-traced source offset beta - x_s must be accurate to far below the FP32 resolution
  // of arcsecond-scale coordinates near a cuspy source.
  double t;            // gamma - 1
  double e1, e2;       // clamped mass eccentricities
  double xc, yc, g1, g2;
  double tlnb;         // t ln B, B = theta_E sqrt(1 - |eps|^2)
  double bmass;        // B
  double w2floor;      // R^2 floor expressed on |w|^2: 1e-12 (1 + |eps|)^2
  double sr, si;       // SIE closed form: s = sqrt(conj(eps))
  double epsabs;
  double c[kMaxTerms]; // series coefficients c_n(t)
  // A = B^t |w|^-t of the ray trace, with |w|^2 = 2^e m, m in [1, 2):
  //   pw[e + kPowExp/2] = B^t 2^(-t e / 2) (e clamped to the table),
  //   pw[kPowExp + 8 j + k] = coefficient k of the Taylor polynomial of m^(-t/2) about
  //   m_j = 1 + (j + 1/2)/16, in x = m - m_j, on the sixteenth of [1, 2) that holds m
  //   (degree 6: truncation below 3e-11 relative for 0 < t < 2)
  double pw[kPowExp + kPowSeg * 8];
  // The sub-pixel, if any, where the elliptical mass radius sits at its floor (the lens
  // centre within ~1e-6 arcsec of a sub-pixel centre; at most one, as sub-pixels are at least
  // kMinPitch apart): its row and column on the sub-pixel grid (-1: none), the deflection
  // there as the floored formula gives it, and its derivatives d alpha / d (t, eps1, eps2,
  // x_c, y_c) (clamped eccentricities), all FP64. The adjoint adds that sub-pixel's mass terms
  // from these instead of from its per-lane Jacobian.
  int fl_i, fl_j;
  double fl_a[2];
  double fl_d[5][2];
  double sxs, sys;     // source centre
  double lxs, lys;     // lens-light centre
  // FP32 part
  float theta_e, tf;   // Einstein radius, t
  float hp, hm;        // 1 - t/2, -t/2
  float xcf, ycf;      // lens centre (FP32, adjoint Jacobian)
  float w2floorf;      // R^2 floor on |w|^2 (FP32)
  float tlnb2;         // t ln B log2(e)
  float iebr, iebi;    // 1 / conj(eps) for |eps| >= kSxClosedMin, else 0 (adjoint Jacobian)
  float e1f, e2f;
  float lnb;
  float tfac;          // t / (2 (1 - |eps|^2))
  float mj11, mj12, mj22;
  LightC lens, src;
  float beta, inv_beta;
  float shp[kMaxShp];  // c_k r_n1 r_n2 / (beta sqrt(pi)), r_n = sqrt(2^n / n!)
  float dc[kMaxTerms]; // d c_n / dt (zero from nterms_d on)
  float nc[kMaxTerms]; // (n + 1) c_{n+1}: coefficients of dS/dy (zero from nterms_d - 1 on)
};

// Prior / bijector of one parameter (the fit).
struct Prior {
  int family;          // GL_PRIOR_*
  float mu, sigma, lo, hi;
  float logc;          // additive constant of log p (normalisation)
};

// One lens system as seen by one launch.
struct SysDesc {
  int H, W, k, K;
  double x0, y0, dxs;  // first sub-pixel centre and sub-pixel pitch (arcsec)
  float inv_k2;
  float s2b, inv_gt;   // sigma_bkg^2, 1 / (G t_exp)
  int mass, shear, lens_light, nmax, d;
  int P;
  int tiles;           // sub-pixel work tiles per particle (adjoint; its accumulator rows)
  int pix_per_tile;
  int ftiles;          // the same for the forward pass
  int fpix_per_tile;
  int mode;            // conv kernel: 0 image, 1 log L, 2 log L + adjoint seed
  int bands;           // banded PSF pass: row bands per particle (1: whole image)
  int band_rows;       // rows per band (a multiple of the strip height)
  int band_split;      // banded pass: lanes that share one strip's PSF columns (1, 2 or 4)
  const float* obs;
  const float* psf;      // K*K
  const float* psf_flip; // K*K, flipped in both axes
  const uint4* psf_mfma; // [2][K][64 lanes][2 parts] Toeplitz fragments (flipped, plain)
  int psf_mfma_exp;      // the fragments hold psf 2^psf_mfma_exp
  int conv_mfma;         // 1: PSF pass on matrix cores
  const float* theta;    // [P][d] physical parameters, or null if z is given
  float* z;              // [P][d] unconstrained parameters (fit), or null
  const Prior* prior;    // [d] (fit)
  float* theta_out;      // [P][d] physical parameters written when z is given
  float* mom1;           // [P][d] Adam first moment (fit)
  float* mom2;           // [P][d] Adam second moment (fit)
  double* logpost;       // [P] log L + log p~ (fit result)
  double* chi2;          // [P] chi^2 (optional output of the likelihood pass)
  int step, nsteps;      // 0-based Adam step, schedule length K
  float lr0, lr1, beta1, beta2, eps_adam;
  uint32_t seed_lo, seed_hi;
  PConst* pc;            // [P]
  float* m0;             // [P][H][W] downsampled image before the PSF
  float* img;            // [P][H][W] model image (mode 0)
  float* sbar;           // [P][H][W] d logL / d (sub-pixel brightness) per pixel
  double* acc;           // [P][tiles][kNAcc]
  double* logl;          // [P]
  float* grad;           // [P][d]
  float* seed;           // [P][H][W] adjoint seed (banded PSF pass)
  float2* beta;          // [P][k^2][H][W] beta - x_s of the forward pass (gradient calls)
  double* lpart;         // [P][max bands][2] log L and chi^2 partial sums per band
  struct FitOut* fit_out;  // result of a served fit (fit_best_kernel), or null
};

// Result of one fit, formed on the device so that it can be copied to the host without
// waiting on the stream: the best particle by log posterior (-1: none finite) and its values.
struct FitOut {
  int best;
  int pad;
  double logl, logpost, chi2;
  float theta[kMaxParams], z[kMaxParams];
};

// PSF pass on matrix cores (v_mfma_f32_16x16x32_f16, operands scaled and split into two fp16
// parts): for each PSF row a the output tile
// [16 rows x N columns] += (image rows shifted by a, a 32-column window) x (the 32 x 16
// Toeplitz matrix T_a[kk][n] = psf[a][kk - n]). N = min(16, 33 - K), rounded down to a
// multiple of 4, columns fit the window.
constexpr int kMfmaMaxK = 21;       // largest PSF for this pass
constexpr int kMfmaWaveTiles = 16;  // output tiles per wave (4 waves: <= 64 tiles per image)

struct MfmaGeom {
  int N;       // useful output columns per tile
  int TR, TC;  // tile rows / columns
  int T;       // tiles
  int Hq;      // rows of the padded image in LDS (image and halo: H + K - 1)
  int pitch;   // row pitch in 16-bit elements (a multiple of 4)
};
__host__ __device__ inline MfmaGeom mfma_geom(int H, int W, int K) {
  MfmaGeom q;
  // a multiple of 4, so that every tile's fragment offset (tile column tc N, lane group 8 g,
  // row pitch) is a multiple of four fp16 and the 8-byte LDS fragment reads stay aligned
  // (K <= 21 gives N >= 12; the geometry of larger PSFs, which never take this pass, keeps
  // N >= 1)
  const int n = 33 - K < 16 ? 33 - K : 16;
  q.N = n >= 4 ? n & ~3 : (n < 1 ? 1 : n);
  q.TR = (H + 15) / 16;
  q.TC = (W + q.N - 1) / q.N;
  q.T = q.TR * q.TC;
  q.Hq = H + K - 1;
  q.pitch = ((q.TC - 1) * q.N + 32 + 3) & ~3;  // the last tile's 32-column window
  return q;
}
// LDS bytes of the pass: the padded image as two fp16 parts, and the FP32 pixel seed. The
// tiles' last 16 - H % 16 rows (outputs past the image, never used) read up to 16 TR - H
// rows past each part; past the second part those reads fall in the seed area, which is
// made at least that long.
__host__ __device__ inline int mfma_lds_bytes(const MfmaGeom& q, int H, int W) {
  const int over = 2 * (q.TR * 16 - H) * q.pitch;
  return 4 * q.Hq * q.pitch + (4 * H * W > over ? 4 * H * W : over);
}

constexpr int kMaxGroup = 10;
constexpr int kConvMaxBands = 8;  // row bands per particle in the small-batch PSF pass

// Systems that share one launch (same kernel configuration). Passed by value.
struct Group {
  int nsys;
  int block0[kMaxGroup + 1];  // first block of each system; block0[nsys] = grid size
  SysDesc sys[kMaxGroup];
};
static_assert(sizeof(Group) <= 4000, "kernel argument size");

}  // namespace glens
