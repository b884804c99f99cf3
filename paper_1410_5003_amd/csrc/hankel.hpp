// Hankel-function kernels for the free-space Helmholtz Green's function
// G = (i/4) H0^(1)(k r) (Sec. 2, eq. (11)), float64.
//
// For x = k r the routine returns
//   h0   = H0^(1)(x)
//   g1m  = (i pi x / 2) H1^(1)(x) - 1      (-> 0 like x^2 log x as x -> 0)
// which is what the layer-potential kernels need: the k-independent 1/r^2
// singularities sit in the "1" that g1m removes, so the self-block difference
// kernels K^{k_i} - K^{k_{i+1}} are formed from g1m and h0 alone.
//
// Three branches, all from Abramowitz & Stegun:
//   x <= 2        ascending series (A&S 9.1.10, 9.1.11, 9.1.13);
//   2 < x < 20    Miller backward recurrence for J_n with the normalisation
//                 J0 + 2 sum J_2k = 1 (A&S 9.1.87) and Neumann series for
//                 Y0 (A&S 9.1.88) and Y1 = -Y0';
//   x >= 20       Hankel asymptotic expansion (A&S 9.2.5-9.2.10).
#pragma once
#include <hip/hip_runtime.h>

namespace mlh {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kEulerGamma = 0.5772156649015328606065120900824024310;
constexpr double kSqrtHalf = 0.7071067811865475244008443621048490393;
constexpr double kHankelSeriesMax = 2.0;
constexpr double kHankelAsympMin = 20.0;

struct cplx {
  double re, im;
};

__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// ascending series for 0 < x <= 2
__host__ __device__ inline void hankel_series(double x, cplx& h0, cplx& g1m) {
  const double z = 0.5 * x;
  const double q = -z * z;
  const double lg = log(z);
  double t0 = 1.0, t1 = 1.0, harm = 0.0;
  double sj0 = 1.0, sj1 = 1.0, sy0 = 0.0;
  double sg = 1.0 - 2.0 * kEulerGamma;  // psi(1) + psi(2)
#pragma unroll
  for (int m = 1; m <= 16; ++m) {
    const double dm = (double)m;
    // reciprocals of constants fold once the loop is unrolled
    t0 *= q * (1.0 / (dm * dm));
    t1 *= q * (1.0 / (dm * (dm + 1.0)));
    harm += 1.0 / dm;
    sj0 += t0;
    sj1 += t1;
    sy0 -= harm * t0;
    sg += (2.0 * (harm - kEulerGamma) + 1.0 / (dm + 1.0)) * t1;
  }
  const double j1 = z * sj1;
  h0.re = sj0;
  h0.im = (2.0 / kPi) * ((lg + kEulerGamma) * sj0 + sy0);
  // (pi x/2) Y1 = -1 + x log(x/2) J1 - (x/2)^2 sum (psi(m+1)+psi(m+2)) (-x^2/4)^m/(m!(m+1)!)
  g1m.re = -x * lg * j1 + z * z * sg;
  g1m.im = 0.5 * kPi * x * j1;
}

// 1/k for a small positive integer k: the hardware reciprocal refined by one
// Newton step (within an ulp, a few instructions instead of a division)
__device__ inline double inv_int(int k) {
  const double d = (double)k;
  const double r = __builtin_amdgcn_rcp(d);
  return __builtin_fma(r, __builtin_fma(-d, r, 1.0), r);
}

// Miller backward recurrence, 2 < x < 20
__device__ inline void hankel_miller(double x, cplx& h0, cplx& g1m) {
  const int nstart = 2 * ((int)(x + 4.0 * sqrt(x) + 16.0) / 2);
  const double tx = 2.0 / x;
  double jn1 = 0.0;      // J_{n+1}
  double jn = 1e-200;    // J_n, arbitrary scale
  double norm = 0.0, sy0 = 0.0, sa = 0.0, sb = 0.0, j1 = 0.0;
  for (int n = nstart; n >= 1; --n) {
    // jn holds J_n here
    if (n & 1) {
      const int ka = (n + 1) / 2;
      const double sgn_a = (ka & 1) ? -1.0 : 1.0;
      sa += sgn_a * jn * inv_int(ka);
      if (n >= 3) {
        const int kb = (n - 1) / 2;
        const double sgn_b = (kb & 1) ? -1.0 : 1.0;
        sb += sgn_b * jn * inv_int(kb);
      }
      if (n == 1) j1 = jn;
    } else {
      const int k = n / 2;
      norm += 2.0 * jn;
      sy0 += ((k & 1) ? -1.0 : 1.0) * jn * inv_int(k);
    }
    const double jm1 = (double)n * tx * jn - jn1;
    jn1 = jn;
    jn = jm1;
  }
  // jn = J_0 (scaled)
  norm += jn;
  const double inv = 1.0 / norm;
  const double J0 = jn * inv, J1 = j1 * inv;
  const double lgg = log(0.5 * x) + kEulerGamma;
  const double Y0 = (2.0 / kPi) * (lgg * J0 - 2.0 * sy0 * inv);
  const double Y1 = (2.0 / kPi) * (-J0 / x + lgg * J1 + (sa - sb) * inv);
  h0.re = J0;
  h0.im = Y0;
  const double hx = 0.5 * kPi * x;
  g1m.re = -hx * Y1 - 1.0;
  g1m.im = hx * J1;
}

// Hankel asymptotic expansion, x >= 20
__host__ __device__ inline void hankel_asymptotic(double x, cplx& h0, cplx& g1m) {
  const double e = 1.0 / (8.0 * x);
  double p0 = 1.0, q0 = 0.0, p1 = 1.0, q1 = 0.0;
  double t0 = 1.0, t1 = 1.0;
#pragma unroll
  for (int k = 1; k <= 22; ++k) {
    const double o = (double)(2 * k - 1);
    // ((nu^2 - o^2) / k) folds to a constant once the loop is unrolled
    t0 *= ((0.0 - o * o) / (double)k) * e;
    t1 *= ((4.0 - o * o) / (double)k) * e;
    // P = sum_{k even} (-1)^{k/2} t_k ; Q = sum_{k odd} (-1)^{(k-1)/2} t_k
    const int r = k & 3;
    const double s = (r == 0 || r == 1) ? 1.0 : -1.0;
    if (k & 1) {
      q0 += s * t0;
      q1 += s * t1;
    } else {
      p0 += s * t0;
      p1 += s * t1;
    }
  }
  double sx, cx;
  sincos(x, &sx, &cx);
  const double amp = sqrt(2.0 / (kPi * x));
  // chi0 = x - pi/4, chi1 = x - 3 pi/4
  const cplx e0 = {kSqrtHalf * (cx + sx), kSqrtHalf * (sx - cx)};
  const cplx e1 = {kSqrtHalf * (sx - cx), -kSqrtHalf * (sx + cx)};
  const cplx a0 = cmul({p0, q0}, e0);
  const cplx a1 = cmul({p1, q1}, e1);
  h0 = {amp * a0.re, amp * a0.im};
  const double hx = 0.5 * kPi * x * amp;
  // (i pi x/2) H1 - 1
  g1m = {-hx * a1.im - 1.0, hx * a1.re};
}

__device__ inline void hankel_pieces(double x, cplx& h0, cplx& g1m) {
  if (x <= kHankelSeriesMax)
    hankel_series(x, h0, g1m);
  else if (x < kHankelAsympMin)
    hankel_miller(x, h0, g1m);
  else
    hankel_asymptotic(x, h0, g1m);
}

// The four layer-potential kernels for target normal n, source normal n',
// dv = t - s, r2 = |dv|^2, nd = n.dv, npd = n'.dv, nn = n.n' (Sec. 2.2,
// eq. (19)-(20)); from dH0/dx = -H1 and H1' = H0 - H1/x:
//   S  = (i/4) H0
//   D  = npd/(2 pi r2) g1,  D* = -nd/(2 pi r2) g1,  g1 = 1 + g1m
//   T  = [ nn g1/(2 pi) + nd npd/r2 ((i/4) x^2 H0 - g1/pi) ] / r2
struct Kern4 {
  cplx S, D, Ds, T;
};

__device__ inline Kern4 lp_kernels(double k, double r2, double nd, double npd, double nn) {
  const double r = sqrt(r2);
  const double x = k * r;
  cplx h0, gm;
  hankel_pieces(x, h0, gm);
  const cplx g1 = {1.0 + gm.re, gm.im};
  const double ir2 = 1.0 / r2;
  const double c2 = 1.0 / (2.0 * kPi);
  Kern4 o;
  o.S = {-0.25 * h0.im, 0.25 * h0.re};
  const double fd = npd * c2 * ir2, fs = -nd * c2 * ir2;
  o.D = {fd * g1.re, fd * g1.im};
  o.Ds = {fs * g1.re, fs * g1.im};
  const double x2 = x * x;
  const double c = nd * npd * ir2;
  // (i/4) x^2 H0 - g1/pi
  const double wr = -0.25 * x2 * h0.im - g1.re * (1.0 / kPi);
  const double wi = 0.25 * x2 * h0.re - g1.im * (1.0 / kPi);
  o.T = {(nn * c2 * g1.re + c * wr) * ir2, (nn * c2 * g1.im + c * wi) * ir2};
  return o;
}

// Wavenumber derivatives dK/dk of the four kernels at fixed geometry, from
// dH0(kr)/dk = -r H1 and d[x H1(x)]/dx = x H0 (so that d g1/dk = (i pi/2) k r^2 H0):
//   dS/dk  = -g1/(2 pi k)
//   dD/dk  = npd (i/4) k H0,   dD*/dk = -nd (i/4) k H0
//   dT/dk  = nn (i/4) k H0 - nd npd k g1/(2 pi r^2)
// The k-independent singular parts of S, D, D*, T drop out: dS/dk is bounded
// and dT/dk is log-singular, like the self-block difference kernels.
__device__ inline Kern4 lp_kernels_dk(double k, double r2, double nd, double npd, double nn) {
  const double r = sqrt(r2);
  cplx h0, gm;
  hankel_pieces(k * r, h0, gm);
  const cplx g1 = {1.0 + gm.re, gm.im};
  const cplx ikh0 = {-0.25 * k * h0.im, 0.25 * k * h0.re};  // (i/4) k H0
  const double c2k = 1.0 / (2.0 * kPi * k);
  Kern4 o;
  o.S = {-g1.re * c2k, -g1.im * c2k};
  o.D = {npd * ikh0.re, npd * ikh0.im};
  o.Ds = {-nd * ikh0.re, -nd * ikh0.im};
  const double f = nd * npd * k / (2.0 * kPi * r2);
  o.T = {nn * ikh0.re - f * g1.re, nn * ikh0.im - f * g1.im};
  return o;
}

// K^{ka} - K^{kb} with the k-independent singular parts cancelled exactly.
__device__ inline Kern4 lp_kernels_diff(double ka, double kb, double r2, double nd,
                                                 double npd, double nn) {
  const double r = sqrt(r2);
  const double xa = ka * r, xb = kb * r;
  cplx ha, ga, hb, gb;
  hankel_pieces(xa, ha, ga);
  hankel_pieces(xb, hb, gb);
  const cplx dg = {ga.re - gb.re, ga.im - gb.im};
  const double ir2 = 1.0 / r2;
  const double c2 = 1.0 / (2.0 * kPi);
  Kern4 o;
  o.S = {-0.25 * (ha.im - hb.im), 0.25 * (ha.re - hb.re)};
  const double fd = npd * c2 * ir2, fs = -nd * c2 * ir2;
  o.D = {fd * dg.re, fd * dg.im};
  o.Ds = {fs * dg.re, fs * dg.im};
  const double c = nd * npd * ir2;
  const double dx2r = xa * xa * ha.re - xb * xb * hb.re;
  const double dx2i = xa * xa * ha.im - xb * xb * hb.im;
  const double wr = -0.25 * dx2i - dg.re * (1.0 / kPi);
  const double wi = 0.25 * dx2r - dg.im * (1.0 / kPi);
  o.T = {(nn * c2 * dg.re + c * wr) * ir2, (nn * c2 * dg.im + c * wi) * ir2};
  return o;
}

}  // namespace mlh
