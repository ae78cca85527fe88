// Modified Bessel functions I0, I1, K0, K1 of a real argument x > 0 for the
// screened kernels in 2D (Appendix A.2: G = -K0(r s)/(2 pi), its derivatives
// through K1; a ball's mean-value factor 1/I0(s R) and gradient factor
// s/I1(s R)).
//
// FP32: the rational approximations of Abramowitz & Stegun 9.8.1-9.8.8
// (relative error below about 5e-7 over the whole range).
// FP64: power series for I0, I1 up to x = 25 and their asymptotic expansion
// above; for K0, K1 the series of Abramowitz & Stegun 9.6.11 (digamma
// coefficients) up to x = 2 and above it the trapezoid rule on
// K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt, which converges
// geometrically for this analytic, rapidly decaying integrand (relative
// error below 1e-14 against reference values over [1e-8, 700]).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bvc {

__device__ __forceinline__ float as_poly(const float* c, int n, float t) {
  float r = c[n - 1];
  for (int i = n - 2; i >= 0; --i) r = fmaf(r, t, c[i]);
  return r;
}

// I0(x), FP32 (A&S 9.8.1, 9.8.2)
__device__ __forceinline__ float bessel_i0f(float x) {
  if (x <= 3.75f) {
    const float c[7] = {1.0f, 3.5156229f, 3.0899424f, 1.2067492f, 0.2659732f, 0.0360768f, 0.0045813f};
    const float t = x * (1.0f / 3.75f);
    return as_poly(c, 7, t * t);
  }
  const float c[9] = {0.39894228f, 0.01328592f, 0.00225319f, -0.00157565f, 0.00916281f,
                      -0.02057706f, 0.02635537f, -0.01647633f, 0.00392377f};
  return expf(x) * rsqrtf(x) * as_poly(c, 9, 3.75f / x);
}

// I1(x), FP32 (A&S 9.8.3, 9.8.4)
__device__ __forceinline__ float bessel_i1f(float x) {
  if (x <= 3.75f) {
    const float c[7] = {0.5f, 0.87890594f, 0.51498869f, 0.15084934f, 0.02658733f, 0.00301532f, 0.00032411f};
    const float t = x * (1.0f / 3.75f);
    return x * as_poly(c, 7, t * t);
  }
  const float c[9] = {0.39894228f, -0.03988024f, -0.00362018f, 0.00163801f, -0.01031555f,
                      0.02282967f, -0.02895312f, 0.01787654f, -0.00420059f};
  return expf(x) * rsqrtf(x) * as_poly(c, 9, 3.75f / x);
}

// K0(x), K1(x), FP32 (A&S 9.8.5-9.8.8)
__device__ __forceinline__ void bessel_k01f(float x, float& k0, float& k1) {
  if (x <= 2.0f) {
    const float c0[7] = {-0.57721566f, 0.42278420f, 0.23069756f, 0.03488590f, 0.00262698f, 0.00010750f, 0.00000740f};
    const float c1[7] = {1.0f, 0.15443144f, -0.67278579f, -0.18156897f, -0.01919402f, -0.00110404f, -0.00004686f};
    const float h = 0.5f * x, t = h * h;
    const float L = logf(h);
    k0 = fmaf(-L, bessel_i0f(x), as_poly(c0, 7, t));
    k1 = fmaf(L, bessel_i1f(x), as_poly(c1, 7, t) / x);
    return;
  }
  const float c0[7] = {1.25331414f, -0.07832358f, 0.02189568f, -0.01062446f, 0.00587872f, -0.00251540f, 0.00053208f};
  const float c1[7] = {1.25331414f, 0.23498619f, -0.03655620f, 0.01504268f, -0.00780353f, 0.00325614f, -0.00068245f};
  const float t = 2.0f / x;
  const float f = expf(-x) * rsqrtf(x);
  k0 = f * as_poly(c0, 7, t);
  k1 = f * as_poly(c1, 7, t);
}

// I0(x), I1(x), FP64
__device__ inline void bessel_i01(double x, double& i0, double& i1) {
  if (x <= 25.0) {
    const double q = 0.25 * x * x;
    double t0 = 1.0, s0 = 1.0, t1 = 1.0, s1 = 1.0;
    for (int k = 1; k < 200; ++k) {
      t0 *= q / ((double)k * k);
      t1 *= q / ((double)k * (k + 1));
      s0 += t0;
      s1 += t1;
      if (t0 < 1e-17 * s0 && t1 < 1e-17 * s1) break;
    }
    i0 = s0;
    i1 = 0.5 * x * s1;
    return;
  }
  // e^x / sqrt(2 pi x) * sum_k (-1)^k prod_{j<=k} (4 nu^2 - (2j-1)^2) / (k! (8x)^k)
  const double f = exp(x) / sqrt(2.0 * 3.141592653589793 * x);
  double out[2];
  for (int nu = 0; nu < 2; ++nu) {
    const double mu = 4.0 * nu * nu;
    double term = 1.0, s = 1.0;
    for (int k = 1; k < 30; ++k) {
      term *= -(mu - (2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k * x);
      s += term;
      if (fabs(term) < 1e-17 * fabs(s)) break;
    }
    out[nu] = f * s;
  }
  i0 = out[0];
  i1 = out[1];
}

// K0(x), K1(x), FP64
__device__ inline void bessel_k01(double x, double& k0, double& k1) {
  const double eg = 0.5772156649015329;  // Euler's constant
  if (x <= 2.0) {
    double i0, i1;
    bessel_i01(x, i0, i1);
    const double q = 0.25 * x * x, L = log(0.5 * x);
    // K0 = -(L + g) I0 + sum_{k>=1} q^k/(k!)^2 H_k
    // K1 = 1/x + L I1 - (x/4) sum_{k>=0} (psi(k+1) + psi(k+2)) q^k/(k!(k+1)!),  psi(k+1) = H_k - g
    double t0 = 1.0, t1 = 1.0, H = 0.0, s0 = 0.0, s1 = 1.0 - 2.0 * eg;
    for (int k = 1; k < 60; ++k) {
      t0 *= q / ((double)k * k);
      t1 *= q / ((double)k * (k + 1));
      H += 1.0 / k;
      s0 += t0 * H;
      s1 += t1 * (2.0 * H + 1.0 / (k + 1) - 2.0 * eg);
      if (t0 < 1e-18 && t1 < 1e-18) break;
    }
    k0 = fma(-(L + eg), i0, s0);
    k1 = 1.0 / x + L * i1 - 0.25 * x * s1;
    return;
  }
  // trapezoid on [0, t_max], x (cosh t_max - 1) = 40, with cosh t - 1 = 2 sinh^2(t/2)
  const double tmax = acosh(1.0 + 40.0 / x);
  const double h0 = 0.5 * fmin(0.5, 1.2 / sqrt(x));
  const int n = (int)ceil(tmax / h0);
  const double h = tmax / n;
  double s0 = 0.5, s1 = 0.5;
  for (int j = 1; j <= n; ++j) {
    const double t = j * h;
    const double sh = sinh(0.5 * t);
    const double e = exp(-2.0 * x * sh * sh);
    s0 += e;
    s1 += e * cosh(t);
  }
  const double f = h * exp(-x);
  k0 = s0 * f;
  k1 = s1 * f;
}

template <typename T>
__device__ __forceinline__ T bessel_i0(T x) {
  if constexpr (sizeof(T) == 4) {
    return bessel_i0f(x);
  } else {
    double i0, i1;
    bessel_i01(x, i0, i1);
    return i0;
  }
}

template <typename T>
__device__ __forceinline__ void bessel_k01t(T x, T& k0, T& k1) {
  if constexpr (sizeof(T) == 4) {
    bessel_k01f(x, k0, k1);
  } else {
    bessel_k01(x, k0, k1);
  }
}

}  // namespace bvc
