// devmath.h -- device math for the non-LTE library (gfx950).
//
// * Voigt function H(a,u) = Re w(u + i a) by the rational series of
//   J.A.C. Weideman, SIAM J. Numer. Anal. 31 (1994) 1497:
//     w(z) = 2 p(Z) / (L - i z)^2 + pi^{-1/2} / (L - i z),  Z = (L + i z)/(L - i z),
//   with p a polynomial of degree N-1 whose coefficients are cosine sums of
//   exp(-t^2)(L^2 + t^2) at t = L tan(theta/2); L = sqrt(N / sqrt 2).  N = 32, in FP64
//   (relative error <= 2e-8 for a >= 1e-4).  FP32 sweeps evaluate the same FP64 series for |u| < 5 and
//   the asymptotic series of w(z) in FP32 beyond; where the damping is small (a < 0.04)
//   they use instead, inside |u| < 5, the Taylor series of w about the real axis (below).
//   Lines without damping use exp(-u^2) directly.  Both series have real coefficients and are summed with Goertzel's
//   second-order recurrence rather than complex Horner steps.
// * Linear short-characteristics coefficients (Kunasz & Auer 1988):
//     e = exp(-x), Psi_o = 1 - (1-e)/x, Psi_u = (1-e)/x - e,
//   with their Taylor series below a precision-dependent threshold.
// * Exponential integral E1 for the fixed bound-free rates: power series for x <= 1,
//   the Laplace continued fraction e^{-x} / (x + 1 - 1^2/(x + 3 - 2^2/(x + 5 - ...)))
//   evaluated bottom-up above.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "voigt_coef.h"

namespace nlte {

constexpr double kH = 6.62607015e-27;      // erg s
constexpr double kC = 2.99792458e10;       // cm/s
constexpr double kKB = 1.380649e-16;       // erg/K
constexpr double kME = 9.1093837015e-28;   // g
constexpr double kAMU = 1.66053906660e-24; // g
constexpr double kPI = 3.14159265358979323846;
constexpr double kSQRTPI = 1.77245385090551602730;
constexpr double kINVSQRTPI = 0.56418958354775628695;

// Small-damping FP32 Voigt function: H(a,u) = Re w(u + i a) = sum_n Re[(i a)^n w^(n)(u) / n!].
// From w' = -2 z w + 2i/sqrt(pi), w^(n) = P_n w + Q_n i/sqrt(pi) with P_{n+1} = P_n' - 2z P_n,
// Q_{n+1} = Q_n' + 2 P_n (P_0 = 1, Q_0 = 0), and on the real axis w(u) = exp(-u^2) +
// (2i/sqrt(pi)) F(u) (Dawson's F).  With G = 1 - 2uF (= F') and t = u^2, the terms up to a^4
// sum to
//   H = exp(-t) [1 + a^2 + a^4/2 - 2(a^2 + a^4) t + (2/3) a^4 t^2]
//       + pi^{-1/2} [(2/3) a^3 - (2a + 2a^3 - (4/3) a^3 t) G],
// whose truncation error is below 2e-7 relative for a < 0.04 and |u| < 5.  G is evaluated
// from a table of cubics on 80 intervals of width 1/16 in |u| (Hermite interpolation of G
// and G' = -2F - 2uG, which the host takes from an accurate integration of F' = 1 - 2uF).
constexpr int kDawIntervals = 80;
constexpr float kDawInvStep = 16.0f;
constexpr float kVoigtSmallA = 0.04f;
// Per interval the cubic's coefficients (c0, c1, c2, c3) in the local coordinate s in [0, 1).
__constant__ float4 c_dawg[kDawIntervals];

// Weideman coefficients, highest power first (voigt_coef.h, compiled-in literals).
template <typename R> struct VoigtTraits;
// Each coefficient passes through an empty volatile asm where it is used, so the compiler
// writes it into a scalar register pair right there (two s_mov) instead of hoisting all
// 64 dwords out of the frequency loop, where they would crowd out the loop's other scalars.
template <> struct VoigtTraits<double> {
    static constexpr int N = kVoigtNd;
    __device__ static double coef(int i) {
        double c = kVoigtCoefD[i];
        asm volatile("" : "+s"(c));
        return c;
    }
    __device__ static constexpr double L() { return kVoigtLd; }
};

__device__ inline float dev_rcp(float x) { return __builtin_amdgcn_rcpf(x); }   // v_rcp_f32, 1 ulp

__device__ inline double dev_rcp(double x) { return 1.0 / x; }
__device__ inline float dev_exp_neg(float x) { return __expf(-x); }
__device__ inline double dev_exp_neg(double x) { return exp(-x); }

// An opacity counts as zero (a transparent point) below 1e-30 cm^-1 in FP32 and
// 1e-150 cm^-1 in FP64: any segment through such a point has optical depth below
// ~1e-20, while the reciprocal of the opacity must stay finite (v_rcp_f32 flushes
// denormal inputs, and the FP64 reciprocal expansion overflows long before the
// smallest normal double).
__device__ inline bool opaque(float chi) { return chi >= 1e-30f; }
__device__ inline bool opaque(double chi) { return chi >= 1e-150; }

// Source function S = (eta_c + e phi) / (chi_c + k phi) and rchi = 1/chi.  Where the
// opacity is negligible (the profile underflowed far out in a wing), S is the limit
// of that ratio as phi -> 0: eta_c/chi_c with a background, else
// the line source function e/k, else 0; rchi is 0 there (the point's own weight
// w phi~ vanishes with phi, but a segment from an opaque upwind point still sees S).
template <typename R>
__device__ inline R source_limit(R chic, R etac, R kpl, R el) {
    if (opaque(chic)) return etac * dev_rcp(chic);
    if (opaque(kpl)) return el * dev_rcp(kpl);
    return R(0);
}

template <typename R>
__device__ inline R source_fn(R chi, R chic, R etac, R kpl, R el, R phi, R& rchi) {
    if (opaque(chi)) {
        rchi = dev_rcp(chi);
        return fma(el, phi, etac) * rchi;
    }
    rchi = R(0);
    return source_limit(chic, etac, kpl, el);
}

// H(a, u) for a >= 0 (Weideman rational series).  p has real coefficients, so p(Z) is
// evaluated by the second-order recurrence for a real polynomial at a complex point
// (Knuth, TAOCP vol. 2, sect. 4.6.4): with r = 2 Re Z and s = |Z|^2,
//   b_j = c_j + r b_{j-1} - s b_{j-2},   p(Z) = Z b_{N-2} + (c_{N-1} - s b_{N-3}),
// two FMAs per coefficient instead of the four of a complex Horner step.
template <typename R>
__device__ inline R voigt_H(R a, R u) {
    using T = VoigtTraits<R>;
    const R L = T::L();
    const R lpa = L + a, lma = L - a;
    const R u2 = u * u;
    const R rden = dev_rcp(fma(lpa, lpa, u2));
    const R zr = fma(lma, lpa, -u2) * rden;
    const R zi = (R(2) * L * u) * rden;
    const R r = R(2) * zr;
    const R sq = fma(lma, lma, u2) * rden;   // |Z|^2
    R b1 = T::coef(0), b2 = R(0);
#pragma unroll
    for (int j = 1; j < T::N - 1; ++j) {
        const R b0 = fma(r, b1, fma(-sq, b2, T::coef(j)));
        b2 = b1;
        b1 = b0;
    }
    const R pr = fma(zr, b1, fma(-sq, b2, T::coef(T::N - 1)));
    const R pi = zi * b1;
    const R rr = lpa * rden, ri = u * rden;
    const R r2r = fma(rr, rr, -ri * ri), r2i = R(2) * rr * ri;
    return fma(R(2), fma(pr, r2r, -pi * r2i), rr * R(kINVSQRTPI));
}

// Wings, |u| >= 5, FP32: w(z) = exp(-z^2) + (2i/sqrt(pi)) F(z) with Dawson's F, whose
// asymptotic series gives (i/sqrt(pi)) z^-1 sum_n (2n-1)!!/2^n z^-2n (10 terms).  Near
// the real axis (a < |u|/2) the real part of exp(-z^2), exp(a^2 - u^2) cos(2au) <=
// e^{-18.75}, is added; further from it that term is cancelled by the continuation of
// F (Stokes phenomenon) and the series alone is w.  Relative error <= 5e-7 for
// 1e-5 <= a <= 500.  The sum is a real polynomial in 1/z^2, evaluated with the same
// recurrence as above.
__device__ inline float voigt_H_wing(float a, float u) {
    const float rd = __builtin_amdgcn_rcpf(fmaf(u, u, a * a));
    const float rr = u * rd, ri = -a * rd;                       // 1/z
    const float r2r = fmaf(rr, rr, -ri * ri), r2i = 2.0f * rr * ri;  // 1/z^2
    const float r = 2.0f * r2r, sq = rd * rd;                    // 2 Re z^-2, |z^-2|^2
    const float cf[10] = {1.0f, 0.5f, 0.75f, 1.875f, 6.5625f, 29.53125f, 162.421875f, 1055.7421875f,
                          7918.06640625f, 67303.564453125f};
    float b1 = cf[9], b2 = 0.0f;
#pragma unroll
    for (int n = 8; n >= 1; --n) {
        const float b0 = fmaf(r, b1, fmaf(-sq, b2, cf[n]));
        b2 = b1;
        b1 = b0;
    }
    const float sr = fmaf(r2r, b1, fmaf(-sq, b2, cf[0]));
    const float si = r2i * b1;
    const float ti = fmaf(rr, si, ri * sr);
    const float gauss = (a < 0.5f * fabsf(u)) ? __expf(fmaf(a, a, -u * u)) * __cosf(2.0f * a * u) : 0.0f;
    return fmaf(-ti, float(kINVSQRTPI), gauss);
}

// Small-damping series above, a < 0.04 and |u| < 5; `tab` holds c_dawg (in LDS or global
// memory).  Relative error below 1e-6: the rounding of t = u^2 before the exponential
// (~5e-7), the table (<= 3.5e-7) and the truncation (<= 2e-7).
__device__ inline float voigt_H_small(float a, float u, const float4* tab) {
    // the coefficients below are recomputed per call rather than held in registers across a
    // caller's frequency loop (the empty asm makes `a` look loop-variant)
    asm volatile("" : "+v"(a));
    const float t = u * u;
    const float x = fabsf(u) * kDawInvStep;
    const int i = min(int(x), kDawIntervals - 1);
    const float sx = x - float(i);
    const float4 c = tab[i];
    const float G = fmaf(fmaf(fmaf(c.w, sx, c.z), sx, c.y), sx, c.x);
    const float a2 = a * a, a3 = a2 * a, a4 = a2 * a2;
    const float ev = fmaf(fmaf(a4 * (2.0f / 3.0f), t, -2.0f * (a2 + a4)), t, 1.0f + a2 + 0.5f * a4);
    // odd part A0 (1 + 2tG) + B0 G with A0 = 2a^3/(3 sqrt(pi)), B0 = -2(a + a^3)/sqrt(pi)
    const float A0 = a3 * float(2.0 / 3.0 * kINVSQRTPI);
    const float od = fmaf(G, -2.0f * float(kINVSQRTPI) * (a + a3), A0 * fmaf(t + t, G, 1.0f));
    return fmaf(__expf(-t), ev, od);
}

// Profile shape: Gaussian for undamped lines, Voigt otherwise.  `tab` is the
// small-damping table of the FP32 evaluation (unused in FP64).
template <typename R>
__device__ inline R profile_H(R a, R u, bool gauss, const float4*) {
    if (gauss) return dev_exp_neg(u * u);
    return voigt_H<R>(a, u);
}
// FP32 sweeps: the Weideman series loses relative accuracy to cancellation in FP32
// where H is small (|u| ~ 3-5, a << 1), so inside |u| < 5 it uses the small-damping
// series for a < 0.04 and otherwise runs in FP64 with the FP64 coefficients (relative
// error ~2e-8 before the final rounding to FP32); the wings use the FP32 asymptotic form.
template <>
__device__ inline float profile_H<float>(float a, float u, bool gauss, const float4* tab) {
    if (gauss) return __expf(-u * u);
    if (fabsf(u) >= 5.0f) return voigt_H_wing(a, u);
    if (a < kVoigtSmallA) return voigt_H_small(a, u, tab);
    // The FP64 series' per-voxel set-up is redone here instead of being kept in registers
    // across the frequency loop: the empty asm makes its input look loop-variant.
    float al = a;
    asm volatile("" : "+v"(al));
    return float(voigt_H<double>(double(al), double(u)));
}

// Linear short-characteristics segment coefficients; omp = 1 - Psi_o is returned
// separately because forming it from Psi_o cancels when Psi_o -> 1 (large dtau).
__device__ inline void sc_coeffs(float x, float& ex, float& pu, float& po, float& omp) {
    ex = __expf(-x);
    if (x < 0.5f) {
        // sum_{n=1}^{8} (-1)^{n+1} x^n/(n+1)!  and  sum (-1)^{n+1} n x^n/(n+1)!
        po = x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f - x * (1.0f / 720.0f
                - x * (1.0f / 5040.0f - x * (1.0f / 40320.0f - x * (1.0f / 362880.0f))))))));
        pu = x * (0.5f - x * (2.0f / 6.0f - x * (3.0f / 24.0f - x * (4.0f / 120.0f - x * (5.0f / 720.0f
                - x * (6.0f / 5040.0f - x * (7.0f / 40320.0f - x * (8.0f / 362880.0f))))))));
        omp = 1.0f - po;
    } else {
        const float r = (1.0f - ex) * __builtin_amdgcn_rcpf(x);
        po = 1.0f - r;
        pu = r - ex;
        omp = r;
    }
}

__device__ inline void sc_coeffs(double x, double& ex, double& pu, double& po, double& omp) {
    ex = exp(-x);
    if (x < 0.1) {
        double so = 0.0, su = 0.0;
        // Horner over n = 12 .. 1 of (-1)^{n+1} x^n/(n+1)! (and n times that)
        double fact[13];
        fact[0] = 1.0;
#pragma unroll
        for (int n = 1; n <= 12; ++n) fact[n] = fact[n - 1] * (n + 1);   // (n+1)!
#pragma unroll
        for (int n = 12; n >= 1; --n) {
            const double sg = (n & 1) ? 1.0 : -1.0;
            so = so * x + sg / fact[n];
            su = su * x + sg * n / fact[n];
        }
        po = so * x;
        pu = su * x;
        omp = 1.0 - po;
    } else {
        const double r = -expm1(-x) / x;
        po = 1.0 - r;
        pu = r - ex;
        omp = r;
    }
}

// Planck function B_nu(T), FP64.
__device__ inline double planck(double nu, double T) {
    return (2.0 * kH * nu * nu * nu / (kC * kC)) / expm1(kH * nu / (kKB * T));
}

// Exponential integral E1(x), x > 0, FP64.
__device__ inline double expint_e1(double x) {
    if (x <= 1.0) {
        // E1(x) = -gamma - ln x - sum_{k>=1} (-x)^k / (k k!)
        double term = 1.0, sum = 0.0;
        for (int k = 1; k < 40; ++k) {
            term *= -x / k;
            const double add = term / k;
            sum += add;
            if (fabs(add) < 1e-18 * fabs(sum)) break;
        }
        return -0.57721566490153286061 - log(x) - sum;
    }
    // continued fraction, evaluated from a fixed depth upward
    const int depth = x > 30.0 ? 12 : (x > 5.0 ? 40 : 120);
    double t = x + 2.0 * depth + 1.0;
    for (int k = depth; k >= 1; --k) t = x + 2.0 * k - 1.0 - double(k) * double(k) / t;
    return exp(-x) / t;
}

// sum_{k>=1} E1(k x): integral of dt / (t (e^t - 1)) from x to infinity.
__device__ inline double bf_planck_integral(double x) {
    double total = 0.0;
    for (int k = 1; k < 100000; ++k) {
        const double t = expint_e1(k * x);
        total += t;
        if (t <= 1e-17 * total) break;
    }
    return total;
}

}  // namespace nlte
