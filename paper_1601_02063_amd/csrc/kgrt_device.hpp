// kgrt_device.hpp -- FP64 device mathematics of the Kerr ray tracer (gfx950).
//
// One ray lives in one lane; everything here is a register-only __device__
// function. E = -1 for every traced ray (the initial-condition step divides
// the rates by sqrt(E^2) and takes the negative root of Eq. (7)), so E and
// E^2 never appear as variables. M = 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kgrt {

// CGS constants (CODATA 2018) and the IAU 2015 nominal solar GM.
constexpr double kC = 2.99792458e10;         // speed of light
constexpr double kQe = 4.80320471e-10;       // elementary charge (esu)
constexpr double kMe = 9.1093837015e-28;     // electron mass
constexpr double kMp = 1.67262192369e-24;    // proton mass
constexpr double kH = 6.62607015e-27;        // Planck constant
constexpr double kKb = 1.380649e-16;         // Boltzmann constant
constexpr double kGMsun = 1.3271244e26;      // solar GM
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kSinFloor = 1e-8;           // pole clamp of section 2.1

// Status bits (mirror include/kgrt.h).
constexpr int32_t ST_CAPTURED = 1, ST_ESCAPED = 2, ST_CROSSED = 4, ST_DISK_HIT = 8, ST_MAXSTEPS = 16,
                  ST_UNDERFLOW = 32, ST_NONFINITE = 64, ST_REFINE_UNCONVERGED = 256, ST_SPOT_HIT = 512;

// Cash & Karp (1990) embedded 5(4) tableau: stage weights a_ij, fifth-order
// weights b_i and differences d_i = b_i - b*_i of the embedded fourth order.
namespace ck {
constexpr double a21 = 1.0 / 5.0;
constexpr double a31 = 3.0 / 40.0, a32 = 9.0 / 40.0;
constexpr double a41 = 3.0 / 10.0, a42 = -9.0 / 10.0, a43 = 6.0 / 5.0;
constexpr double a51 = -11.0 / 54.0, a52 = 5.0 / 2.0, a53 = -70.0 / 27.0, a54 = 35.0 / 27.0;
constexpr double a61 = 1631.0 / 55296.0, a62 = 175.0 / 512.0, a63 = 575.0 / 13824.0,
                 a64 = 44275.0 / 110592.0, a65 = 253.0 / 4096.0;
constexpr double b1 = 37.0 / 378.0, b3 = 250.0 / 621.0, b4 = 125.0 / 594.0, b6 = 512.0 / 1771.0;
constexpr double d1 = b1 - 2825.0 / 27648.0, d3 = b3 - 18575.0 / 48384.0, d4 = b4 - 13525.0 / 55296.0,
                 d5 = -277.0 / 14336.0, d6 = b6 - 1.0 / 4.0;
}  // namespace ck

struct State {
    double r, th, ph, t, pr, pth;
};

// max(s, floor) in one instruction (a NaN s gives the floor; the state's own
// finiteness test catches NaN states)
__device__ __forceinline__ double clamp_sin(double s) { return fmax(s, kSinFloor); }

// sin and cos of one argument for |x| < 2^20 (polar angles stay near [0, pi]).
// Cody-Waite reduction by a three-part pi/2 (fused multiply-adds keep the
// reduced argument exact to about 2^-100), then polynomials on |r| <= pi/4 and
// the quadrant rotation: sin r = r + r^3 S(r^2), cos r = 1 - r^2/2 + r^4 C(r^2)
// with S, C of degree 5 fitted near-minimax by csrc/gen_poly.py (their
// approximation error 0.18 and 0.011 ulp; the truncated Taylor series needs
// two more terms each for the same accuracy). About 1 ulp in all; much lighter
// than the general-argument library routine, whose large-argument path costs
// registers.
namespace trig {
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPio2Hi = 1.5707963267948966;      // 0x1.921fb54442d18p+0
constexpr double kPio2Mid = 6.123233995736766e-17;  // 0x1.1a62633145c07p-54
constexpr double kPio2Lo = -1.4973849048591698e-33; // -0x1.f1976b7ed8fbcp-110
// S and C, highest power of z = r^2 first
constexpr double kSinPoly[6] = {1.5918129294866608e-10, -2.5051131845003624e-08, 2.755731610255244e-06,
                                -0.00019841269836758574, 0.008333333333330948, -0.16666666666666666};
constexpr double kCosPoly[6] = {-1.1382632425521717e-11, 2.08761462684032e-09, -2.7557317271729793e-07,
                                2.480158729876569e-05, -0.0013888888888887398, 0.041666666666666664};
// e^r - 1 = r + r^2/2 + r^3 E(r) on |r| <= ln(2)/2 and atanh f = f + f^3 A(f^2)
// on |f| <= 3 - 2 sqrt(2), E and A from the same generator
constexpr double kExpm1Poly[10] = {2.091122972975856e-09,  2.5100375832561234e-08, 2.755728298405588e-07,
                                   2.7557268480310024e-06, 2.4801587317135164e-05, 0.00019841269863040545,
                                   0.0013888888888886554,  0.008333333333330065,   0.041666666666666664,
                                   0.16666666666666669};
constexpr double kAtanhPoly[7] = {0.07308224842521703, 0.07665860800278021, 0.09091444562630861, 0.1111110556739754,
                                  0.14285714312987743, 0.19999999999949752, 0.3333333333333335};
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
// 1/n! as a compile-time constant (a class-template constant forces constant evaluation)
template <int N>
struct InvFact {
    static constexpr double value = 1.0 / fact(N);
};
}  // namespace trig

__host__ __device__ __forceinline__ void sincos_bounded(double x, double* sp, double* cp) {
    using namespace trig;
    const double k = rint(x * kTwoOverPi);
    double r = fma(-k, kPio2Hi, x);
    r = fma(-k, kPio2Mid, r);
    r = fma(-k, kPio2Lo, r);
    const double z = r * r;
    double ps = kSinPoly[0], pc = kCosPoly[0];
#pragma unroll
    for (int i = 1; i < 6; ++i) {
        ps = fma(ps, z, kSinPoly[i]);
        pc = fma(pc, z, kCosPoly[i]);
    }
    const double sr = fma(r * z, ps, r);
    const double cr = fma(z, fma(z, pc, -0.5), 1.0);
    // quadrant rotation: swap for odd k, then the signs as bit flips of the high word
    const int q = (int)k;
    const double s1 = (q & 1) ? cr : sr;
    const double c1 = (q & 1) ? sr : cr;
    const uint64_t ssign = (uint64_t)(uint32_t)(q & 2) << 62, csign = (uint64_t)(uint32_t)((q + 1) & 2) << 62;
    *sp = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, s1) ^ ssign);
    *cp = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, c1) ^ csign);
}

// ---------------------------------------------------------------------------
// Light FP64 elementary functions for the per-step path. The general library
// versions carry wide-range and special-case machinery whose register cost
// would halve the kernel's occupancy; these cover the argument ranges that
// occur here, with ~1-3 ulp accuracy (checked on the host against a
// multiple-precision reference). All from textbook methods:
//   exp/expm1: Cody & Waite reduction x = k ln2 + r, |r| <= ln2/2, polynomial;
//   log: x = m 2^e with m in [sqrt(1/2), sqrt(2)), log m = 2 atanh((m-1)/(m+1)), polynomial;
//   (the polynomials: leading Taylor terms plus a near-minimax remainder, above);
//   x^(-1/n): single-precision seed 2^(-log2(x)/n) and two Newton steps
//             y <- y + y (1 - x y^n)/n in double (quadratic convergence);
//   1/x: hardware reciprocal seed and two Newton steps r <- r + r (1 - x r).
namespace fm {
constexpr double kLn2Hi = 0.6931471805599453;
constexpr double kLn2Lo = 2.3190468138462996e-17;
constexpr double kLog2e = 1.4426950408889634;
constexpr double kSqrtHalf = 0.7071067811865476;

__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// 1/x to about 2^-46 relative (one Newton step), for the step-size controller's
// error norm: it only decides acceptance against 1 and scales the next step.
__device__ __forceinline__ double rcp_coarse(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// e^r - 1 for |r| <= ln2/2.
__host__ __device__ __forceinline__ double expm1_reduced(double r) {
    double p = trig::kExpm1Poly[0];
#pragma unroll
    for (int i = 1; i < 10; ++i) p = fma(p, r, trig::kExpm1Poly[i]);
    p = fma(p, r, 0.5);
    return fma(r * r, p, r);
}

__host__ __device__ __forceinline__ double exp(double x) {
    if (x < -745.5) return 0.0;
    if (x > 709.8) return __builtin_huge_val();
    if (!(x == x)) return x;
    const double k = rint(x * kLog2e);
    double r = fma(-k, kLn2Hi, x);
    r = fma(-k, kLn2Lo, r);
    return ldexp(1.0 + expm1_reduced(r), (int)k);
}

__host__ __device__ __forceinline__ double expm1(double x) {
    if (fabs(x) <= 0.5 * kLn2Hi) return expm1_reduced(x);
    return fm::exp(x) - 1.0;
}

// a/b within an ulp: quotient from a reciprocal seed (two Newton steps on the
// device, the IEEE reciprocal on the host) and one residual correction.
__host__ __device__ __forceinline__ double div(double a, double b) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double r = rcp(b);
#else
    const double r = 1.0 / b;
#endif
    const double q = a * r;
    return fma(r, fma(-b, q, a), q);
}

// Natural logarithm for finite x > 0.
__host__ __device__ __forceinline__ double log(double x) {
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < kSqrtHalf) {
        m *= 2.0;
        e -= 1;
    }
    const double f = div(m - 1.0, m + 1.0);
    const double s = f * f;
    double p = trig::kAtanhPoly[0];
#pragma unroll
    for (int i = 1; i < 7; ++i) p = fma(p, s, trig::kAtanhPoly[i]);
    const double lm = fma(2.0 * f * s, p, 2.0 * f);  // 2 atanh(f)
    return fma((double)e, kLn2Hi, fma((double)e, kLn2Lo, lm));
}

// y^N by repeated squaring (4 multiplications for N = 12, 2 for 4, 3 for 5).
template <int N>
__device__ __forceinline__ double ipow(double y) {
    if constexpr (N == 1) {
        return y;
    } else if constexpr (N % 2 == 0) {
        const double h = ipow<N / 2>(y);
        return h * h;
    } else {
        return ipow<N - 1>(y) * y;
    }
}

// 1/sqrt(x) for positive normal x: hardware seed (relative error about 2^-23)
// and two Newton steps y <- y + y (1 - x y^2)/2.
__device__ __forceinline__ double rsqrt(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = fma(y * 0.5, fma(-x * y, y, 1.0), y);
    y = fma(y * 0.5, fma(-x * y, y, 1.0), y);
    return y;
}

// x^(-1/N) for 1e-30 <= x <= 1e30.
template <int N>
__device__ __forceinline__ double inv_root(double x) {
    if constexpr (N == 2) return rsqrt(x);
    const float xf = (float)x;
    double y = (double)__builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(xf) * (1.0f / N));
#pragma unroll
    for (int it = 0; it < 2; ++it) y = fma(y * (1.0 / N), fma(-x, ipow<N>(y), 1.0), y);
    return y;
}

// Step-size factors of the error controller: 0.9 errmax^(-1/4) on rejection
// (errmax > 1, result floored at 0.1 by the caller) and 0.9 errmax^(-1/5) on
// acceptance (1.89e-4 < errmax <= 1).
__device__ __forceinline__ double pow_m025(double x) {
    if (x > 1e8) return 0.0;  // 0.9 x^-1/4 < 0.1 there: the floor applies
    return inv_root<4>(x);
}
__device__ __forceinline__ double pow_m02(double x) { return inv_root<5>(x); }
}  // namespace fm

// Geodesic right-hand side, section 2.1 (photons, E = -1): r' and theta' from
// Eqs. (4)-(5), phi' Eq. (12), t' Eq. (9), p_theta' Eq. (15). For p_r' the
// form of Eq. (14) before the null condition replaces W^2/Delta is used,
//   p_r' = [2 r E W / Delta - (r - 1)(W^2/Delta^2 + p_r^2)] / Sigma,  W = (r^2+a^2)E - aL,
// equal to the printed form on the null cone; it keeps 2 Sigma H conserved,
// which the printed form does not on ingoing rays.
// With sin(theta) (clamped) and cos(theta) of y given.
// h f(y): the right-hand side scaled by the step size h (the Cash-Karp stages
// only ever use h k_i, so the scale is folded into the two common factors
// 1/(Sigma Delta) and 1/Sigma instead of multiplying every component).
__device__ __forceinline__ State rhs_sc(const State& y, double s, double c, double a, double a2, double L, double h) {
    const double r = y.r;
    const double r2a2 = r * r + a2;
    const double Sigma = r * r + a2 * c * c;
    const double Delta = r2a2 - 2.0 * r;
    // one reciprocal for both 1/(Sigma Delta) and 1/sin^2
    const double SD = Sigma * Delta, s2 = s * s;
    const double R = fm::rcp(SD * s2);
    const double iSD = R * s2;
    const double iD = Sigma * iSD;
    const double is2 = R * SD;
    const double hSD = h * iSD;     // h/(Sigma Delta)
    const double hS = Delta * hSD;  // h/Sigma
    const double W = -r2a2 - a * L;
    const double WiD = W * iD;
    State d;
    d.r = Delta * y.pr * hS;
    d.th = y.pth * hS;
    d.ph = (-2.0 * a * r + (Sigma - 2.0 * r) * L * is2) * hSD;
    d.t = -h - 2.0 * r * (r2a2 + a * L) * hSD;
    d.pr = (-2.0 * r * WiD - (r - 1.0) * (WiD * WiD + y.pr * y.pr)) * hS;
    d.pth = s * c * hS * (L * L * is2 * is2 - a2);
    return d;
}

__device__ __forceinline__ State rhs(const State& y, double a, double a2, double L, double h) {
    double s, c;
    sincos_bounded(y.th, &s, &c);
    return rhs_sc(y, clamp_sin(s), c, a, a2, L, h);
}

// y + sum(w_i k_i) componentwise (k_i already scaled by h), written out per field.
#define KGRT_STAGE(OUT, Y, EXPR_R, EXPR_TH, EXPR_PH, EXPR_T, EXPR_PR, EXPR_PTH)                                 \
    State OUT{(Y).r + (EXPR_R), (Y).th + (EXPR_TH), (Y).ph + (EXPR_PH), (Y).t + (EXPR_T), (Y).pr + (EXPR_PR), \
              (Y).pth + (EXPR_PTH)}

// One Cash-Karp step of size h from y with k1 = h f(y): fifth-order result in
// y5, embedded error estimate (y5 - y4) in err. Five RHS evaluations, each
// returning h f at its stage point.
__device__ __forceinline__ void cash_karp(const State& y, const State& k1, double h, double a, double a2, double L,
                                          State& y5, State& err) {
    using namespace ck;
#define S2(f) (a21 * k1.f)
    KGRT_STAGE(y2, y, S2(r), S2(th), S2(ph), S2(t), S2(pr), S2(pth));
#undef S2
    const State k2 = rhs(y2, a, a2, L, h);
#define S3(f) (a31 * k1.f + a32 * k2.f)
    KGRT_STAGE(y3, y, S3(r), S3(th), S3(ph), S3(t), S3(pr), S3(pth));
#undef S3
    const State k3 = rhs(y3, a, a2, L, h);
#define S4(f) (a41 * k1.f + a42 * k2.f + a43 * k3.f)
    KGRT_STAGE(y4, y, S4(r), S4(th), S4(ph), S4(t), S4(pr), S4(pth));
#undef S4
    const State k4 = rhs(y4, a, a2, L, h);
#define S5(f) (a51 * k1.f + a52 * k2.f + a53 * k3.f + a54 * k4.f)
    KGRT_STAGE(y5s, y, S5(r), S5(th), S5(ph), S5(t), S5(pr), S5(pth));
#undef S5
    const State k5 = rhs(y5s, a, a2, L, h);
#define S6(f) (a61 * k1.f + a62 * k2.f + a63 * k3.f + a64 * k4.f + a65 * k5.f)
    KGRT_STAGE(y6s, y, S6(r), S6(th), S6(ph), S6(t), S6(pr), S6(pth));
#undef S6
    const State k6 = rhs(y6s, a, a2, L, h);
#define B5(f) (b1 * k1.f + b3 * k3.f + b4 * k4.f + b6 * k6.f)
    KGRT_STAGE(yo, y, B5(r), B5(th), B5(ph), B5(t), B5(pr), B5(pth));
    y5 = yo;
#undef B5
#define DE(f) (d1 * k1.f + d3 * k3.f + d4 * k4.f + d5 * k5.f + d6 * k6.f)
    err = State{DE(r), DE(th), DE(ph), DE(t), DE(pr), DE(pth)};
#undef DE
}

__device__ __forceinline__ bool finite6(const State& y) {
    return isfinite(y.r) && isfinite(y.th) && isfinite(y.ph) && isfinite(y.t) && isfinite(y.pr) && isfinite(y.pth);
}

// Prograde marginally stable orbit, Bardeen, Press & Teukolsky (1972).
__device__ __host__ inline double isco_radius(double a) {
    const double z1 = 1.0 + cbrt(1.0 - a * a) * (cbrt(1.0 + a) + cbrt(1.0 - a));
    const double z2 = sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

// ------------------------------------------------------------ ray start

// Pixel -> start state, section 2.2: Eqs. (18)-(19) image plane -> Cartesian,
// Eqs. (20)-(22) Cartesian -> Boyer-Lindquist, Eqs. (24)-(26) rates of a ray
// along the line of sight, Eq. (7) energy (negative root, rates scaled so
// E = -1), Eq. (8) L_z, Eqs. (4)-(5) covariant momenta. Returns false when
// the start point is unusable (E^2 <= 0 or non-finite values).
__device__ __forceinline__ bool start_ray(double a, double a2, double r_obs, double sqrt_ro2a2, double sin_i,
                                          double cos_i, double sin_p, double cos_p, double phi_obs, double x,
                                          double y, State& st, double& L) {
    const double D = sqrt_ro2a2 * sin_i - y * cos_i;
    const double xp = D * cos_p - x * sin_p;
    const double yp = D * sin_p + x * cos_p;
    const double zp = r_obs * cos_i + y * sin_i;
    const double w = xp * xp + yp * yp + zp * zp - a2;
    const double r = sqrt((w + sqrt(w * w + 4.0 * a2 * zp * zp)) / 2.0);
    const double th = acos(zp / r);
    const double ph = atan2(yp, xp);
    const double R = sqrt(r * r + a2);
    double sP, cP;
    sincos_bounded(ph - phi_obs, &sP, &cP);
    double sn, cs;
    sincos_bounded(th, &sn, &cs);
    const double Sigma = r * r + a2 * cs * cs;
    double rdot = -(r * R * sn * sin_i * cP + R * R * cs * cos_i) / Sigma;
    double thdot = (r * sn * cos_i - R * cs * sin_i * cP) / Sigma;
    double phdot = sin_i * sP / (R * sn);
    const double Delta = r * r - 2.0 * r + a2;
    const double E2 = ((Sigma - 2.0 * r) / (Sigma * Delta)) * (Sigma * rdot * rdot + Sigma * Delta * thdot * thdot) +
                      Delta * phdot * phdot * sn * sn;
    bool ok = (E2 > 0.0) && isfinite(E2);
    const double inv = 1.0 / sqrt(E2);
    rdot *= inv;
    thdot *= inv;
    phdot *= inv;
    L = (Sigma * Delta * phdot + 2.0 * a * r) * sn * sn / (Sigma - 2.0 * r);
    st = State{r, th, ph, 0.0, Sigma * rdot / Delta, Sigma * thdot};
    return ok && finite6(st) && isfinite(L);
}

// Redshift g = nu_obs/nu_emit (Eq. (2)) of an emitter on a circular Keplerian
// orbit, Omega = 1/(r^3/2 + a) in Boyer-Lindquist r at any theta, u^r = u^theta = 0,
// seen by an observer at rest at infinity; the zero-angular-momentum
// observer replaces it where u.u = -1 has no solution. xi = L_z/E.
// With sin(theta) (clamped) and cos(theta) given.
// Returns g and sets ig = 1/g.
__device__ __forceinline__ double redshift_sc(double r, double s, double c, double a, double a2, double xi,
                                              double& ig) {
    const double s2 = s * s;
    const double Sigma = r * r + a2 * c * c;
    const double iS = fm::rcp(Sigma);
    const double gtt = -(1.0 - 2.0 * r * iS);
    const double gtp = -2.0 * a * r * s2 * iS;
    const double gpp = (r * r + a2 + 2.0 * a2 * r * s2 * iS) * s2;
    double Om = fm::rcp(fma(r * r, fm::rsqrt(r), a));  // 1/(r^3/2 + a)
    double arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    if (!(arg > 0.0)) {
        Om = -gtp * fm::rcp(gpp);
        arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    }
    // g = 1/(u^t (1 - xi Omega)) with u^t = arg^-1/2
    ig = (1.0 - xi * Om) * fm::rsqrt(arg);
    return fm::rcp(ig);
}

// As redshift_sc for matter moving with a given angular velocity Om0 (the hot
// spot of section 4.4 moves rigidly with its centre; a simulation snapshot
// gives the plasma's own Omega), the zero-angular-momentum observer where that
// motion is not timelike. Returns g and sets ig = 1/g.
__device__ __forceinline__ double redshift_omega_sc(double r, double s, double c, double a, double a2, double xi,
                                                    double Om0, double& ig) {
    const double s2 = s * s;
    const double Sigma = r * r + a2 * c * c;
    const double iS = fm::rcp(Sigma);
    const double gtt = -(1.0 - 2.0 * r * iS);
    const double gtp = -2.0 * a * r * s2 * iS;
    const double gpp = (r * r + a2 + 2.0 * a2 * r * s2 * iS) * s2;
    double Om = Om0;
    double arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    if (!(arg > 0.0)) {
        Om = -gtp * fm::rcp(gpp);
        arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    }
    ig = (1.0 - xi * Om) * fm::rsqrt(arg);
    return fm::rcp(ig);
}

__device__ __forceinline__ double redshift_omega(double r, double s, double c, double a, double a2, double xi,
                                                 double Om0) {
    double ig;
    return redshift_omega_sc(r, s, c, a, a2, xi, Om0, ig);
}

__device__ __forceinline__ double redshift(double r, double th, double a, double a2, double xi) {
    double s, c, ig;
    sincos_bounded(th, &s, &c);
    return redshift_sc(r, clamp_sin(s), c, a, a2, xi, ig);
}

// Modified Bessel function K_2(x), x > 0, to ~1e-15 relative.
//  x <= 2: the ascending series of Abramowitz & Stegun 9.6.11 for n = 2,
//     K_2 = 2/x^2 - 1/2 + q sum_k c_k q^k [B_k - gamma - ln(x/2)],  q = x^2/4,
//     c_k = 1/(k! (k+2)!), B_k = (H_k + H_{k+2})/2 (H the harmonic numbers),
//     summed as two polynomials in q (13 terms: c_12 q^12 < 1e-20 for q <= 1);
//  x > 2: K_2 = f(t) e^-x / sqrt(x) with f(t) = sqrt(x) e^x K_2(x), t = 2/x,
//     a smooth function on (0, 1] evaluated from its Chebyshev expansion in
//     s = 2t - 1 (Clenshaw's recurrence; coefficients by csrc/gen_k2_cheb.py).
// Inlined: out of line, the call made the integrator save and restore the
// uniform values it keeps in SGPRs around every call (measured 1-2% slower
// than inline once the kernel no longer spilled; in an earlier build that still
// spilled, inlining had raised the spills instead).
namespace k2 {
constexpr double harm(int n) { return n == 0 ? 0.0 : harm(n - 1) + 1.0 / n; }
template <int K> struct C { static constexpr double value = 1.0 / (trig::fact(K) * trig::fact(K + 2)); };
template <int K> struct CB {
    static constexpr double value = C<K>::value * 0.5 * (harm(K) + harm(K + 2));
};
// max relative error of the expansion on t in (0, 1]: 3.53e-17
constexpr double kCheb[23] = {
    1.9262890227982927,
    6.9995586038264909e-1,
    2.6170713479740811e-2,
    -7.5018244642171226e-4,
    5.3674324702843297e-5,
    -5.5565569992929136e-6,
    7.1755728106304028e-7,
    -1.0803493404324407e-7,
    1.8257625536999556e-8,
    -3.3812091171936075e-9,
    6.7503021694118435e-10,
    -1.4356710508630012e-10,
    3.2240349844618053e-11,
    -7.5919911324572731e-12,
    1.8643740164153105e-12,
    -4.7532395845036968e-13,
    1.2534874890086944e-13,
    -3.4086052776469779e-14,
    9.5326307419863909e-15,
    -2.735364562022107e-15,
    8.03195174582688e-16,
    -2.3917930684419428e-16,
    6.6717415083862169e-17,
};
}  // namespace k2

// lnh = ln(x/2), which the caller has from the logarithm it already takes;
// ix = 1/x, which the caller also has without a division.
__device__ inline double bessel_k2(double x, double ix, double lnh) {
    if (x <= 2.0) {
        const double q = 0.25 * x * x;
        const double lg = lnh + kEulerGamma;
        double pb = k2::CB<12>::value, pc = k2::C<12>::value;
#define KGRT_K2_TERM(K)                      \
    pb = fma(pb, q, k2::CB<K>::value);       \
    pc = fma(pc, q, k2::C<K>::value);
        KGRT_K2_TERM(11) KGRT_K2_TERM(10) KGRT_K2_TERM(9) KGRT_K2_TERM(8) KGRT_K2_TERM(7) KGRT_K2_TERM(6)
        KGRT_K2_TERM(5) KGRT_K2_TERM(4) KGRT_K2_TERM(3) KGRT_K2_TERM(2) KGRT_K2_TERM(1) KGRT_K2_TERM(0)
#undef KGRT_K2_TERM
        return fma(q, fma(-lg, pc, pb), fma(2.0 * ix, ix, -0.5));  // 1/(2q) = 2/x^2
    }
    const double s = fma(4.0, ix, -1.0);
    const double s2 = 2.0 * s;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int j = 22; j >= 1; --j) {
        const double b0 = fma(s2, b1, k2::kCheb[j] - b2);
        b2 = b1;
        b1 = b0;
    }
    const double f = fma(s, b1, k2::kCheb[0] - b2);
    return f * fm::exp(-x) * fm::inv_root<2>(x);
}

// Torus and emission parameters in the form the kernels use.
struct TorusParams {
    double n0, inv_rnorm, n_index, inv_2h2, T0, T_index, eps_B, rg, r_emit_max;
    // products of constants, set on the host: B^2 = cB n_e / r, Theta_e = cTheta T_e/T0 = 1/(cInvTheta T0/T_e),
    // nu_c = cNu B Theta_e^2, so 1/nu_c^2 = 1/(cNuC n_e (T_e/T0)^4 / r) with cNuC = cB cNu^2 cTheta^4,
    // j prefactor = cJ n_e / K_2(1/Theta_e), ln(1/(2 Theta_e)) = T_index ln(r/r_norm) + cLnHalfInvTheta,
    // h/(k T_e) = cH T0/T_e, 1/B_nu = cBnu expm1(h nu/(k T_e)) / nu^3
    double cB, cTheta, cInvTheta, cLnHalfInvTheta, cNu, cNuC, cJ, cH, cBnu;
};

// Emission and absorption per unit affine parameter at (r, theta), redshift g,
// observed frequency nu: a_lam = r_g alpha_0(nu/g)/g and e_lam = r_g g^2 j_0(nu/g)
// (Eqs. (30)-(31)), with j_0 the thermal-synchrotron emissivity of Eqs. (37)-(39)
// divided by 4 pi (Eq. (37) is angle-integrated) and alpha_0 = j_0/B_nu(T_e)
// (Kirchhoff's law, section 4.5). Frequency-independent plasma quantities are
// computed once per point by torus_plasma().
struct Plasma {
    double ne, Te, inv_nu_c, jpref, hkT;  // jpref = n e^2/(sqrt(3) c K_2(1/Theta_e)), hkT = h/(k T_e)
    bool emits;
};

// cth = cos(theta).
__device__ inline Plasma torus_plasma(const TorusParams& P, double r, double cth, double r_cap) {
    Plasma q;
    q.emits = (r > r_cap) && !(r > P.r_emit_max);
    if (!q.emits) {
        q.ne = q.Te = q.inv_nu_c = q.jpref = q.hkT = 0.0;
        return q;
    }
    const double lx = fm::log(r * P.inv_rnorm);
    q.ne = P.n0 * fm::exp(-P.n_index * lx - cth * cth * P.inv_2h2);  // z^2/r^2 = cos^2(theta)
    const double eT = fm::exp(-P.T_index * lx);                       // T_e/T0
    const double ieT = fm::rcp(eT);
    q.Te = P.T0 * eT;
    const double eT2 = eT * eT;
    q.inv_nu_c = fm::rsqrt(P.cNuC * q.ne * (eT2 * eT2) * fm::rcp(r));  // 1/(cNu B Theta_e^2)
    // K_2 at x = 1/Theta_e: 1/x = Theta_e = cTheta T_e/T0
    q.jpref = q.ne * P.cJ * fm::rcp(bessel_k2(ieT * P.cInvTheta, P.cTheta * eT, fma(P.T_index, lx, P.cLnHalfInvTheta)));
    q.hkT = P.cH * ieT;
    return q;
}

// ig = 1/g; inv_nu = 1/nu.
__device__ inline void torus_coeffs(const Plasma& q, const TorusParams& P, double g, double ig, double nu,
                                    double inv_nu, double& a_lam, double& e_lam) {
    if (!q.emits) {
        a_lam = 0.0;
        e_lam = 0.0;
        return;
    }
    const double nu0 = nu * ig;
    const double xm = nu0 * q.inv_nu_c;
    double j = 0.0;
    if (xm < 1e9) {  // beyond, exp(-1.8899 x^1/3) underflows to zero
        // w = x^(-1/12): x^(-1/6) = w^2, x^(-1/4) = w^3, x^(-1/2) = w^6, x^(1/3) = x w^8
        const double w = fm::inv_root<12>(fmax(xm, 1e-30));
        const double w2 = w * w, w3 = w2 * w, w6 = w3 * w3, w8 = w6 * w2;
        const double Mx = 4.0505 * w2 * (1.0 + 0.40 * w3 + 0.5316 * w6) * fm::exp(-1.8899 * (xm * w8));  // Eq. (38)
        j = nu0 * q.jpref * Mx;                                                                          // Eq. (37)/(4 pi)
    }
    double alpha = 0.0;
    if (j > 0.0) {
        const double inv_nu0 = g * inv_nu;
        alpha = j * fm::expm1(nu0 * q.hkT) * P.cBnu * (inv_nu0 * inv_nu0 * inv_nu0);  // j / B_nu(T_e)
    }
    a_lam = P.rg * alpha * ig;
    e_lam = P.rg * g * g * j;
}

// A plasma snapshot of the kind GRMHD simulations write out (section 6), in the
// form the integrator reads it: nodes[(i nth + j) nph + k] = (ln n_e, ln T_e,
// ln B, Omega) at ln r_i = ln r_min + i dlnr, theta_j = j pi/(nth - 1),
// phi_k = 2 pi k/nph (periodic). One node is one 16-byte load.
struct GridParams {
    const float4* nodes;
    int32_t nr, nth, nph, pad;
    double r_min, r_max, ln_rmin;
    double u1_scale;    // (nr - 1)/(ln r_max - ln r_min)
    double u2_scale;    // (nth - 1)/pi
    double u3_scale;    // nph/(2 pi)
    double inv_nph;     // 1/nph
    double ln_theta1;   // ln(k_B/(m_e c^2)): ln Theta_e = ln T_e + ln_theta1
    double inv_cnu;     // 1/cNu: 1/nu_c = Theta_e^-2 B^-1/cNu (nu_c as for the torus)
    double h_mec2;      // h/(m_e c^2): h/(k_B T_e) = h_mec2/Theta_e
};

// The snapshot at (r, theta, phi): trilinear interpolation in (ln r, theta, phi)
// of the node values (theta clamped to [0, pi], phi periodic). No plasma at or
// inside the capture radius nor outside [r_min, r_max]: returns false and
// leaves v alone. Cell indices are clamped into the grid, so every load stays
// inside the nr nth nph nodes whatever r, theta and phi are.
__device__ inline bool grid_sample(const GridParams& G, double r, double th, double ph, double r_cap, double v[4]) {
    if (!(r > r_cap) || !(r >= G.r_min) || !(r <= G.r_max)) return false;
    const double u3 = ph * G.u3_scale;
    if (!(fabs(u3) < 1e15)) return false;  // a non-finite or absurd azimuth: no sample
    const double u1 = (fm::log(r) - G.ln_rmin) * G.u1_scale;
    const double u2 = fmin(fmax(th * G.u2_scale, 0.0), (double)(G.nth - 1));
    const int i0 = min(max((int)floor(u1), 0), G.nr - 2);
    const int j0 = min(max((int)floor(u2), 0), G.nth - 2);
    const double k0f = floor(u3);
    const double w1 = u1 - i0, w2 = u2 - j0, w3 = u3 - k0f;
    int k0 = (int)(k0f - (double)G.nph * floor(k0f * G.inv_nph));  // k0f mod nph
    if (k0 >= G.nph) k0 -= G.nph;
    if (k0 < 0) k0 += G.nph;
    k0 = min(max(k0, 0), G.nph - 1);
    const int k1 = (k0 + 1 == G.nph) ? 0 : k0 + 1;
    const int64_t row0 = ((int64_t)i0 * G.nth + j0) * G.nph;  // (i0, j0); +nph: j0 + 1; +nth nph: i0 + 1
    const int64_t sj = G.nph, si = (int64_t)G.nth * G.nph;
    const float4* __restrict__ n = G.nodes;
    const float4 c000 = n[row0 + k0], c001 = n[row0 + k1];
    const float4 c010 = n[row0 + sj + k0], c011 = n[row0 + sj + k1];
    const float4 c100 = n[row0 + si + k0], c101 = n[row0 + si + k1];
    const float4 c110 = n[row0 + si + sj + k0], c111 = n[row0 + si + sj + k1];
    const double wk0 = 1.0 - w3, wj0 = 1.0 - w2, wi0 = 1.0 - w1;
#define KGRT_TRILERP(q)                                                                                    \
    {                                                                                                       \
        const double e00 = wk0 * (double)c000.q + w3 * (double)c001.q;                                      \
        const double e01 = wk0 * (double)c010.q + w3 * (double)c011.q;                                      \
        const double e10 = wk0 * (double)c100.q + w3 * (double)c101.q;                                      \
        const double e11 = wk0 * (double)c110.q + w3 * (double)c111.q;                                      \
        v[q##_i] = wi0 * (wj0 * e00 + w2 * e01) + w1 * (wj0 * e10 + w2 * e11);                              \
    }
    constexpr int x_i = 0, y_i = 1, z_i = 2, w_i = 3;
    KGRT_TRILERP(x) KGRT_TRILERP(y) KGRT_TRILERP(z) KGRT_TRILERP(w)
#undef KGRT_TRILERP
    return true;
}

// Frequency-independent synchrotron quantities (as torus_plasma) from the sampled
// ln n_e, ln T_e, ln B: Theta_e = k_B T_e/(m_e c^2), K_2 at 1/Theta_e,
// 1/nu_c = 1/(cNu B Theta_e^2), h/(k_B T_e). cJ is the torus's emissivity prefactor.
__device__ inline Plasma grid_plasma(const GridParams& G, double cJ, const double v[4]) {
    Plasma q;
    q.emits = true;
    q.ne = fm::exp(v[0]);
    const double lnth = v[1] + G.ln_theta1;  // ln Theta_e
    const double th = fm::exp(lnth);         // Theta_e
    const double x = fm::rcp(th);            // 1/Theta_e
    q.Te = 0.0;                              // not used by the coefficients
    q.inv_nu_c = x * x * fm::exp(-v[2]) * G.inv_cnu;
    q.jpref = q.ne * cJ * fm::rcp(bessel_k2(x, th, -lnth - 0.69314718055994531));  // ln(x/2)
    q.hkT = G.h_mec2 * x;
    return q;
}

}  // namespace kgrt
