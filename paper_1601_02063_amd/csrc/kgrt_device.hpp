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
                  ST_UNDERFLOW = 32, ST_NONFINITE = 64, ST_REFINE_UNCONVERGED = 256;

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

__device__ __forceinline__ double clamp_sin(double s) { return (s < kSinFloor) ? kSinFloor : s; }

// Geodesic right-hand side, section 2.1 (photons, E = -1): r' and theta' from
// Eqs. (4)-(5), phi' Eq. (12), t' Eq. (9), p_theta' Eq. (15). For p_r' the
// form of Eq. (14) before the null condition replaces W^2/Delta is used,
//   p_r' = [2 r E W / Delta - (r - 1)(W^2/Delta^2 + p_r^2)] / Sigma,  W = (r^2+a^2)E - aL,
// equal to the printed form on the null cone; it keeps 2 Sigma H conserved,
// which the printed form does not on ingoing rays.
__device__ __forceinline__ State rhs(const State& y, double a, double a2, double L) {
    double s, c;
    sincos(y.th, &s, &c);
    s = clamp_sin(s);
    const double r = y.r;
    const double r2a2 = r * r + a2;
    const double Sigma = r * r + a2 * c * c;
    const double Delta = r2a2 - 2.0 * r;
    const double iS = 1.0 / Sigma;
    const double iD = 1.0 / Delta;
    const double is2 = 1.0 / (s * s);
    const double iSD = iS * iD;
    const double W = -r2a2 - a * L;
    const double WiD = W * iD;
    State d;
    d.r = Delta * y.pr * iS;
    d.th = y.pth * iS;
    d.ph = (-2.0 * a * r + (Sigma - 2.0 * r) * L * is2) * iSD;
    d.t = -1.0 - 2.0 * r * (r2a2 + a * L) * iSD;
    d.pr = (-2.0 * r * WiD - (r - 1.0) * (WiD * WiD + y.pr * y.pr)) * iS;
    d.pth = s * c * iS * (L * L * is2 * is2 - a2);
    return d;
}

__device__ __forceinline__ State axpy(const State& y, double h, const State& k) {
    return State{y.r + h * k.r, y.th + h * k.th, y.ph + h * k.ph, y.t + h * k.t, y.pr + h * k.pr, y.pth + h * k.pth};
}

// y + h * sum(w_i k_i) componentwise, written out per field.
#define KGRT_STAGE(OUT, Y, H, EXPR_R, EXPR_TH, EXPR_PH, EXPR_T, EXPR_PR, EXPR_PTH) \
    State OUT{(Y).r + (H) * (EXPR_R), (Y).th + (H) * (EXPR_TH), (Y).ph + (H) * (EXPR_PH), (Y).t + (H) * (EXPR_T), \
              (Y).pr + (H) * (EXPR_PR), (Y).pth + (H) * (EXPR_PTH)}

// One Cash-Karp step of size h from y with k1 = f(y): fifth-order result in
// y5, embedded error estimate (y5 - y4) in err. Five RHS evaluations.
__device__ __forceinline__ void cash_karp(const State& y, const State& k1, double h, double a, double a2, double L,
                                          State& y5, State& err) {
    using namespace ck;
#define S2(f) (a21 * k1.f)
    KGRT_STAGE(y2, y, h, S2(r), S2(th), S2(ph), S2(t), S2(pr), S2(pth));
#undef S2
    const State k2 = rhs(y2, a, a2, L);
#define S3(f) (a31 * k1.f + a32 * k2.f)
    KGRT_STAGE(y3, y, h, S3(r), S3(th), S3(ph), S3(t), S3(pr), S3(pth));
#undef S3
    const State k3 = rhs(y3, a, a2, L);
#define S4(f) (a41 * k1.f + a42 * k2.f + a43 * k3.f)
    KGRT_STAGE(y4, y, h, S4(r), S4(th), S4(ph), S4(t), S4(pr), S4(pth));
#undef S4
    const State k4 = rhs(y4, a, a2, L);
#define S5(f) (a51 * k1.f + a52 * k2.f + a53 * k3.f + a54 * k4.f)
    KGRT_STAGE(y5s, y, h, S5(r), S5(th), S5(ph), S5(t), S5(pr), S5(pth));
#undef S5
    const State k5 = rhs(y5s, a, a2, L);
#define S6(f) (a61 * k1.f + a62 * k2.f + a63 * k3.f + a64 * k4.f + a65 * k5.f)
    KGRT_STAGE(y6s, y, h, S6(r), S6(th), S6(ph), S6(t), S6(pr), S6(pth));
#undef S6
    const State k6 = rhs(y6s, a, a2, L);
#define B5(f) (b1 * k1.f + b3 * k3.f + b4 * k4.f + b6 * k6.f)
    y5 = State{y.r + h * B5(r), y.th + h * B5(th), y.ph + h * B5(ph), y.t + h * B5(t), y.pr + h * B5(pr),
               y.pth + h * B5(pth)};
#undef B5
#define DE(f) (h * (d1 * k1.f + d3 * k3.f + d4 * k4.f + d5 * k5.f + d6 * k6.f))
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

// Redshift g = nu_obs/nu_emit (Eq. (2)) of an emitter on a circular Keplerian
// orbit, Omega = 1/(r^3/2 + a) in Boyer-Lindquist r at any theta, u^r = u^theta = 0,
// seen by an observer at rest at infinity; the zero-angular-momentum
// observer replaces it where u.u = -1 has no solution. xi = L_z/E.
__device__ __forceinline__ double redshift(double r, double th, double a, double a2, double xi) {
    double s, c;
    sincos(th, &s, &c);
    s = clamp_sin(s);
    const double s2 = s * s;
    const double Sigma = r * r + a2 * c * c;
    const double iS = 1.0 / Sigma;
    const double gtt = -(1.0 - 2.0 * r * iS);
    const double gtp = -2.0 * a * r * s2 * iS;
    const double gpp = (r * r + a2 + 2.0 * a2 * r * s2 * iS) * s2;
    double Om = 1.0 / (r * sqrt(r) + a);
    double arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    if (!(arg > 0.0)) {
        Om = -gtp / gpp;
        arg = -(gtt + 2.0 * Om * gtp + Om * Om * gpp);
    }
    // 1/(u^t (1 - xi Omega)) with u^t = arg^-1/2
    return sqrt(arg) / (1.0 - xi * Om);
}

// Modified Bessel function K_2(x), x > 0, to ~1e-15 relative.
//  x <= 2: the ascending series of Abramowitz & Stegun 9.6.11 for n = 2,
//     K_2 = 2/x^2 - 1/2 + (x^2/4) sum_k t_k [ (H_k + H_{k+2})/2 - gamma - ln(x/2) ],
//     t_k = (x^2/4)^k / (k! (k+2)!), H_k the harmonic numbers;
//  x > 2: the trapezoidal rule on K_2(x) = int_0^inf exp(-x cosh u) cosh(2u) du
//     (A&S 9.6.24), step min(0.2, 0.6/sqrt(x)), which converges geometrically
//     for this entire, doubly-exponentially decaying integrand; cosh(k h) - 1
//     and cosh(2 k h) come from a Chebyshev-type recurrence.
__device__ inline double bessel_k2(double x) {
    if (x <= 2.0) {
        const double q = 0.25 * x * x;
        const double lg = log(0.5 * x) + kEulerGamma;
        double t = 0.5, hk = 0.0, hk2 = 1.5;
        double sum = t * (0.5 * (hk + hk2) - lg);
#pragma unroll
        for (int k = 1; k < 16; ++k) {
            t *= q / (k * (k + 2.0));
            hk += 1.0 / k;
            hk2 += 1.0 / (k + 2.0);
            sum += t * (0.5 * (hk + hk2) - lg);
        }
        return 2.0 / (x * x) - 0.5 + q * sum;
    }
    const double h = fmin(0.2, 0.6 / sqrt(x));
    const double sh = sinh(0.5 * h);
    const double e1 = 2.0 * sh * sh;  // cosh(h) - 1
    const double c1 = 1.0 + e1;
    double em1 = 0.0, e = e1, sum = 0.5;
    for (int k = 1; k < 64; ++k) {
        const double term = exp(-x * e) * (1.0 + 4.0 * e + 2.0 * e * e);
        sum += term;
        if (term < 1e-18 * sum) break;
        const double en = 2.0 * c1 * e - em1 + 2.0 * e1;
        em1 = e;
        e = en;
    }
    return h * exp(-x) * sum;
}

// Torus and emission parameters in the form the kernels use.
struct TorusParams {
    double n0, inv_rnorm, n_index, inv_2h2, T0, T_index, eps_B, rg, r_emit_max;
};

// Emission and absorption per unit affine parameter at (r, theta), redshift g,
// observed frequency nu: a_lam = r_g alpha_0(nu/g)/g and e_lam = r_g g^2 j_0(nu/g)
// (Eqs. (30)-(31)), with j_0 the thermal-synchrotron emissivity of Eqs. (37)-(39)
// divided by 4 pi (Eq. (37) is angle-integrated) and alpha_0 = j_0/B_nu(T_e)
// (Kirchhoff's law, section 4.5). Frequency-independent plasma quantities are
// computed once per point by torus_plasma().
struct Plasma {
    double ne, Te, nu_c, jpref, hkT;  // jpref = n e^2/(sqrt(3) c K_2(1/Theta_e)), hkT = h/(k T_e)
    bool emits;
};

__device__ inline Plasma torus_plasma(const TorusParams& P, double r, double th, double r_cap) {
    Plasma q;
    q.emits = (r > r_cap) && !(r > P.r_emit_max);
    if (!q.emits) {
        q.ne = q.Te = q.nu_c = q.jpref = q.hkT = 0.0;
        return q;
    }
    const double z = r * cos(th);
    const double lx = log(r * P.inv_rnorm);
    q.ne = P.n0 * exp(-P.n_index * lx - z * z * P.inv_2h2 / (r * r));
    q.Te = P.T0 * exp(-P.T_index * lx);
    const double B = sqrt(8.0 * kPi * P.eps_B * q.ne * kMp * kC * kC / (6.0 * r));
    const double theta_e = kKb * q.Te / (kMe * kC * kC);
    q.nu_c = 3.0 * kQe * B / (4.0 * kPi * kMe * kC) * theta_e * theta_e;
    q.jpref = q.ne * kQe * kQe / (1.7320508075688772 * kC * bessel_k2(1.0 / theta_e));
    q.hkT = kH / (kKb * q.Te);
    return q;
}

__device__ inline void torus_coeffs(const Plasma& q, const TorusParams& P, double g, double nu, double& a_lam,
                                    double& e_lam) {
    if (!q.emits) {
        a_lam = 0.0;
        e_lam = 0.0;
        return;
    }
    const double nu0 = nu / g;
    const double xm = nu0 / q.nu_c;
    const double x3 = cbrt(xm);
    const double x2 = sqrt(xm);
    const double x4 = sqrt(x2);
    const double x6 = sqrt(x3);
    const double Mx = 4.0505 / x6 * (1.0 + 0.40 / x4 + 0.5316 / x2) * exp(-1.8899 * x3);  // Eq. (38)
    const double j = nu0 * q.jpref * Mx;                                               // Eq. (37)/(4 pi)
    double alpha = 0.0;
    if (j > 0.0) {
        const double bnu = 2.0 * kH * nu0 * nu0 * nu0 / (kC * kC) / expm1(nu0 * q.hkT);
        alpha = j / bnu;
    }
    a_lam = P.rg * alpha / g;
    e_lam = P.rg * g * g * j;
}

}  // namespace kgrt
