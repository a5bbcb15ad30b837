// kgrt_mino.hpp -- the first equatorial crossing radius of a Kerr photon from
// its constants of motion, Newton-polished from an estimate (gfx950, FP64).
//
// With Carter's Mino time (d tau = d lambda / Sigma) the radial and polar
// motions of a null geodesic separate: dr/dtau = +-sqrt(R(r)),
// dmu/dtau = +-sqrt(M(mu)) with mu = cos(theta) and, for E = 1 and the
// constants xi = L_z/E, eta = Q/E^2 of Eqs. (8) and (13),
//   R(r)  = (r^2 + a^2 - a xi)^2 - Delta (eta + (xi - a)^2),
//   M(mu) = eta + (a^2 - eta - xi^2) mu^2 - a^2 mu^4.
// The ray reaches the equator first after the Mino time G_mu the polar motion
// needs from mu_obs to 0 (through its polar turning point if it starts moving
// away from the equator), and the crossing radius r_c is where the radial
// motion has used the same Mino time. Both integrals are evaluated in FP64:
//   * G_mu in closed form, mu = mu_+ sin(psi): int_0^mu = sin(Psi)/sqrt(B) *
//     R_F(cos^2 Psi, 1 + (A/B) sin^2 Psi, 1), A = a^2 mu_+^2, B = eta/mu_+^2
//     (Carlson's symmetric elliptic integral R_F, by his duplication method);
//   * the radial Mino time in u = 1/r, where u^4 R(1/u) = P(u) is a quartic
//     with P(0) = 1, by 32-point Gauss-Legendre quadrature; beyond the radial
//     turning point u_tp (the largest root of R, found by Newton's method from
//     above) the integrand's square-root singularity is removed by
//     u = u_tp - (u_tp - u_x) t^2 and deflating P by (u - u_tp).
// The crossing then solves J(u_c) = T on the leg the Mino times select
// (inbound before the turning point, outbound after it, or inbound to the
// horizon when there is none), by Newton's method in s = sqrt(u_tp - u)
// (or in u without a turning point), started from the estimate.
#pragma once

#include <hip/hip_runtime.h>

#include "kgrt_device.hpp"

namespace kgrt_mino {

// 1/sqrt(x), x > 0, to about an ulp: the hardware seed and two Newton steps (kgrt::fm::rsqrt)
__device__ __forceinline__ double rsq(double x) { return kgrt::fm::rsqrt(x); }

// 32-point Gauss-Legendre rule on [0, 1]: the 16 nodes below 1/2 (the others
// are 1 - t) and their weights, from csrc/gen_gauss_legendre.py (mpmath).
constexpr double kGlT[16] = {0.0013680690752592182, 0.0071942442273658323, 0.017618872206246785,
                             0.032546962031130155,  0.051839422116973938,  0.075316193133715015,
                             0.1027581020160288,    0.13390894062985516,   0.1684778665348924,
                             0.20614212137961884,   0.2465500455338853,    0.28932436193468233,
                             0.33406569885893618,   0.38035631887393146,   0.42776401920860175,
                             0.47584616715613084};
constexpr double kGlW[16] = {0.0035093050047350483, 0.0081371973654528353, 0.01269603265463103,
                             0.017136931456510717,  0.02141794901111334,   0.025499029631188088,
                             0.029342046739267774,  0.032911111388180923,  0.036172897054424253,
                             0.039096947893535153,  0.041655962113473378,  0.043826046502201906,
                             0.045586939347881942,  0.046922199540402283,  0.04781936003963743,
                             0.0482700442573639};

// Carlson's R_F(x, y, z) by duplication (Carlson 1995, Numer. Algorithms 10):
// iterate until the arguments agree to 1e-4, then the fifth-order series
// (truncation error below 1e-20 relative).
__device__ inline double carlson_rf(double x, double y, double z) {
    for (int it = 0; it < 30; ++it) {
        const double m = (x + y + z) * (1.0 / 3.0);
        if (fmax(fabs(x - m), fmax(fabs(y - m), fabs(z - m))) < 1e-4 * m) break;
        const double sx = sqrt(x), sy = sqrt(y), sz = sqrt(z);
        const double lam = sx * sy + sy * sz + sz * sx;
        x = 0.25 * (x + lam);
        y = 0.25 * (y + lam);
        z = 0.25 * (z + lam);
    }
    const double m = (x + y + z) * (1.0 / 3.0);
    const double X = 1.0 - x / m, Y = 1.0 - y / m, Z = 1.0 - z / m;
    const double E2 = X * Y - Z * Z, E3 = X * Y * Z;
    return (1.0 - E2 / 10.0 + E3 / 14.0 + E2 * E2 / 24.0 - 3.0 * E2 * E3 / 44.0) / sqrt(m);
}

// Polar Mino time from mu0 to the equator (eta > 0). toward: the ray starts
// moving toward the equator; otherwise it first reaches its turning point mu_+.
__device__ inline double polar_mino(double a, double xi, double eta, double mu0, bool toward) {
    const double b = a * a - eta - xi * xi;
    const double sd = sqrt(b * b + 4.0 * a * a * eta);
    // mu_+^2, the positive root of a^2 v^2 - b v - eta = 0, in the form without cancellation
    const double vp = (b <= 0.0) ? 2.0 * eta / (sd - b) : (b + sd) / (2.0 * a * a);
    const double A = a * a * vp, B = eta / vp, ib = 1.0 / sqrt(B), k = A / B;
    const double sp = sqrt(vp);
    auto part = [&](double mu) {  // int_0^mu dmu / sqrt(M)
        double s = fmin(fabs(mu) / sp, 1.0);
        const double c2 = fmax(1.0 - s * s, 0.0);
        return s * ib * carlson_rf(c2, 1.0 + k * s * s, 1.0);
    };
    const double i0 = part(mu0);
    return toward ? i0 : 2.0 * part(sp) - i0;
}

// P(u) = u^4 R(1/u) = k4 u^4 + k3 u^3 + k2 u^2 + 1
struct Quartic {
    double k4, k3, k2;
    __device__ double P(double u) const { return fma(fma(fma(k4, u, k3), u, k2), u * u, 1.0); }
};

// int_{ux}^{utp} du / sqrt(P(u)) with P = (u - utp) q3(u): u = utp - (utp - ux) t^2.
__device__ inline double j_tp(const Quartic& q, double utp, double ux) {
    const double b3 = q.k4, b2 = fma(utp, b3, q.k3), b1 = fma(utp, b2, q.k2), b0 = utp * b1;
    const double d = utp - ux;
    double acc = 0.0;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        const double ta = kGlT[k], tb = 1.0 - kGlT[k];
        const double ua = fma(-d * ta, ta, utp), ub = fma(-d * tb, tb, utp);
        const double qa = fma(fma(fma(b3, ua, b2), ua, b1), ua, b0);
        const double qb = fma(fma(fma(b3, ub, b2), ub, b1), ub, b0);
        acc = fma(kGlW[k], rsq(-qa) + rsq(-qb), acc);
    }
    return 2.0 * sqrt(d) * acc;
}

// dJ/ds at s = sqrt(utp - u): 2 / sqrt(-q3(u))
__device__ inline double dj_ds(const Quartic& q, double utp, double u) {
    const double b3 = q.k4, b2 = fma(utp, b3, q.k3), b1 = fma(utp, b2, q.k2), b0 = utp * b1;
    return 2.0 * rsq(-fma(fma(fma(b3, u, b2), u, b1), u, b0));
}

// int_{u0}^{u1} du / sqrt(P(u)) where P > 0 (no turning point).
__device__ inline double k_direct(const Quartic& q, double u0, double u1) {
    const double d = u1 - u0;
    double acc = 0.0;
#pragma unroll 4
    for (int k = 0; k < 16; ++k) {
        acc = fma(kGlW[k], rsq(q.P(fma(d, kGlT[k], u0))) + rsq(q.P(fma(d, 1.0 - kGlT[k], u0))), acc);
    }
    return d * acc;
}

// Largest real root of R(r) = r^4 + p r^2 + qq r + s above r_floor, or 0 if none:
// Newton's method from above all roots (Fujiwara's bound) in the convex region
// r^2 > -p/6, where it decreases monotonically to the largest root.
__device__ inline double largest_root(double p, double qq, double s, double r_floor) {
    auto R = [&](double r) { return fma(fma(r, r, p), r * r, fma(qq, r, s)); };
    auto dR = [&](double r) { return fma(4.0 * r * r, r, fma(2.0 * p, r, qq)); };
    const double ri = sqrt(fmax(-p / 6.0, 0.0));
    const double lo = fmax(ri, r_floor);
    if (R(lo) > 0.0 && dR(lo) >= 0.0) return 0.0;  // increasing and convex beyond: no root there
    double r = 2.0 * fmax(sqrt(fabs(p)), fmax(cbrt(fabs(qq)), sqrt(sqrt(fabs(0.5 * s)))));
    r = fmax(r, lo) + 1.0;
    for (int it = 0; it < 100; ++it) {
        const double d = dR(r);
        if (!(d > 0.0)) return 0.0;  // passed the minimum without a sign change: no root
        const double step = R(r) / d;
        r -= step;
        if (fabs(step) <= 1e-15 * r) break;
    }
    return (r > r_floor && R(r) <= 1e-12 * r * r * r * r) ? r : 0.0;
}

// The first equatorial crossing radius of the photon (E = 1 normalisation:
// xi = L_z/E, eta = Q/E^2), observed from r_obs, polar position mu0 = cos(theta)
// moving toward the equator (toward) or away from it, polished from r_guess.
// Returns 0 when the ray never reaches the equator outside r_cap, and -1 when
// the solution cannot be certified (no Newton step below 1e-7 relative within
// 8 steps, eta <= 0, guesses that land outside the leg), in which case the
// caller integrates the ray instead. Newton converges quadratically here, so a
// last step of 1e-7 leaves an error near 1e-14; a tighter stop (1e-13) sat at
// the quadrature's FP64 rounding and sent 2% of a thin-disk image's rays to
// the integrator for nothing.
__device__ inline double crossing_radius(double a, double xi, double eta, double r_obs, double mu0, bool toward,
                                         double r_cap, double r_guess) {
    if (!(eta > 0.0)) return -1.0;
    const double Gm = polar_mino(a, xi, eta, mu0, toward);
    const double al = a * a - a * xi, C = eta + (xi - a) * (xi - a);
    const Quartic q{al * al - a * a * C, 2.0 * C, 2.0 * al - C};
    const double uo = 1.0 / r_obs, ucap = 1.0 / r_cap;
    const double rtp = largest_root(a * a - xi * xi - eta, 2.0 * C, -a * a * eta, r_cap);
    if (rtp > 0.0) {
        const double utp = 1.0 / rtp;
        const double Jo = j_tp(q, utp, uo);
        // the leg is decided by comparing Mino times; too close a call is left to the integrator
        if (fabs(Gm - Jo) <= 1e-9 * Jo || fabs(Gm - 2.0 * Jo) <= 1e-9 * Jo) return -1.0;
        double T;
        if (Gm < Jo) {
            T = Jo - Gm;  // inbound leg
        } else if (Gm < 2.0 * Jo) {
            T = Gm - Jo;  // outbound leg, after the turning point
        } else {
            return 0.0;  // back out at the observer's radius before reaching the equator
        }
        if (!(r_guess > rtp)) r_guess = rtp * (1.0 + 1e-3);
        double s = sqrt(fmax(utp - 1.0 / r_guess, 0.0));
        const double smax = sqrt(utp - uo);
        for (int it = 0; it < 8; ++it) {
            const double u = fma(-s, s, utp);
            const double ds = (j_tp(q, utp, u) - T) / dj_ds(q, utp, u);
            s = fmin(fmax(s - ds, 0.0), smax);
            if (fabs(ds) <= 1e-7 * fmax(s, 1e-6)) return 1.0 / fma(-s, s, utp);
        }
        return -1.0;
    }
    // no turning point: inbound to the horizon
    const double Kcap = k_direct(q, uo, ucap);
    if (fabs(Gm - Kcap) <= 1e-9 * Kcap) return -1.0;
    if (!(Gm < Kcap)) return 0.0;  // captured before it reaches the equator
    double u = (r_guess > r_cap) ? 1.0 / r_guess : 0.5 * (uo + ucap);
    for (int it = 0; it < 8; ++it) {
        const double du = (k_direct(q, uo, u) - Gm) * sqrt(q.P(u));
        u = fmin(fmax(u - du, uo), ucap);
        if (fabs(du) <= 1e-7 * u) return 1.0 / u;
    }
    return -1.0;
}

}  // namespace kgrt_mino
