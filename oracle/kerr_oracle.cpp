// kerr_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU reference of the method of Pu, Yun, Younsi & Yoon
// (2016), "Odyssey: a public GPU-based code for general-relativistic radiative
// transfer in Kerr spacetime": backward tracing of Kerr null geodesics from a
// flat image plane with an adaptive fifth-order Runge-Kutta scheme, with the
// radiative-transfer integrals for tau and I_nu carried along each ray.
//
// Only the test suite, the smoke check and the CPU-baseline leg of the
// benchmark may load this file's library. The GPU library shares no code,
// header, table or constant with it.
//
// Rules kept here on purpose: one ray at a time, formulas written in the
// order the paper states them, double precision, no FMA contraction
// (built with -ffp-contract=off), glibc/libstdc++ math only.
//
// Readings of points the paper leaves open are marked "reading:"; the same
// readings are implemented independently by the GPU path.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <thread>
#include <vector>
#include <algorithm>

extern "C" {

// ---------------------------------------------------------------- structs

// Scene = black hole + observer + emission model + integrator controls.
// Layout mirrored by the ctypes shim (oracle/__init__.py).
typedef struct orc_scene {
    double a;             // spin a/M, |a| < 1                       (Eq. 1)
    double mass;          // M; 1 for every physical run, 0 only for the flat-space limit test
    double incl_deg;      // observer inclination theta_obs           (section 2.2)
    double phi_obs_deg;   // observer azimuth phi_obs                 (section 2.2)
    double r_obs;         // observer distance (1000 M)               (section 2.2)
    double rtol;          // relative tolerance of the RK error control
    double hmax_frac;     // step cap |h| <= hmax_frac * r
    double horizon_delta; // capture when r <= r_plus * (1 + horizon_delta)
    int32_t max_steps;    // accepted-step cap
    int32_t model;        // 0 = geodesic only, 1 = thin disk, 2 = torus, 3 = thick thin disk through every
                          // crossing, 4 = orbiting hot spot, 5 = gridded plasma
    int32_t stop_at_crossing; // terminate at the first equatorial crossing (projection workload)
    int32_t nfreq;        // number of observing frequencies (torus)
    double freqs_hz[16];  // observing frequencies
    // thin Keplerian disk (section 4.3)
    double r_in;          // <= 0 means r_ISCO(a)
    double r_out;
    // analytic torus (synthetic stand-in for section 4.5's shell)
    double n0_cgs, r_norm, n_index, h_over_r, T0_K, T_index, eps_B, mbh_msun, r_emit_max;
    // orbiting hot spot (section 4.4): orbit radius (<= 0 means r_ISCO(a)), spot
    // radius r_spot, azimuth of its centre at t = 0, and the observer time of the image
    double spot_r, spot_size, spot_phi0, t_obs;
    // Form of Eq. (14): 0 = before the null condition eliminates W^2/Delta
    // (default, see orc_rhs), 1 = as printed (kappa form).
    int32_t pr_form;
    int32_t reserved;
    // gridded plasma (model 5): a snapshot of the kind GRMHD simulations write out (section 6),
    // float32 values grid[((i * grid_nth + j) * grid_nph + k) * 4 + q] on the nodes
    //   ln r_i = ln grid_r_min + i (ln grid_r_max - ln grid_r_min) / (grid_nr - 1),
    //   theta_j = j pi / (grid_nth - 1),  phi_k = 2 pi k / grid_nph (periodic in phi),
    // q = 0: ln n_e (cm^-3), 1: ln T_e (K), 2: ln B (G), 3: the flow's angular velocity Omega (1/M)
    const float* grid;
    int32_t grid_nr, grid_nth, grid_nph, grid_reserved;
    double grid_r_min, grid_r_max;
} orc_scene;

typedef struct orc_ray {
    int32_t status;       // bit flags, see ORC_* below
    int32_t steps;        // accepted RK steps
    int32_t attempts;     // attempted RK steps (accepted + rejected)
    int32_t rhs_evals;    // right-hand-side evaluations (incl. crossing refinement)
    double r_cross, g, phi_cross, t_cross;  // first equatorial crossing (0 when none)
    double intensity;     // thin disk: g^3 j(r_c); torus: unused (see I[])
    double i_bol;         // thin disk: g^4 j(r_c)
    double I[16];         // torus: observed I_nu per frequency (cgs)
    double tau[16];       // torus: optical depth per frequency
    double final_state[6];
    double E, L, Q, kappa;      // constants of motion of the traced ray
    double max_H_rel, max_Q_rel; // largest null-condition and Carter-Q drift seen
    double lambda_end;          // affine parameter at termination
    double min_sin;             // smallest sin(theta) over the accepted points (pole approach)
    int32_t n_cross;            // model 3: equatorial crossings outside the capture radius, the emitting one included
    int32_t reserved;
} orc_ray;

enum {
    ORC_CAPTURED = 1, ORC_ESCAPED = 2, ORC_CROSSED = 4, ORC_DISK_HIT = 8,
    ORC_MAXSTEPS = 16, ORC_UNDERFLOW = 32, ORC_NONFINITE = 64,
    ORC_REFINE_UNCONVERGED = 256, ORC_SPOT_HIT = 512
};

// ------------------------------------------------------- physical constants
// CGS, CODATA 2018; solar GM from the IAU 2015 nominal value.
static const double C_LIGHT = 2.99792458e10;
static const double Q_E = 4.80320471e-10;
static const double ME_G = 9.1093837015e-28;
static const double MP_G = 1.67262192369e-24;
static const double H_PLANCK = 6.62607015e-27;
static const double K_BOLTZ = 1.380649e-16;
static const double GM_SUN = 1.3271244e26;
static const double PI = 3.14159265358979323846;

// ------------------------------------------------------------ geometry

// Outer horizon r_+ = M + sqrt(M^2 - a^2) (root of Delta, Eq. 1).
static double horizon_radius(const orc_scene* s) {
    return s->mass + std::sqrt(s->mass * s->mass - s->a * s->a);
}

// Prograde marginally stable orbit of Bardeen, Press & Teukolsky (1972),
// which the paper cites for the disk inner edge (section 4.3). M = 1.
double orc_isco(double a) {
    double z1 = 1.0 + std::cbrt(1.0 - a * a) * (std::cbrt(1.0 + a) + std::cbrt(1.0 - a));
    double z2 = std::sqrt(3.0 * a * a + z1 * z1);
    return 3.0 + z2 - std::sqrt((3.0 - z1) * (3.0 + z1 + 2.0 * z2));
}

// Clamped sine of section 2.1: sin(theta) is replaced by 1e-8 when smaller.
// reading: the clamped value is used wherever sin(theta) appears.
static double clamped_sin(double th) {
    double s = std::sin(th);
    if (s < 1e-8) s = 1e-8;
    return s;
}

// Right-hand side of the six equations (r, theta, phi, t, p_r, p_theta)' of
// section 2.1: Eqs. (4)-(5) inverted for r' and theta', Eq. (9) for t',
// Eq. (12) for phi', Eq. (14) for p_r' and Eq. (15) for p_theta', photons
// (mu = 0). E, L_z, kappa are the constants of the ray. The mass M is kept
// as a parameter (1 in every physical run) so that the flat-space limit can
// be tested.
//
// reading of Eq. (14): the printed form is what -dH/dr becomes after the null
// condition H = 0 has been used to replace W^2/Delta by
// Delta p_r^2 + kappa - 2aEL (W = (r^2+a^2)E - aL). Off the null cone the
// printed form turns any violation C = 2 Sigma H into a growing mode on
// ingoing rays (C Delta is carried unchanged, so an error made at r = 1000
// grows like r^4 by the time the ray nears the hole). By default p_r' is
// therefore evaluated before that substitution,
//     p_r' = [2 r E W / Delta - (r - M)(W^2/Delta^2 + p_r^2)] / Sigma,
// which equals Eq. (14) on the null cone and, with Eq. (15) (already of this
// form), makes the six equations the Hamiltonian flow of C/(2 Sigma), so C is
// conserved. pr_form = 1 selects the printed form.
void orc_rhs(const orc_scene* s, const double* y, const double* c, double* dy) {
    const double M = s->mass, a = s->a;
    const double E = c[0], L = c[1], kappa = c[3];
    const double r = y[0], th = y[1], pr = y[4], pth = y[5];
    const double sn = clamped_sin(th), cs = std::cos(th);
    const double r2a2 = r * r + a * a;
    const double Sigma = r * r + a * a * cs * cs;
    const double Delta = r * r - 2.0 * M * r + a * a;
    const double sn2 = sn * sn;
    dy[0] = Delta * pr / Sigma;                                   // Eq. (4)
    dy[1] = pth / Sigma;                                          // Eq. (5)
    dy[2] = (2.0 * M * a * r * E + (Sigma - 2.0 * M * r) * L / sn2) / (Sigma * Delta);      // Eq. (12)
    dy[3] = E + (2.0 * M * r * r2a2 * E - 2.0 * M * a * r * L) / (Sigma * Delta);           // Eq. (9)
    if (s->pr_form == 1) {
        dy[4] = (-kappa * (r - M) + 2.0 * r * r2a2 * E * E - 2.0 * M * a * E * L) / (Sigma * Delta)
                - 2.0 * pr * pr * (r - M) / Sigma;                // Eq. (14) as printed
    } else {
        const double W = r2a2 * E - a * L;
        dy[4] = (2.0 * r * E * W / Delta - (r - M) * (W * W / (Delta * Delta) + pr * pr)) / Sigma;  // Eq. (14), see above
    }
    dy[5] = sn * cs / Sigma * (L * L / (sn2 * sn2) - a * a * E * E);  // Eq. (15)
}

// Null condition: 2*Sigma*H = Delta p_r^2 + p_th^2 + (L/s - a E s)^2 - W^2/Delta,
// W = (r^2+a^2)E - aL. Returned relative to the sum of the magnitudes of its terms.
static double null_residual(const orc_scene* s, const double* y, const double* c) {
    const double M = s->mass, a = s->a, E = c[0], L = c[1];
    const double r = y[0], th = y[1], pr = y[4], pth = y[5];
    const double sn = clamped_sin(th);
    const double Delta = r * r - 2.0 * M * r + a * a;
    const double W = (r * r + a * a) * E - a * L;
    const double t1 = Delta * pr * pr, t2 = pth * pth;
    const double t3 = (L / sn - a * E * sn) * (L / sn - a * E * sn);
    const double t4 = W * W / Delta;
    return std::fabs(t1 + t2 + t3 - t4) / (std::fabs(t1) + t2 + t3 + std::fabs(t4));
}

// Carter constant, Eq. (13) with mu = 0.
static double carter_q(const orc_scene* s, const double* y, const double* c) {
    const double a = s->a, E = c[0], L = c[1];
    const double sn = clamped_sin(y[1]), cs = std::cos(y[1]);
    return y[5] * y[5] + (L * L / (sn * sn) - a * a * E * E) * cs * cs;
}

// Initial state of the ray through image-plane point (x, y), section 2.2.
// Out: y6 = (r, theta, phi, t, p_r, p_theta); c4 = (E, L_z, Q, kappa).
// Returns 0, or -1 when the start point is unusable (E^2 <= 0 or non-finite).
//
// reading: of the two roots of Eq. (7) the negative one is taken, because the
// received ray is traced backwards in time; all rates are divided by sqrt(E^2)
// so that the traced ray has E = -1 and the affine parameter is measured in M
// far from the hole. The physical photon is the same geodesic reversed
// (E = +1, L_phys = -L_z, same Q).
int orc_initial_state(const orc_scene* s, double x, double yimg, double* y6, double* c4) {
    const double M = s->mass, a = s->a, ro = s->r_obs;
    const double tho = s->incl_deg * PI / 180.0, pho = s->phi_obs_deg * PI / 180.0;
    const double z = 0.0;  // rays start on the image plane
    // Eqs. (18)-(19): image plane -> black-hole Cartesian frame.
    const double D = (std::sqrt(ro * ro + a * a) - z) * std::sin(tho) - yimg * std::cos(tho);
    const double xp = D * std::cos(pho) - x * std::sin(pho);
    const double yp = D * std::sin(pho) + x * std::cos(pho);
    const double zp = (ro - z) * std::cos(tho) + yimg * std::sin(tho);
    // Eqs. (20)-(22): Cartesian -> Boyer-Lindquist.
    const double w = xp * xp + yp * yp + zp * zp - a * a;
    const double r = std::sqrt((w + std::sqrt(w * w + 4.0 * a * a * zp * zp)) / 2.0);
    const double th = std::acos(zp / r);
    const double ph = std::atan2(yp, xp);
    // Eqs. (24)-(26): rates for a ray moving along +z of the image frame.
    const double R = std::sqrt(r * r + a * a);
    const double Phi = ph - pho;
    const double sn = std::sin(th), cs = std::cos(th);
    const double Sigma = r * r + a * a * cs * cs;
    double rdot = -(r * R * sn * std::sin(tho) * std::cos(Phi) + R * R * cs * std::cos(tho)) / Sigma;
    double thdot = (r * sn * std::cos(tho) - R * cs * std::sin(tho) * std::cos(Phi)) / Sigma;
    double phdot = std::sin(tho) * std::sin(Phi) / (R * sn);
    // Eq. (7), mu = 0.
    const double Delta = r * r - 2.0 * M * r + a * a;
    const double E2 = ((Sigma - 2.0 * M * r) / (Sigma * Delta)) * (Sigma * rdot * rdot + Sigma * Delta * thdot * thdot)
                      + Delta * phdot * phdot * sn * sn;
    if (!(E2 > 0.0) || !std::isfinite(E2)) return -1;
    const double norm = std::sqrt(E2);
    rdot /= norm; thdot /= norm; phdot /= norm;
    const double E = -1.0;
    // Eq. (8).
    const double L = (Sigma * Delta * phdot - 2.0 * M * a * r * E) * sn * sn / (Sigma - 2.0 * M * r);
    // Eqs. (4)-(5).
    const double pr = Sigma * rdot / Delta;
    const double pth = Sigma * thdot;
    y6[0] = r; y6[1] = th; y6[2] = ph; y6[3] = 0.0; y6[4] = pr; y6[5] = pth;
    c4[0] = E; c4[1] = L;
    c4[2] = 0.0; c4[3] = 0.0;
    c4[2] = carter_q(s, y6, c4);                              // Eq. (13)
    c4[3] = c4[2] + L * L + a * a * E * E;                    // kappa, section 2.1
    for (int i = 0; i < 6; ++i) if (!std::isfinite(y6[i])) return -1;
    return 0;
}

// ------------------------------------------------------------- redshift

// Four-velocity of the emitter. reading: circular Keplerian motion with
// Omega = M^1/2/(r^3/2 + a M^1/2) in Boyer-Lindquist r at every theta, u^theta = u^r = 0
// (sections 4.3 and 4.5), u^t from u.u = -1; if that has no real solution
// (inside the circular-photon-orbit region) the zero-angular-momentum
// observer, Omega = -g_tphi/g_phiphi, is used instead.
// Returns g = nu_obs/nu_emit, Eq. (2), for an observer at rest at infinity.
// xi = L_z/E of the ray (the same for the traced ray and the physical photon).
double orc_redshift(const orc_scene* s, double r, double th, double xi) {
    const double M = s->mass, a = s->a;
    const double sn = clamped_sin(th), cs = std::cos(th);
    const double Sigma = r * r + a * a * cs * cs;
    const double gtt = -(1.0 - 2.0 * M * r / Sigma);
    const double gtp = -2.0 * M * a * r * sn * sn / Sigma;
    const double gpp = (r * r + a * a + 2.0 * M * a * a * r * sn * sn / Sigma) * sn * sn;
    double Omega = std::sqrt(M) / (r * std::sqrt(r) + a * std::sqrt(M));
    double arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    if (!(arg > 0.0)) {
        Omega = -gtp / gpp;
        arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    }
    const double ut = 1.0 / std::sqrt(arg);
    // -p.u / E_phys = u^t (1 - xi Omega) for u^r = u^theta = 0.
    return 1.0 / (ut * (1.0 - xi * Omega));
}

// ----------------------------------------------------- torus emission model

// Modified Bessel function K_2 (libstdc++ C++17 special function).
double orc_k2(double x) { return std::cyl_bessel_k(2.0, x); }

// Planck function B_nu(T), cgs.
static double planck(double nu, double T) {
    return 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT) / std::expm1(H_PLANCK * nu / (K_BOLTZ * T));
}

// Thermal synchrotron emissivity of Mahadevan et al. (1996), section 4.5,
// Eqs. (37)-(39). reading: Eq. (37) is the angle-integrated coefficient, so
// the per-steradian j_nu used for I_nu is Eq. (37)/(4 pi).
double orc_synchrotron_j(double nu, double ne, double Te, double B) {
    const double theta_e = K_BOLTZ * Te / (ME_G * C_LIGHT * C_LIGHT);
    const double nu_c = 3.0 * Q_E * B / (4.0 * PI * ME_G * C_LIGHT) * theta_e * theta_e;  // Eq. (39)
    const double xm = nu / nu_c;
    const double Mx = 4.0505 / std::pow(xm, 1.0 / 6.0)
                      * (1.0 + 0.40 / std::pow(xm, 0.25) + 0.5316 / std::pow(xm, 0.5))
                      * std::exp(-1.8899 * std::pow(xm, 1.0 / 3.0));                    // Eq. (38)
    const double j4pi = nu * 4.0 * PI * ne * Q_E * Q_E / (std::sqrt(3.0) * C_LIGHT * orc_k2(1.0 / theta_e)) * Mx;  // Eq. (37)
    return j4pi / (4.0 * PI);
}

// Emission and absorption per unit affine parameter seen along the ray at
// (r, theta) with redshift g, observed frequency nu (Eqs. (30)-(31)):
//   a_lam = r_g alpha_0(nu/g) / g,   e_lam = r_g g^2 j_0(nu/g).
// reading: n_e, T_e, B of the synthetic torus are
//   n_e = n0 (r/r_norm)^-n_index exp(-z^2 / (2 (h r)^2)), z = r cos(theta),
//   T_e = T0 (r/r_norm)^-T_index,  B^2/(8 pi) = eps_B n_e m_p c^2 / (6 r),
// with emission only for r_capture < r <= r_emit_max; absorption from
// Kirchhoff's law (section 4.5), alpha_0 = j_0 / B_nu(T_e) at nu_0 = nu/g.
void orc_torus_coeffs(const orc_scene* s, double r, double th, double g, double nu,
                      double* a_lam, double* e_lam) {
    const double rcap = horizon_radius(s) * (1.0 + s->horizon_delta);
    *a_lam = 0.0; *e_lam = 0.0;
    if (!(r > rcap) || r > s->r_emit_max) return;
    const double zc = r * std::cos(th);
    const double hr = s->h_over_r * r;
    const double ne = s->n0_cgs * std::pow(r / s->r_norm, -s->n_index) * std::exp(-zc * zc / (2.0 * hr * hr));
    const double Te = s->T0_K * std::pow(r / s->r_norm, -s->T_index);
    const double B = std::sqrt(8.0 * PI * s->eps_B * ne * MP_G * C_LIGHT * C_LIGHT / (6.0 * r));
    const double nu0 = nu / g;
    const double j = orc_synchrotron_j(nu0, ne, Te, B);
    // reading: no emission means no absorption (guards 0/0 when B_nu underflows).
    const double alpha = (j > 0.0) ? j / planck(nu0, Te) : 0.0;
    const double rg = GM_SUN * s->mbh_msun / (C_LIGHT * C_LIGHT);
    *a_lam = rg * alpha / g;
    *e_lam = rg * g * g * j;
}

// ------------------------------------------------------ gridded plasma

// Redshift (Eq. (2)) of matter circulating with angular velocity Omega at (r, theta),
// u = u^t (1, 0, 0, Omega) with u^t from u.u = -1; the zero-angular-momentum
// observer where that motion is not timelike. xi = L_z/E of the ray.
double orc_redshift_omega(const orc_scene* s, double r, double th, double xi, double Omega) {
    const double M = s->mass, a = s->a;
    const double sn = clamped_sin(th), cs = std::cos(th);
    const double Sigma = r * r + a * a * cs * cs;
    const double gtt = -(1.0 - 2.0 * M * r / Sigma);
    const double gtp = -2.0 * M * a * r * sn * sn / Sigma;
    const double gpp = (r * r + a * a + 2.0 * M * a * a * r * sn * sn / Sigma) * sn * sn;
    double arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    if (!(arg > 0.0)) {
        Omega = -gtp / gpp;
        arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    }
    const double ut = 1.0 / std::sqrt(arg);
    return 1.0 / (ut * (1.0 - xi * Omega));
}

// The plasma of a simulation snapshot sampled at (r, theta, phi). reading: the
// snapshot is frozen while the light crosses it (the "fast light" reading of
// section 6); values between the nodes are the trilinear interpolation in
// (ln r, theta, phi) of the stored values, phi periodic, theta clamped to
// [0, pi]; there is no plasma outside [grid_r_min, grid_r_max] nor at or
// inside the capture radius. Writes the four interpolated values (ln n_e,
// ln T_e, ln B, Omega) to v; returns 0 where there is no plasma, else 1.
int orc_grid_sample(const orc_scene* s, double r, double th, double ph, double* v) {
    for (int q = 0; q < 4; ++q) v[q] = 0.0;
    const double rcap = horizon_radius(s) * (1.0 + s->horizon_delta);
    if (!(r > rcap) || r < s->grid_r_min || r > s->grid_r_max) return 0;
    const int nr = s->grid_nr, nt = s->grid_nth, np = s->grid_nph;
    // fractional node coordinates along each axis
    double u1 = (std::log(r) - std::log(s->grid_r_min)) / (std::log(s->grid_r_max) - std::log(s->grid_r_min))
                * (nr - 1);
    double u2 = th / PI * (nt - 1);
    if (u2 < 0.0) u2 = 0.0;
    if (u2 > nt - 1) u2 = nt - 1;
    const double u3 = ph / (2.0 * PI) * np;
    int i0 = (int)std::floor(u1);
    if (i0 > nr - 2) i0 = nr - 2;
    if (i0 < 0) i0 = 0;
    int j0 = (int)std::floor(u2);
    if (j0 > nt - 2) j0 = nt - 2;
    const double k0f = std::floor(u3);
    const double w1 = u1 - i0, w2 = u2 - j0, w3 = u3 - k0f;
    int k0 = (int)std::fmod(k0f, (double)np);
    if (k0 < 0) k0 += np;
    const int k1 = (k0 + 1) % np;
    const int ii[2] = {i0, i0 + 1}, jj[2] = {j0, j0 + 1}, kk[2] = {k0, k1};
    const double wi[2] = {1.0 - w1, w1}, wj[2] = {1.0 - w2, w2}, wk[2] = {1.0 - w3, w3};
    for (int ia = 0; ia < 2; ++ia)
        for (int jb = 0; jb < 2; ++jb)
            for (int kc = 0; kc < 2; ++kc) {
                const double w = wi[ia] * wj[jb] * wk[kc];
                const float* node = s->grid + ((int64_t)(ii[ia] * nt + jj[jb]) * np + kk[kc]) * 4;
                for (int q = 0; q < 4; ++q) v[q] += w * (double)node[q];
            }
    return 1;
}

// Emission and absorption per unit affine parameter from the gridded plasma
// (Eqs. (30)-(31)), as for the torus: thermal synchrotron j_0 of Eqs. (37)-(39)
// per steradian and Kirchhoff absorption at nu_0 = nu/g, with g of matter
// moving with the gridded Omega. Also returns that g (0 where there is no plasma).
void orc_grid_coeffs(const orc_scene* s, double r, double th, double ph, double xi, double nu,
                     double* a_lam, double* e_lam, double* g_out) {
    double v[4];
    *a_lam = 0.0; *e_lam = 0.0; *g_out = 0.0;
    if (!orc_grid_sample(s, r, th, ph, v)) return;
    const double ne = std::exp(v[0]), Te = std::exp(v[1]), B = std::exp(v[2]);
    const double g = orc_redshift_omega(s, r, th, xi, v[3]);
    const double nu0 = nu / g;
    const double j = orc_synchrotron_j(nu0, ne, Te, B);
    const double alpha = (j > 0.0) ? j / planck(nu0, Te) : 0.0;
    const double rg = GM_SUN * s->mbh_msun / (C_LIGHT * C_LIGHT);
    *a_lam = rg * alpha / g;
    *e_lam = rg * g * g * j;
    *g_out = g;
}

// ----------------------------------------------------------- hot spot

// The orbiting hot spot of section 4.4. reading: its centre moves on the
// equatorial circle of Boyer-Lindquist radius r_s with the Keplerian angular
// velocity Omega_s = 1/(r_s^3/2 + a) (prograde), azimuth phi_0 + Omega_s t at
// coordinate time t. Positions are compared in the pseudo-Cartesian coordinates
// of section 2.2 (x = sqrt(r^2+a^2) sin(theta) cos(phi), y = ... sin(phi),
// z = r cos(theta)). The spot is the region z > 0, d < 4 r_spot, d the distance
// from the centre; it is optically thick, so a ray ends where it first enters
// the region, and the emissivity there is exp(-d^2 / (2 r_spot^2)) (Eq. (36)).
static double spot_orbit_radius(const orc_scene* s) { return (s->spot_r > 0.0) ? s->spot_r : orc_isco(s->a); }

static double spot_omega(const orc_scene* s) {
    const double rs = spot_orbit_radius(s);
    return 1.0 / (rs * std::sqrt(rs) + s->a);
}

// Squared distance from the spot centre of the point y (r, theta, phi, t, ...) at
// the emission time t_obs + t (the traced ray's t runs backwards from 0).
static double spot_distance2(const orc_scene* s, const double* y) {
    const double a = s->a, rs = spot_orbit_radius(s);
    const double t_emm = s->t_obs + y[3];
    const double phic = s->spot_phi0 + spot_omega(s) * t_emm;
    const double Rs = std::sqrt(rs * rs + a * a);
    const double R = std::sqrt(y[0] * y[0] + a * a);
    const double dx = R * std::sin(y[1]) * std::cos(y[2]) - Rs * std::cos(phic);
    const double dy = R * std::sin(y[1]) * std::sin(y[2]) - Rs * std::sin(phic);
    const double dz = y[0] * std::cos(y[1]);
    return dx * dx + dy * dy + dz * dz;
}

static bool in_spot(const orc_scene* s, const double* y) {
    const double cut = 4.0 * s->spot_size;
    return y[0] * std::cos(y[1]) > 0.0 && spot_distance2(s, y) < cut * cut;
}

// Redshift (Eq. (2)) of spot material at (r, theta). reading: the spot moves
// rigidly with its centre, u = u^t (1, 0, 0, Omega_s), u^t from u.u = -1; the
// zero-angular-momentum observer where that is not timelike.
double orc_spot_redshift(const orc_scene* s, double r, double th, double xi) {
    const double M = s->mass, a = s->a;
    const double sn = clamped_sin(th), cs = std::cos(th);
    const double Sigma = r * r + a * a * cs * cs;
    const double gtt = -(1.0 - 2.0 * M * r / Sigma);
    const double gtp = -2.0 * M * a * r * sn * sn / Sigma;
    const double gpp = (r * r + a * a + 2.0 * M * a * a * r * sn * sn / Sigma) * sn * sn;
    double Omega = spot_omega(s);
    double arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    if (!(arg > 0.0)) {
        Omega = -gtp / gpp;
        arg = -(gtt + 2.0 * Omega * gtp + Omega * Omega * gpp);
    }
    const double ut = 1.0 / std::sqrt(arg);
    return 1.0 / (ut * (1.0 - xi * Omega));
}

// ----------------------------------------------------- Cash-Karp stepper

// Embedded Runge-Kutta 5(4) pair of Cash & Karp (1990, ACM TOMS 16, 201);
// reading of "fifth-order Runge-Kutta with adaptive step size" (section 2.1).
// The fifth-order solution is propagated; err = y5 - y4.
static const double CK_A21 = 1.0 / 5.0;
static const double CK_A31 = 3.0 / 40.0, CK_A32 = 9.0 / 40.0;
static const double CK_A41 = 3.0 / 10.0, CK_A42 = -9.0 / 10.0, CK_A43 = 6.0 / 5.0;
static const double CK_A51 = -11.0 / 54.0, CK_A52 = 5.0 / 2.0, CK_A53 = -70.0 / 27.0, CK_A54 = 35.0 / 27.0;
static const double CK_A61 = 1631.0 / 55296.0, CK_A62 = 175.0 / 512.0, CK_A63 = 575.0 / 13824.0,
                    CK_A64 = 44275.0 / 110592.0, CK_A65 = 253.0 / 4096.0;
static const double CK_B1 = 37.0 / 378.0, CK_B3 = 250.0 / 621.0, CK_B4 = 125.0 / 594.0, CK_B6 = 512.0 / 1771.0;
static const double CK_D1 = 37.0 / 378.0 - 2825.0 / 27648.0, CK_D3 = 250.0 / 621.0 - 18575.0 / 48384.0,
                    CK_D4 = 125.0 / 594.0 - 13525.0 / 55296.0, CK_D5 = -277.0 / 14336.0,
                    CK_D6 = 512.0 / 1771.0 - 1.0 / 4.0;

// One Cash-Karp step of size h from y with k1 = f(y). Writes the fifth-order
// result to yout and the embedded error estimate to yerr. 5 RHS calls.
static void cash_karp(const orc_scene* s, const double* c, const double* y, const double* k1, double h,
                      double* yout, double* yerr) {
    double k2[6], k3[6], k4[6], k5[6], k6[6], yt[6];
    for (int i = 0; i < 6; ++i) yt[i] = y[i] + h * (CK_A21 * k1[i]);
    orc_rhs(s, yt, c, k2);
    for (int i = 0; i < 6; ++i) yt[i] = y[i] + h * (CK_A31 * k1[i] + CK_A32 * k2[i]);
    orc_rhs(s, yt, c, k3);
    for (int i = 0; i < 6; ++i) yt[i] = y[i] + h * (CK_A41 * k1[i] + CK_A42 * k2[i] + CK_A43 * k3[i]);
    orc_rhs(s, yt, c, k4);
    for (int i = 0; i < 6; ++i)
        yt[i] = y[i] + h * (CK_A51 * k1[i] + CK_A52 * k2[i] + CK_A53 * k3[i] + CK_A54 * k4[i]);
    orc_rhs(s, yt, c, k5);
    for (int i = 0; i < 6; ++i)
        yt[i] = y[i] + h * (CK_A61 * k1[i] + CK_A62 * k2[i] + CK_A63 * k3[i] + CK_A64 * k4[i] + CK_A65 * k5[i]);
    orc_rhs(s, yt, c, k6);
    for (int i = 0; i < 6; ++i) {
        yout[i] = y[i] + h * (CK_B1 * k1[i] + CK_B3 * k3[i] + CK_B4 * k4[i] + CK_B6 * k6[i]);
        yerr[i] = h * (CK_D1 * k1[i] + CK_D3 * k3[i] + CK_D4 * k4[i] + CK_D5 * k5[i] + CK_D6 * k6[i]);
    }
}

static bool all_finite(const double* y) {
    for (int i = 0; i < 6; ++i) if (!std::isfinite(y[i])) return false;
    return true;
}

// ---------------------------------------------------------------- tracer

// Transfer coefficients at the point y of a ray with xi = L_z/E: the torus
// (model 2) or the gridded plasma (model 5).
static void point_coeffs(const orc_scene* s, const double* y, double xi, double nu, double* a_lam,
                         double* e_lam) {
    if (s->model == 5) {
        double g;
        orc_grid_coeffs(s, y[0], y[1], y[2], xi, nu, a_lam, e_lam, &g);
        return;
    }
    const double g = orc_redshift(s, y[0], y[1], xi);
    orc_torus_coeffs(s, y[0], y[1], g, nu, a_lam, e_lam);
}

// Traces one ray from image-plane point (x, y). If path != nullptr the state
// after every accepted step is appended (up to path_cap rows of 7 doubles:
// lambda, y[6]).
static void trace_one(const orc_scene* s, double x, double yimg, orc_ray* out,
                      double* path, int64_t path_cap, int64_t* path_len) {
    std::memset(out, 0, sizeof(*out));
    if (path_len) *path_len = 0;
    double y[6], c[4];
    if (orc_initial_state(s, x, yimg, y, c) != 0) {
        out->status = ORC_NONFINITE;
        return;
    }
    out->E = c[0]; out->L = c[1]; out->Q = c[2]; out->kappa = c[3];
    const double xi = c[1] / c[0];
    const double rplus = horizon_radius(s);
    const double rcap = rplus * (1.0 + s->horizon_delta);
    const double r_in = (s->r_in > 0.0) ? s->r_in : orc_isco(s->a);
    const int nf = (s->model == 2 || s->model == 5) ? s->nfreq : 0;
    const bool want_cross = (s->model != 2 && s->model != 4 && s->model != 5);
    // model 3: the disk of section 4.3 is optically thick and the ray is followed
    // through every equatorial crossing until one lands on it (the direct image and
    // the higher-order images the hole's lensing makes of the same disk)
    const bool every_crossing = (s->model == 3);
    int32_t n_cross = 0;
    const bool spot = (s->model == 4);
    const double q0 = c[2];
    const double qden = std::max(std::fabs(c[3]), 1.0);

    // Radiative transfer state (section 2.3). reading: coefficients are
    // evaluated once per accepted endpoint (the start point included) and
    // each step adds the exponential-trapezoid increment, exact for
    // coefficients constant over the step:
    //   dtau = h (a_k + a_k+1)/2,  dI = exp(-tau_k) h (e_k + e_k+1)/2 * (1 - exp(-dtau))/dtau.
    double a_prev[16], e_prev[16];
    for (int f = 0; f < nf; ++f) {
        point_coeffs(s, y, xi, s->freqs_hz[f], &a_prev[f], &e_prev[f]);
        out->I[f] = 0.0; out->tau[f] = 0.0;
    }

    double h = s->hmax_frac * s->r_obs;  // reading: initial step = cap at the observer
    double lambda = 0.0;
    double k1[6], yn[6], ye[6];
    int steps = 0, attempts = 0, rhs = 0;
    bool crossed = false;
    int status = 0;
    double maxH = null_residual(s, y, c), maxQ = 0.0;
    double min_sin = std::fabs(std::sin(y[1]));
    if (path && path_cap > 0) { path[0] = 0.0; for (int i = 0; i < 6; ++i) path[1 + i] = y[i]; *path_len = 1; }

    orc_rhs(s, y, c, k1); ++rhs;
    for (;;) {
        // ---- attempt a step (section 2.1, adaptive step size)
        double errmax;
        for (;;) {
            cash_karp(s, c, y, k1, h, yn, ye);
            rhs += 5; ++attempts;
            errmax = 0.0;
            for (int i = 0; i < 6; ++i) {
                const double scale = std::fabs(y[i]) + std::fabs(h * k1[i]) + 1e-12;
                const double e = std::fabs(ye[i]) / (s->rtol * scale);
                if (e > errmax) errmax = e;
            }
            if (!(errmax <= 1.0)) {
                // reading: a NaN error estimate is treated as a rejection
                if (!std::isfinite(errmax)) errmax = 1e10;
                double shrink = 0.9 * std::pow(errmax, -0.25);
                if (shrink < 0.1) shrink = 0.1;
                h = h * shrink;
                if (std::fabs(h) < 1e-12 * std::max(1.0, y[0])) { status |= ORC_UNDERFLOW; goto done; }
                continue;
            }
            break;
        }
        // ---- accepted: y_k -> y_{k+1} over [lambda, lambda + h]
        {
            const double hdone = h;
            double hnext = (errmax > 1.89e-4) ? h * (0.9 * std::pow(errmax, -0.2)) : h * 5.0;
            ++steps;
            double yprev[6];
            for (int i = 0; i < 6; ++i) { yprev[i] = y[i]; y[i] = yn[i]; }
            lambda += hdone;
            if (!all_finite(y)) { status |= ORC_NONFINITE; goto done; }
            if (path && *path_len < path_cap) {
                double* row = path + 7 * (*path_len);
                row[0] = lambda; for (int i = 0; i < 6; ++i) row[1 + i] = y[i];
                ++*path_len;
            }
            {
                const double hr = null_residual(s, y, c);
                if (hr > maxH) maxH = hr;
                const double dq = std::fabs(carter_q(s, y, c) - q0) / qden;
                if (dq > maxQ) maxQ = dq;
                const double sabs = std::fabs(std::sin(y[1]));
                if (sabs < min_sin) min_sin = sabs;
            }
            // hot spot: the first accepted point inside the spot ends the ray; its entry
            // point is located by bisection of the step size from y_k (each trial one full
            // Cash-Karp step without error control), 48 halvings of the accepted step
            if (spot && in_spot(s, y)) {
                double lo = 0.0, hi = hdone, yin[6], yt[6], yte[6];
                for (int i = 0; i < 6; ++i) yin[i] = y[i];
                for (int it = 0; it < 48; ++it) {
                    const double hm = 0.5 * (lo + hi);
                    cash_karp(s, c, yprev, k1, hm, yt, yte);
                    rhs += 5;
                    if (in_spot(s, yt)) {
                        hi = hm;
                        for (int i = 0; i < 6; ++i) yin[i] = yt[i];
                    } else {
                        lo = hm;
                    }
                }
                const double d2 = spot_distance2(s, yin);
                const double j = std::exp(-d2 / (2.0 * s->spot_size * s->spot_size));  // Eq. (36)
                status |= ORC_SPOT_HIT;
                out->r_cross = yin[0];
                out->phi_cross = yin[2];
                out->t_cross = s->t_obs + yin[3];  // emission time t_emm = t_obs - Delta t
                out->g = orc_spot_redshift(s, yin[0], yin[1], xi);
                out->intensity = out->g * out->g * out->g * j;
                out->i_bol = out->g * out->g * out->g * out->g * j;
                for (int i = 0; i < 6; ++i) y[i] = yin[i];
                goto done;
            }
            // radiative transfer over the accepted step (Eqs. (30)-(31))
            if (nf > 0) {
                for (int f = 0; f < nf; ++f) {
                    double a1, e1;
                    point_coeffs(s, y, xi, s->freqs_hz[f], &a1, &e1);
                    const double dtau = hdone * (a_prev[f] + a1) / 2.0;
                    const double phi = (dtau > 0.0) ? -std::expm1(-dtau) / dtau : 1.0;
                    out->I[f] += std::exp(-out->tau[f]) * hdone * (e_prev[f] + e1) / 2.0 * phi;
                    out->tau[f] += dtau;
                    a_prev[f] = a1; e_prev[f] = e1;
                }
            }
            // first equatorial crossing. reading: a sign change of cos(theta)
            // over an accepted step is located by Newton iteration on the
            // step size from y_k, each iterate one full Cash-Karp step without
            // error control; integration then continues from y_{k+1}.
            if (want_cross && (!crossed || every_crossing)) {
                const double c0 = std::cos(yprev[1]), c1 = std::cos(y[1]);
                if ((c0 > 0.0 && c1 <= 0.0) || (c0 < 0.0 && c1 >= 0.0)) {
                    crossed = true;
                    const double* kprev = k1;  // f(y_k), computed before the step
                    double hs = hdone * c0 / (c0 - c1);
                    double ys[6], yse[6];
                    bool conv = false;
                    for (int it = 0; it < 7; ++it) {
                        cash_karp(s, c, yprev, kprev, hs, ys, yse); rhs += 5;
                        const double cz = std::cos(ys[1]);
                        if (std::fabs(cz) <= 1e-13) { conv = true; break; }
                        if (it == 6) break;
                        const double thdot = ys[5] / (ys[0] * ys[0] + s->a * s->a * cz * cz);
                        hs = hs + cz / (std::sin(ys[1]) * thdot);
                    }
                    if (!conv) status |= ORC_REFINE_UNCONVERGED;
                    const double rc = ys[0];
                    if (every_crossing) {
                        if (rc > rcap) {
                            ++n_cross;
                            if (rc >= r_in && rc <= s->r_out) {
                                // reading: the first crossing on the disk is where the ray ends
                                status |= ORC_CROSSED | ORC_DISK_HIT;
                                out->r_cross = rc;
                                out->phi_cross = ys[2];
                                out->t_cross = ys[3];
                                out->g = orc_redshift(s, rc, PI / 2.0, xi);
                                const double j = 1.0 / (rc * rc * rc);  // emissivity r^-3
                                out->intensity = out->g * out->g * out->g * j;
                                out->i_bol = out->g * out->g * out->g * out->g * j;
                                goto done;
                            }
                        }
                    } else if (rc > rcap) {
                        status |= ORC_CROSSED;
                        out->r_cross = rc;
                        out->phi_cross = ys[2];
                        out->t_cross = ys[3];
                        // the disk lies in the equatorial plane: redshift there
                        out->g = orc_redshift(s, rc, PI / 2.0, xi);
                        if (s->model == 1 && rc >= r_in && rc <= s->r_out) {
                            status |= ORC_DISK_HIT;
                            const double j = 1.0 / (rc * rc * rc);  // emissivity r^-3
                            out->intensity = out->g * out->g * out->g * j;
                            out->i_bol = out->g * out->g * out->g * out->g * j;
                        }
                        if (s->stop_at_crossing) goto done;
                    }
                }
            }
            if (y[0] <= rcap) { status |= ORC_CAPTURED; goto done; }
            if (y[4] > 0.0 && y[0] > s->r_obs) { status |= ORC_ESCAPED; goto done; }
            if (steps >= s->max_steps) { status |= ORC_MAXSTEPS; goto done; }
            // step-size cap, reading of the controller: |h| <= hmax_frac * r
            const double hcap = s->hmax_frac * y[0];
            if (hnext > hcap) hnext = hcap;
            h = hnext;
            orc_rhs(s, y, c, k1); ++rhs;
        }
    }
done:
    out->status = status;
    out->steps = steps;
    out->attempts = attempts;
    out->rhs_evals = rhs;
    out->lambda_end = lambda;
    for (int i = 0; i < 6; ++i) out->final_state[i] = y[i];
    out->max_H_rel = maxH;
    out->max_Q_rel = maxQ;
    out->min_sin = min_sin;
    out->n_cross = n_cross;
}

int orc_trace_ray(const orc_scene* s, double x, double y, orc_ray* out) {
    trace_one(s, x, y, out, nullptr, 0, nullptr);
    return 0;
}

int64_t orc_trace_path(const orc_scene* s, double x, double y, orc_ray* out, double* path, int64_t cap) {
    int64_t n = 0;
    trace_one(s, x, y, out, path, cap, &n);
    return n;
}

// Traces n rays; xy holds image-plane (x, y) pairs. Rays are striped over
// nthreads std::threads (rays are independent, section 1).
int orc_trace_points(const orc_scene* s, int64_t n, const double* xy, orc_ray* out, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) {
        pool.emplace_back([=]() {
            for (int64_t i = t; i < n; i += nthreads) trace_one(s, xy[2 * i], xy[2 * i + 1], &out[i], nullptr, 0, nullptr);
        });
    }
    for (auto& th : pool) th.join();
    return 0;
}

// Ray-list mode: each ray carries its own spin, inclination and image-plane
// point (a, incl_deg, x, y); everything else comes from the base scene.
int orc_trace_ray_list(const orc_scene* base, int64_t n, const double* rays4, orc_ray* out, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    std::vector<std::thread> pool;
    for (int t = 0; t < nthreads; ++t) {
        pool.emplace_back([=]() {
            for (int64_t i = t; i < n; i += nthreads) {
                orc_scene s = *base;
                s.a = rays4[4 * i];
                s.incl_deg = rays4[4 * i + 1];
                trace_one(&s, rays4[4 * i + 2], rays4[4 * i + 3], &out[i], nullptr, 0, nullptr);
            }
        });
    }
    for (auto& th : pool) th.join();
    return 0;
}

int orc_sizeof_scene() { return (int)sizeof(orc_scene); }
int orc_sizeof_ray() { return (int)sizeof(orc_ray); }

}  // extern "C"
