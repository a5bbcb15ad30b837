// kgrt.hip -- persistent FP64 integrator kernels and the C ABI (include/kgrt.h).
//
// Design (gfx950, wave64):
//  * one ray per lane, the whole ray state (6 doubles, step size, counters,
//    per-frequency tau and I) register resident for the life of the ray;
//  * a persistent grid sized to the device's occupancy; each wave refills its
//    idle lanes from a global ray counter with one ballot and one atomicAdd
//    (lane offsets from a popcount prefix), so rays of very different step
//    counts never leave a wave waiting for its slowest member;
//  * ray ids are image-major, so freshly claimed lanes of a wave write
//    neighbouring pixels (coalesced SoA outputs);
//  * per-image uniforms (spin, observer angles, capture radius, disk edges) are
//    precomputed on the host once per image.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kgrt.h"
#include "kgrt_device.hpp"

namespace kgrt {

// Everything a lane needs to start a ray of one image.
struct ImageDesc {
    double a, a2, r_obs, sqrt_ro2a2;
    double sin_i, cos_i, sin_p, cos_p, phi_obs;
    double x_min, x_w, y_min, y_w;
    double r_cap, r_in;  // r_in: the disk's inner edge, or the hot spot's orbit radius
    double t_obs;        // observer time of the image (hot spot)
    int64_t ray_offset;
    int32_t nx, ny;
};

struct Outputs {
    int32_t *status, *steps, *attempts;
    double *r_cross, *g, *phi_cross, *t_cross, *intensity, *i_bol, *tau;
    int32_t* n_cross;
};

struct KParams {
    ImageDesc image0;           // single-image mode (nimg == 1)
    const ImageDesc* images;    // device table, nimg > 1
    const double* rays4;        // ray-list mode
    unsigned long long* counter;
    int64_t nrays;
    int32_t nimg;
    int32_t list_mode;
    double list_r_obs, list_phi_obs, list_sin_p, list_cos_p;
    // model
    int32_t model, nf;
    double freqs[16];
    double inv_freqs[16];
    double r_in_cfg, r_out;
    double spot_r_cfg, spot_phi0, spot_cut2, spot_inv_2s2;  // hot spot: orbit (<= 0: ISCO), phase, (4 r_spot)^2, 1/(2 r_spot^2)
    TorusParams torus;
    GridParams grid;  // gridded plasma (snapshot) model
    // integrator
    double rtol, hmax_frac, horizon_delta;
    int32_t max_steps;
    uint32_t flags;
    int32_t refill_min;
    int32_t naive;  // 1: one ray per thread, no queue (the paper's mapping, kept as a baseline)
    const int64_t* count_dev;  // if set, only rays [0, *count_dev) exist (lists built on the device)
    Outputs out;
};

// Ray id -> start state and the per-ray uniforms (spin, capture radius,
// disk inner edge, observer distance).
__device__ __forceinline__ bool start_from_id(const KParams& P, int64_t rid, State& st, double& a, double& a2,
                                              double& L, double& r_cap, double& r_in, double& r_obs,
                                              double& t_obs) {
    if (P.list_mode) {
        const double* q = P.rays4 + 4 * rid;
        const double aa = q[0], incl = q[1], x = q[2], y = q[3];
        const double tho = incl * kPi / 180.0;
        double si, ci;
        sincos_bounded(tho, &si, &ci);
        a = aa;
        a2 = aa * aa;
        r_obs = P.list_r_obs;
        bool ok = start_ray(aa, a2, r_obs, sqrt(r_obs * r_obs + a2), si, ci, P.list_sin_p, P.list_cos_p,
                            P.list_phi_obs, x, y, st, L);
        r_cap = (1.0 + sqrt(1.0 - a2)) * (1.0 + P.horizon_delta);
        const double r_in_c = (P.model == KGRT_MODEL_HOT_SPOT) ? P.spot_r_cfg : P.r_in_cfg;
        r_in = (r_in_c > 0.0) ? r_in_c : isco_radius(aa);
        t_obs = 0.0;
        if (!(fabs(aa) < 1.0) || !(incl > 0.0 && incl < 180.0) || !isfinite(x) || !isfinite(y)) ok = false;
        return ok;
    }
    const ImageDesc* d = &P.image0;
    if (P.nimg > 1) {
        int lo = 0, hi = P.nimg - 1;  // last image with ray_offset <= rid
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (P.images[mid].ray_offset <= rid) lo = mid; else hi = mid - 1;
        }
        d = &P.images[lo];
    }
    const int64_t p = rid - d->ray_offset;
    const int32_t i = (int32_t)(p % d->nx), j = (int32_t)(p / d->nx);
    // cell centres, same operation order as the documented rule
    const double x = d->x_min + ((i + 0.5) * d->x_w) / d->nx;
    const double y = d->y_min + ((j + 0.5) * d->y_w) / d->ny;
    a = d->a;
    a2 = d->a2;
    r_obs = d->r_obs;
    r_cap = d->r_cap;
    r_in = d->r_in;
    t_obs = d->t_obs;
    return start_ray(d->a, d->a2, d->r_obs, d->sqrt_ro2a2, d->sin_i, d->cos_i, d->sin_p, d->cos_p, d->phi_obs, x,
                     y, st, L);
}

// The hot spot of section 4.4 at the emission time t_obs + y.t of the point y (the
// traced ray's t runs backwards from 0): its centre sits at pseudo-Cartesian
// cylindrical radius rho_c and azimuth phi0 + om_s (t_obs + y.t) in the
// equatorial plane. Squared distance from the centre by the law of cosines in
// the cylindrical coordinates of section 2.2 (rho = sqrt(r^2 + a^2) sin(theta),
// z = r cos(theta)); s, c are sin(theta), cos(theta) (unclamped).
__device__ __forceinline__ double spot_d2(const State& y, double s, double c, double a2, double t_obs, double om_s,
                                          double rho_c, double phi0) {
    const double rho = sqrt(fma(y.r, y.r, a2)) * s;
    const double z = y.r * c;
    double sd, cd;
    sincos_bounded(y.ph - fma(om_s, t_obs + y.t, phi0), &sd, &cd);
    return fma(rho, rho - 2.0 * rho_c * cd, fma(rho_c, rho_c, z * z));
}

// The spot is the region z > 0, d < 4 r_spot (cut2 = (4 r_spot)^2).
__device__ __forceinline__ bool spot_inside(const State& y, double s, double c, double a2, double t_obs, double om_s,
                                            double rho_c, double phi0, double cut2) {
    return y.r * c > 0.0 && spot_d2(y, s, c, a2, t_obs, om_s, rho_c, phi0) < cut2;
}

// Per-ray start record written by start_kernel and read by the integrator at
// refill, structure-of-arrays over the rays of one chunk:
//   r, theta, phi, p_r, p_theta, L_z, a, r_capture, r_in, r_obs, t_obs.
// A non-finite r marks an unusable start point.
constexpr int kRecFields = 11;

// ------------------------------------------------------------ kernels

// The kernel's first argument (KParams: explicit kernel arguments start the
// kernarg segment, in order), read again with scalar loads where it is used.
// The torus and frequency parameters of the transfer are uniform values that
// the compiler would otherwise load once and keep across the persistent loop;
// with the SGPRs that loop needs they do not fit, so they would be parked in
// VGPR lanes and restored with one v_readlane (a vector instruction) per 32
// bits at every accepted step. The empty asm makes the pointer opaque, so the
// loads cannot be hoisted out of the loop; they stay scalar loads from the
// constant address space.
__device__ __forceinline__ const KParams& reread_params() {
    typedef const __attribute__((address_space(4))) KParams CK;
    CK* p = (CK*)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const KParams*)p;
}

__global__ void reset_counter(unsigned long long* c) { *c = 0ull; }

// One thread per ray of the chunk [base, base + count): ray start (section 2.2).
__global__ void __launch_bounds__(256) start_kernel(const KParams P, int64_t base, int64_t count, double* rec,
                                                    int64_t cap) {
    if (P.count_dev) count = std::max<int64_t>(0, std::min<int64_t>(count, *P.count_dev - base));
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += (int64_t)gridDim.x * blockDim.x) {
        State st;
        double a, a2, L, r_cap, r_in, r_obs, t_obs;
        const bool ok = start_from_id(P, base + k, st, a, a2, L, r_cap, r_in, r_obs, t_obs);
        rec[0 * cap + k] = ok ? st.r : __builtin_nan("");
        rec[1 * cap + k] = st.th;
        rec[2 * cap + k] = st.ph;
        rec[3 * cap + k] = st.pr;
        rec[4 * cap + k] = st.pth;
        rec[5 * cap + k] = L;
        rec[6 * cap + k] = a;
        rec[7 * cap + k] = r_cap;
        rec[8 * cap + k] = r_in;
        rec[9 * cap + k] = r_obs;
        rec[10 * cap + k] = t_obs;
    }
}

// Waves per SIMD the register allocation targets, per model and number of
// frequencies carried (measured on MI355X, with the build's machine-LICM
// setting for this file). The one-frequency torus kernel and the thin-disk and
// projection kernels run fastest at four waves: the register budget of 128
// costs them a few spilled words (the disk kernel, 157 VGPRs at three waves,
// spills 128 B at four and is still 3.5% faster). The eight-frequency kernel
// keeps its per-frequency sums in LDS and runs at three (below); the 2- and
// 4-frequency kernels (143 and 163 VGPRs) fit three as well, but small images
// give them too few rays per lane there, so their launches fall back to the
// residency of two waves when three would leave fewer than kMinRaysPerLane rays
// per lane (measured: at 1024^2 three waves are 6-11% faster, at 512^2 18%
// slower); the 16-frequency kernel (256 VGPRs) runs at two. One wave is 35%
// slower.
#ifndef KGRT_WAVES_DISK
#define KGRT_WAVES_DISK 4
#endif
#ifndef KGRT_WAVES_TORUS
#define KGRT_WAVES_TORUS 4
#endif
#ifndef KGRT_WAVES_TORUS_MULTI
#define KGRT_WAVES_TORUS_MULTI 2
#endif
// The eight-frequency kernel keeps each thread's optical depths, intensities
// and attenuations in LDS (three slots per frequency, 48 KB per 256-thread
// block) instead of VGPRs: it then fits three waves per SIMD without spills.
template <int NF> struct AccInLds {
    static constexpr bool value = (NF == 8);
};
template <int NF> struct RayCountResidency {
    static constexpr bool value = (NF == 2 || NF == 4);
};
constexpr int kMinRaysPerLane = 3;
#ifndef KGRT_WAVES_SPOT
#define KGRT_WAVES_SPOT 3
#endif
// the models that carry the transfer of Eqs. (30)-(31) along the ray
template <int MODEL> struct Transfer {
    static constexpr bool value = (MODEL == KGRT_MODEL_TORUS || MODEL == KGRT_MODEL_GRID);
};
template <int MODEL, int NF> struct WavesPerEU {
    static constexpr int value =
        (MODEL == KGRT_MODEL_HOT_SPOT) ? KGRT_WAVES_SPOT
        : !Transfer<MODEL>::value
            ? KGRT_WAVES_DISK
            : (NF == 1 ? KGRT_WAVES_TORUS
                       : ((AccInLds<NF>::value || RayCountResidency<NF>::value) ? 3 : KGRT_WAVES_TORUS_MULTI));
};
// Refill granularity when the caller sets none: a wave refills only when all 64 lanes are idle
// (it takes 64 consecutive rays of the queue, neighbouring pixels that stay in step: less
// divergence and refill work; 2-13% faster than refilling lane by lane on every model up to four
// frequencies, measured), except the kernels of eight and more frequencies, which refill lane by
// lane (the eight-frequency kernel was 2-8% slower at 8..64).
template <int MODEL, int NF> struct DefaultRefill {
    static constexpr int value = (NF < 8) ? 64 : 1;
};
// dynamic LDS bytes of one block of `block` threads
template <int NF> constexpr size_t acc_lds_bytes(int block) {
    return AccInLds<NF>::value ? (size_t)3 * NF * block * sizeof(double) : 0;
}

// Frequency-independent transfer quantities at the point y (sy, cy: its clamped
// sin and cos of theta) of a ray with L_z = L: the redshift g (ig = 1/g) of the
// emitting matter and the plasma there. The torus flows on Keplerian circles;
// the snapshot's plasma moves with its gridded Omega.
template <int MODEL>
__device__ __forceinline__ Plasma point_plasma(const KParams& PR, const State& y, double sy, double cy, double a,
                                               double a2, double L, double r_cap, double& g, double& ig) {
    if constexpr (MODEL == KGRT_MODEL_GRID) {
        double v[4];
        if (!grid_sample(PR.grid, y.r, y.th, y.ph, r_cap, v)) {
            Plasma q;
            q.emits = false;
            q.ne = q.Te = q.inv_nu_c = q.jpref = q.hkT = 0.0;
            g = ig = 1.0;
            return q;
        }
        g = redshift_omega_sc(y.r, sy, cy, a, a2, -L, v[3], ig);
        return grid_plasma(PR.grid, PR.torus.cJ, v);
    } else {
        return torus_plasma(PR.torus, y.r, cy, r_cap);
    }
}

// Persistent integrator over the rays of one chunk. MODEL selects the
// crossing-tracking models (geodesic, thin disk, disk images, hot spot) or a
// transfer model (torus, gridded plasma); NF bounds the number of frequencies
// carried in registers.
template <int MODEL, int NF>
__global__ void __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(WavesPerEU<MODEL, NF>::value, WavesPerEU<MODEL, NF>::value)))
trace_kernel(const KParams P, int64_t base, int64_t count, const double* __restrict__ rec, int64_t cap) {
    constexpr bool kRT = Transfer<MODEL>::value;
    constexpr bool kDisk = !kRT;
    // an optically thick disk seen through every crossing: refine each equatorial
    // crossing, end the ray at the first one on the disk (direct or higher-order image)
    constexpr bool kEvery = (MODEL == KGRT_MODEL_DISK_IMAGES);
    // the orbiting hot spot: no crossing tracking; the first accepted point inside
    // the spot starts a bisection of that step for the entry point
    constexpr bool kSpot = (MODEL == KGRT_MODEL_HOT_SPOT);
    constexpr bool kCross = kDisk && !kSpot;
    if (P.count_dev) count = std::max<int64_t>(0, std::min<int64_t>(count, *P.count_dev - base));
    const int lane = __lane_id();
    const uint64_t lane_mask_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    bool active = false, done = false, fresh = true;
    int64_t rid = 0;
    State y{};
    double h = 0.0, a = 0.0, a2 = 0.0, L = 0.0, r_cap = 0.0, r_in = 0.0, r_obs = 0.0;
    // sin(theta) (clamped, section 2.1) and cos(theta) of y, computed once per
    // point and shared by the first RHS stage, the redshift, the plasma and the
    // crossing test; syk, cyk those of the parked y_k+1 while a crossing is refined
    double sy = 0.0, cy = 0.0, syk = 0.0, cyk = 0.0;
    int32_t steps = 0, attempts = 0, status = 0;
    // crossing refinement (thin disk / geodesic): Newton iteration on the
    // step size from y_k, run in lockstep with the other lanes' attempts; the
    // accepted y_k+1 and the next adaptive step wait in yk and hs meanwhile
    bool crossed = false, refine = false;
    int32_t rit = 0, ncross = 0;
    double hs = 0.0;
    State yk{};
    // hot spot, per ray: observer time, the centre's angular velocity and its
    // pseudo-Cartesian cylindrical radius sqrt(r_s^2 + a^2); while a lane bisects,
    // yk holds the latest trial inside the spot, hs that trial's step and syk the
    // largest step known to end outside
    double t_obs = 0.0, om_s = 0.0, rho_c = 0.0;
    // per frequency: optical depth, intensity, attenuation e^-tau (carried as a
    // product of the steps' e^-dtau), coefficients at the last accepted point;
    // the first three in registers or in the thread's LDS slots
    // (slot (3 f + k) blockDim.x + threadIdx.x: consecutive lanes, consecutive words)
    constexpr bool kLds = AccInLds<NF>::value;
    extern __shared__ double acc_lds[];
    double tau[kLds ? 1 : NF], Iacc[kLds ? 1 : NF], att[kLds ? 1 : NF], ap[NF], ep[NF];
    double* const lds_t = acc_lds + threadIdx.x;  // slot of (f, k): lds_t[(3 f + k) blockDim.x]
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        ap[f] = ep[f] = 0.0;
        if constexpr (kLds) {
            lds_t[(3 * f) * blockDim.x] = lds_t[(3 * f + 1) * blockDim.x] = 0.0;
            lds_t[(3 * f + 2) * blockDim.x] = 1.0;
        } else {
            tau[f] = Iacc[f] = 0.0;
            att[f] = 1.0;
        }
    }
    const Outputs O = P.out;
    const int nf = P.nf;
    const int64_t nall = P.nrays;

    for (;;) {
        // ---- refill idle lanes from the chunk's ray queue
        const bool need = !active && !done;
        const uint64_t want = __ballot(need);
        if (want != 0ull) {
            const int cnt = __popcll(want);
            if (P.naive || cnt >= P.refill_min || __ballot(active) == 0ull) {
                unsigned long long qb = 0ull;
                if (!P.naive) {
                    const int leader = __ffsll((unsigned long long)want) - 1;
                    if (lane == leader) qb = atomicAdd(P.counter, (unsigned long long)cnt);
                    qb = __shfl(qb, leader);
                }
                if (need) {
                    unsigned long long my = qb + (unsigned long long)__popcll(want & lane_mask_lt);
                    if (P.naive) {
                        my = fresh ? (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x : ~0ull;
                        fresh = false;
                    }
                    if (my < (unsigned long long)count) {
                        const int64_t k = (int64_t)my;
                        rid = base + k;
                        y = State{rec[0 * cap + k], rec[1 * cap + k], rec[2 * cap + k], 0.0, rec[3 * cap + k],
                                  rec[4 * cap + k]};
                        L = rec[5 * cap + k];
                        a = rec[6 * cap + k];
                        a2 = a * a;
                        r_cap = rec[7 * cap + k];
                        r_in = rec[8 * cap + k];
                        r_obs = rec[9 * cap + k];
                        if (kSpot) {
                            t_obs = rec[10 * cap + k];
                            om_s = fm::rcp(fma(r_in, sqrt(r_in), a));  // 1/(r_s^3/2 + a), r_s in the r_in slot
                            rho_c = sqrt(fma(r_in, r_in, a2));
                        }
                        h = P.hmax_frac * r_obs;
                        steps = attempts = status = 0;
                        ncross = 0;
                        crossed = refine = false;
                        sincos_bounded(y.th, &sy, &cy);
                        sy = clamp_sin(sy);
                        if (isfinite(y.r)) {
                            active = true;
                            if (kRT) {
                                double ig0, g0 = 0.0;
                                if constexpr (MODEL == KGRT_MODEL_TORUS) g0 = redshift_sc(y.r, sy, cy, a, a2, -L, ig0);
                                const KParams& PR = reread_params();
                                const Plasma q = point_plasma<MODEL>(PR, y, sy, cy, a, a2, L, r_cap, g0, ig0);
#pragma unroll
                                for (int f = 0; f < NF; ++f) {
                                    if constexpr (kLds) {
                                        lds_t[(3 * f) * blockDim.x] = lds_t[(3 * f + 1) * blockDim.x] = 0.0;
                                        lds_t[(3 * f + 2) * blockDim.x] = 1.0;
                                    } else {
                                        tau[f] = 0.0;
                                        Iacc[f] = 0.0;
                                        att[f] = 1.0;
                                    }
                                    if (f < nf)
                                        torus_coeffs(q, PR.torus, g0, ig0, PR.freqs[f], PR.inv_freqs[f], ap[f], ep[f]);
                                }
                            }
                        } else {
                            // unusable start point: report and move on
                            if (O.status) O.status[rid] = ST_NONFINITE;
                            if (O.steps) O.steps[rid] = 0;
                            if (O.attempts) O.attempts[rid] = 0;
                            if (O.r_cross) O.r_cross[rid] = 0.0;
                            if (O.g) O.g[rid] = 0.0;
                            if (O.phi_cross) O.phi_cross[rid] = 0.0;
                            if (O.t_cross) O.t_cross[rid] = 0.0;
                            if (O.i_bol) O.i_bol[rid] = 0.0;
                            if (kEvery && O.n_cross) O.n_cross[rid] = 0;
                            if (kRT) {
                                for (int f = 0; f < nf; ++f) {
                                    if (O.intensity) O.intensity[(int64_t)f * nall + rid] = 0.0;
                                    if (O.tau) O.tau[(int64_t)f * nall + rid] = 0.0;
                                }
                            } else if (O.intensity) {
                                O.intensity[rid] = 0.0;
                            }
                        }
                    } else {
                        done = true;
                    }
                }
            }
        }
        if (__ballot(active || !done) == 0ull) break;
        if (!active) continue;

        // ---- one Cash-Karp evaluation (section 2.1) of size h from y: an adaptive
        // attempt, or, for a lane refining a crossing, a Newton trial step from y_k
        // (while refining, y holds y_k, yk holds the accepted y_k+1 and hs the next
        // adaptive step, so every lane starts from y with step h and no state is
        // selected per lane)
        bool terminate = false;
        const State k1 = rhs_sc(y, sy, cy, a, a2, L, h);
        State yn, ye;
        cash_karp(y, k1, h, a, a2, L, yn, ye);
        bool check_end = false;

        if (kSpot && refine) {
            // bisection of the step size for the spot's entry point (no error control)
            double sz, cz;
            sincos_bounded(yn.th, &sz, &cz);
            ++rit;
            if (spot_inside(yn, sz, cz, a2, t_obs, om_s, rho_c, P.spot_phi0, P.spot_cut2)) {
                yk = yn;
                hs = h;
            } else {
                syk = h;
            }
            if (rit == 48) {
                refine = false;
                double sk, ck;
                sincos_bounded(yk.th, &sk, &ck);
                const double j = fm::exp(-spot_d2(yk, sk, ck, a2, t_obs, om_s, rho_c, P.spot_phi0) * P.spot_inv_2s2);
                const double g = redshift_omega(yk.r, clamp_sin(sk), ck, a, a2, -L, om_s);
                status |= ST_SPOT_HIT;
                if (O.r_cross) O.r_cross[rid] = yk.r;
                if (O.g) O.g[rid] = g;
                if (O.phi_cross) O.phi_cross[rid] = yk.ph;
                if (O.t_cross) O.t_cross[rid] = t_obs + yk.t;  // emission time t_obs - Delta t
                if (O.intensity) O.intensity[rid] = g * g * g * j;
                if (O.i_bol) O.i_bol[rid] = g * g * g * g * j;
                terminate = true;
            } else {
                h = 0.5 * (syk + hs);
            }
        } else if (kCross && refine) {
            // Newton step on h* for cos(theta(h*)) = 0 (no error control)
            double sz, cz;
            sincos_bounded(yn.th, &sz, &cz);
            ++rit;
            if (fabs(cz) <= 1e-13 || rit == 7) {
                if (!(fabs(cz) <= 1e-13)) status |= ST_REFINE_UNCONVERGED;
                refine = false;
                const double rc = yn.r;
                if (kEvery) {
                    if (rc > r_cap) {
                        ++ncross;
                        if (rc >= r_in && rc <= P.r_out) {
                            // the first crossing on the disk: the ray ends there
                            status |= ST_CROSSED | ST_DISK_HIT;
                            const double g = redshift(rc, kPi / 2.0, a, a2, -L);
                            const double j = 1.0 / (rc * rc * rc);  // emissivity r^-3
                            if (O.r_cross) O.r_cross[rid] = rc;
                            if (O.g) O.g[rid] = g;
                            if (O.phi_cross) O.phi_cross[rid] = yn.ph;
                            if (O.t_cross) O.t_cross[rid] = yn.t;
                            if (O.intensity) O.intensity[rid] = g * g * g * j;
                            if (O.i_bol) O.i_bol[rid] = g * g * g * g * j;
                            terminate = true;
                        }
                    }
                } else if (rc > r_cap) {
                    status |= ST_CROSSED;
                    const double g = redshift(rc, kPi / 2.0, a, a2, -L);
                    double I = 0.0, Ib = 0.0;
                    if (P.model == KGRT_MODEL_THIN_DISK && rc >= r_in && rc <= P.r_out) {
                        status |= ST_DISK_HIT;
                        const double j = 1.0 / (rc * rc * rc);  // emissivity r^-3
                        I = g * g * g * j;
                        Ib = g * g * g * g * j;
                    }
                    if (O.r_cross) O.r_cross[rid] = rc;
                    if (O.g) O.g[rid] = g;
                    if (O.phi_cross) O.phi_cross[rid] = yn.ph;
                    if (O.t_cross) O.t_cross[rid] = yn.t;
                    if (O.intensity) O.intensity[rid] = I;
                    if (O.i_bol) O.i_bol[rid] = Ib;
                    if (P.flags & KGRT_STOP_AT_CROSSING) terminate = true;
                }
                // back to the accepted y_k+1, which still has to pass the end-of-step tests
                y = yk;
                sy = syk;
                cy = cyk;
                h = hs;
                check_end = !terminate;
            } else {
                const double thdot = yn.pth / (yn.r * yn.r + a2 * cz * cz);
                h = h + cz / (sz * thdot);
            }
        } else {
            ++attempts;
            double errmax = 0.0;
            {
                const double tol = P.rtol;
#define KGRT_ERR(f)                                                                   \
    {                                                                                 \
        const double e = fabs(ye.f) * fm::rcp_coarse(tol * (fabs(y.f) + fabs(k1.f) + 1e-12)); \
        if (e > errmax) errmax = e;                                                   \
    }
                KGRT_ERR(r) KGRT_ERR(th) KGRT_ERR(ph) KGRT_ERR(t) KGRT_ERR(pr) KGRT_ERR(pth)
#undef KGRT_ERR
            }
            if (!(errmax <= 1.0)) {
                // rejected: shrink and retry
                if (!isfinite(errmax)) errmax = 1e10;
                double shrink = 0.9 * fm::pow_m025(errmax);
                if (shrink < 0.1) shrink = 0.1;
                h = h * shrink;
                if (fabs(h) < 1e-12 * fmax(1.0, y.r)) {
                    status |= ST_UNDERFLOW;
                    terminate = true;
                }
            } else {
                // accepted: y_k -> y_k+1 over [lambda, lambda + hdone]
                const double hdone = h;
                double hnext = (errmax > 1.89e-4) ? h * (0.9 * fm::pow_m02(errmax)) : h * 5.0;
                ++steps;
                const double c0 = cy;  // cos(theta) at y_k
                double sn, cn;
                sincos_bounded(yn.th, &sn, &cn);
                sn = clamp_sin(sn);
                bool start_refine = false;
                if (!finite6(yn)) {
                    y = yn;
                    status |= ST_NONFINITE;
                    terminate = true;
                } else if (kCross && (kEvery || !crossed) && ((c0 > 0.0 && cn <= 0.0) || (c0 < 0.0 && cn >= 0.0))) {
                    // first equatorial crossing inside this step: park y_k+1 and refine from
                    // y_k over the next evaluations, starting from linear interpolation of cos(theta)
                    crossed = true;
                    refine = true;
                    start_refine = true;
                    rit = 0;
                    yk = yn;
                    syk = sn;
                    cyk = cn;
                    const double hcap = P.hmax_frac * yn.r;
                    hs = (hnext > hcap) ? hcap : hnext;
                    h = hdone * c0 / (c0 - cn);
                } else if (kSpot && spot_inside(yn, sn, cn, a2, t_obs, om_s, rho_c, P.spot_phi0, P.spot_cut2)) {
                    // the step ends inside the spot: bisect [0, hdone] from y_k for the entry
                    refine = true;
                    start_refine = true;
                    rit = 0;
                    yk = yn;
                    hs = hdone;
                    syk = 0.0;
                    h = 0.5 * hdone;
                } else {
                    y = yn;
                    sy = sn;
                    cy = cn;
                    check_end = true;
                    if (kRT) {
                        // transfer over the accepted step (Eqs. (30)-(31)): coefficients at
                        // each accepted endpoint, exponential-trapezoid increment
                        double ig1, g1 = 0.0;
                        if constexpr (MODEL == KGRT_MODEL_TORUS) g1 = redshift_sc(y.r, sy, cy, a, a2, -L, ig1);
                        const KParams& PR = reread_params();
                        const Plasma q = point_plasma<MODEL>(PR, y, sy, cy, a, a2, L, r_cap, g1, ig1);
#pragma unroll
                        for (int f = 0; f < NF; ++f) {
                            if (f < nf) {
                                double a1, e1;
                                torus_coeffs(q, PR.torus, g1, ig1, PR.freqs[f], PR.inv_freqs[f], a1, e1);
                                const double dtau = hdone * (ap[f] + a1) / 2.0;
                                const double em = fm::expm1(-dtau);  // e^-dtau - 1
                                const double phi = (dtau > 0.0) ? -em * fm::rcp(dtau) : 1.0;
                                if constexpr (kLds) {
                                    double* const t = lds_t + (3 * f) * blockDim.x;
                                    const double at = t[2 * blockDim.x];
                                    t[blockDim.x] += at * hdone * (ep[f] + e1) / 2.0 * phi;
                                    t[0] += dtau;
                                    t[2 * blockDim.x] = at + at * em;
                                } else {
                                    Iacc[f] += att[f] * hdone * (ep[f] + e1) / 2.0 * phi;
                                    tau[f] += dtau;
                                    att[f] += att[f] * em;
                                }
                                ap[f] = a1;
                                ep[f] = e1;
                            }
                        }
                    }
                }
                if (!start_refine) {
                    const double hcap = P.hmax_frac * y.r;
                    if (hnext > hcap) hnext = hcap;
                    h = hnext;
                }
            }
        }
        if (check_end) {
            if (y.r <= r_cap) {
                status |= ST_CAPTURED;
                terminate = true;
            } else if (y.pr > 0.0 && y.r > r_obs) {
                status |= ST_ESCAPED;
                terminate = true;
            } else if (steps >= P.max_steps) {
                status |= ST_MAXSTEPS;
                terminate = true;
            }
        }

        if (terminate) {
            if (O.status) O.status[rid] = status;
            if (O.steps) O.steps[rid] = steps;
            if (O.attempts) O.attempts[rid] = attempts;
            if (kEvery && O.n_cross) O.n_cross[rid] = ncross;
            if (kRT) {
                for (int f = 0; f < NF; ++f) {
                    if (f < nf) {
                        const double If = kLds ? lds_t[(3 * f + 1) * blockDim.x] : Iacc[kLds ? 0 : f];
                        const double tf = kLds ? lds_t[(3 * f) * blockDim.x] : tau[kLds ? 0 : f];
                        if (O.intensity) O.intensity[(int64_t)f * nall + rid] = If;
                        if (O.tau) O.tau[(int64_t)f * nall + rid] = tf;
                    }
                }
            }
            if (!(status & (ST_CROSSED | ST_SPOT_HIT))) {
                if (O.r_cross) O.r_cross[rid] = 0.0;
                if (O.g) O.g[rid] = 0.0;
                if (O.phi_cross) O.phi_cross[rid] = 0.0;
                if (O.t_cross) O.t_cross[rid] = 0.0;
                if (O.i_bol) O.i_bol[rid] = 0.0;
                if (!kRT && O.intensity) O.intensity[rid] = 0.0;
            }
            active = false;
        }
    }
}

}  // namespace kgrt

// =================================================================== host

using namespace kgrt;

// Scratch of the allocation-free trace (kgrt_trace_noalloc): the work-queue
// counter in the first 256 bytes, then the ray-start records of at most
// KGRT_NOALLOC_MAX_RAYS rays, [kRecFields][KGRT_NOALLOC_MAX_RAYS]. Every device
// the library is loaded on holds its own copy until the process ends (23 MB).
// Host code never uses the array's name as an address: its device address is
// taken once per device with hipGetSymbolAddress (noalloc_scratch below).
namespace kgrt {
constexpr int64_t kNoAllocLead = 32;  // doubles before the records (the counter's 256 bytes)
static_assert(KGRT_NOALLOC_MAX_RAYS % 64 == 0, "record planes stay 512-byte aligned");
__device__ __align__(256) double scratch[kNoAllocLead + kRecFields * (int64_t)KGRT_NOALLOC_MAX_RAYS];
}  // namespace kgrt

struct kgrt_ctx {
    int device = 0;
    int num_cus = 0;
    double* scratch = nullptr;  // this device's copy of kgrt::scratch (device address), or NULL
    unsigned long long* counter = nullptr;
    double* rec = nullptr;  // ray start records of one chunk, [kRecFields][rec_cap]
    int64_t rec_cap = 0;
    int64_t chunk_max = int64_t(1) << 22;  // rays per chunk (4 Mi rays -> 320 MiB of records)
    kgrt_launch launch{};
    std::string last_error;
};

namespace {

int fail(kgrt_ctx* ctx, int code, const std::string& msg) {
    if (ctx) ctx->last_error = msg;
    return code;
}

bool is_finite(double v) { return std::isfinite(v); }

// Argument checks shared by every entry point (see include/kgrt.h).
int check(std::string& msg, const kgrt_camera* cam, const kgrt_model* m, const double* freqs, int32_t nfreq,
          const kgrt_integrator* in) {
    if (cam) {
        if (!(std::fabs(cam->a) < 1.0)) { msg = "camera.a must satisfy |a| < 1"; return KGRT_E_INVALID_ARG; }
        if (!(cam->incl_deg > 0.0 && cam->incl_deg < 180.0)) { msg = "camera.incl_deg must be in (0, 180)"; return KGRT_E_INVALID_ARG; }
        if (!is_finite(cam->phi_obs_deg)) { msg = "camera.phi_obs_deg must be finite"; return KGRT_E_INVALID_ARG; }
        const double rplus = 1.0 + std::sqrt(1.0 - cam->a * cam->a);
        if (!(is_finite(cam->r_obs) && cam->r_obs > 10.0 * rplus)) { msg = "camera.r_obs must exceed 10 r_+"; return KGRT_E_INVALID_ARG; }
        if (cam->nx < 0 || cam->ny < 0) { msg = "camera.nx, ny must be >= 0"; return KGRT_E_INVALID_ARG; }
        if (!(is_finite(cam->x_min) && is_finite(cam->x_max) && cam->x_min < cam->x_max)) { msg = "camera x extent invalid"; return KGRT_E_INVALID_ARG; }
        if (!(is_finite(cam->y_min) && is_finite(cam->y_max) && cam->y_min < cam->y_max)) { msg = "camera y extent invalid"; return KGRT_E_INVALID_ARG; }
        if (!is_finite(cam->t_obs)) { msg = "camera.t_obs must be finite"; return KGRT_E_INVALID_ARG; }
    }
    if (!m) { msg = "model is NULL"; return KGRT_E_INVALID_ARG; }
    if (m->reserved != 0) { msg = "model.reserved must be 0"; return KGRT_E_INVALID_ARG; }
    if (m->kind == KGRT_MODEL_HOT_SPOT) {
        if (!(is_finite(m->spot_size) && m->spot_size > 0.0)) { msg = "model.spot_size must be finite and > 0"; return KGRT_E_INVALID_ARG; }
        if (!is_finite(m->spot_r) || !is_finite(m->spot_phi0)) { msg = "model.spot_r and spot_phi0 must be finite"; return KGRT_E_INVALID_ARG; }
    }
    if (m->kind == KGRT_MODEL_THIN_DISK || m->kind == KGRT_MODEL_GEODESIC || m->kind == KGRT_MODEL_DISK_IMAGES ||
        m->kind == KGRT_MODEL_HOT_SPOT) {
        if (m->kind != KGRT_MODEL_GEODESIC && m->kind != KGRT_MODEL_HOT_SPOT) {
            if (!(is_finite(m->r_out) && m->r_out > 0.0)) { msg = "model.r_out must be finite and > 0"; return KGRT_E_INVALID_ARG; }
            if (!is_finite(m->r_in) || (m->r_in > 0.0 && !(m->r_in < m->r_out))) { msg = "model.r_in must be <= 0 or < r_out"; return KGRT_E_INVALID_ARG; }
        }
    } else if (m->kind == KGRT_MODEL_GRID) {
        if (!m->grid_dev) { msg = "model.grid_dev is NULL"; return KGRT_E_INVALID_ARG; }
        if ((uintptr_t)m->grid_dev % 16 != 0) { msg = "model.grid_dev must be 16-byte aligned"; return KGRT_E_INVALID_ARG; }
        if (m->grid_reserved != 0) { msg = "model.grid_reserved must be 0"; return KGRT_E_INVALID_ARG; }
        if (m->grid_nr < 2 || m->grid_nth < 2 || m->grid_nph < 1) { msg = "grid needs grid_nr >= 2, grid_nth >= 2, grid_nph >= 1"; return KGRT_E_INVALID_ARG; }
        if ((int64_t)m->grid_nr * m->grid_nth * m->grid_nph >= (int64_t(1) << 31)) { msg = "grid has 2^31 or more nodes"; return KGRT_E_INVALID_ARG; }
        if (!(is_finite(m->grid_r_min) && is_finite(m->grid_r_max) && m->grid_r_min > 0.0 && m->grid_r_min < m->grid_r_max)) { msg = "grid radii must satisfy 0 < grid_r_min < grid_r_max"; return KGRT_E_INVALID_ARG; }
        if (!(is_finite(m->mbh_msun) && m->mbh_msun > 0.0)) { msg = "model.mbh_msun must be finite and > 0"; return KGRT_E_INVALID_ARG; }
        if (nfreq < 1 || nfreq > 16) { msg = "the gridded plasma needs 1 <= nfreq <= 16"; return KGRT_E_INVALID_ARG; }
        if (!freqs) { msg = "freqs_hz is NULL"; return KGRT_E_INVALID_ARG; }
        for (int f = 0; f < nfreq; ++f)
            if (!(is_finite(freqs[f]) && freqs[f] > 0.0)) { msg = "frequencies must be finite and > 0"; return KGRT_E_INVALID_ARG; }
    } else if (m->kind == KGRT_MODEL_TORUS) {
        const double v[9] = {m->n0_cgs, m->r_norm, m->n_index, m->h_over_r, m->T0_K, m->T_index, m->eps_B, m->mbh_msun, m->r_emit_max};
        for (double x : v) if (!is_finite(x)) { msg = "torus parameters must be finite"; return KGRT_E_INVALID_ARG; }
        if (!(m->n0_cgs >= 0.0 && m->r_norm > 0.0 && m->h_over_r > 0.0 && m->T0_K > 0.0 && m->eps_B >= 0.0 &&
              m->mbh_msun > 0.0 && m->r_emit_max > 0.0)) { msg = "torus parameters out of range"; return KGRT_E_INVALID_ARG; }
        if (nfreq < 1 || nfreq > 16) { msg = "torus needs 1 <= nfreq <= 16"; return KGRT_E_INVALID_ARG; }
        if (!freqs) { msg = "freqs_hz is NULL"; return KGRT_E_INVALID_ARG; }
        for (int f = 0; f < nfreq; ++f)
            if (!(is_finite(freqs[f]) && freqs[f] > 0.0)) { msg = "frequencies must be finite and > 0"; return KGRT_E_INVALID_ARG; }
    } else {
        msg = "unknown model.kind";
        return KGRT_E_INVALID_ARG;
    }
    if (!in) { msg = "integrator is NULL"; return KGRT_E_INVALID_ARG; }
    if (!(in->rtol >= 1e-14 && in->rtol <= 1e-2)) { msg = "integrator.rtol must be in [1e-14, 1e-2]"; return KGRT_E_INVALID_ARG; }
    if (!(in->hmax_frac > 0.0 && in->hmax_frac <= 1.0)) { msg = "integrator.hmax_frac must be in (0, 1]"; return KGRT_E_INVALID_ARG; }
    if (!(in->horizon_delta > 0.0 && in->horizon_delta <= 0.5)) { msg = "integrator.horizon_delta must be in (0, 0.5]"; return KGRT_E_INVALID_ARG; }
    if (in->max_steps < 1) { msg = "integrator.max_steps must be >= 1"; return KGRT_E_INVALID_ARG; }
    if (in->flags & ~KGRT_STOP_AT_CROSSING) { msg = "unknown integrator flags"; return KGRT_E_INVALID_ARG; }
    return KGRT_OK;
}

ImageDesc make_image(const kgrt_camera* c, const kgrt_model* m, double horizon_delta, int64_t offset) {
    // Same host libm as any CPU reference, computed once per image.
    ImageDesc d{};
    const double pi = 3.14159265358979323846;
    const double tho = c->incl_deg * pi / 180.0, pho = c->phi_obs_deg * pi / 180.0;
    d.a = c->a;
    d.a2 = c->a * c->a;
    d.r_obs = c->r_obs;
    d.sqrt_ro2a2 = std::sqrt(c->r_obs * c->r_obs + c->a * c->a);
    d.sin_i = std::sin(tho);
    d.cos_i = std::cos(tho);
    d.sin_p = std::sin(pho);
    d.cos_p = std::cos(pho);
    d.phi_obs = pho;
    d.x_min = c->x_min;
    d.x_w = c->x_max - c->x_min;
    d.y_min = c->y_min;
    d.y_w = c->y_max - c->y_min;
    d.r_cap = (1.0 + std::sqrt(1.0 - c->a * c->a)) * (1.0 + horizon_delta);
    const double r_in_c = (m->kind == KGRT_MODEL_HOT_SPOT) ? m->spot_r : m->r_in;
    d.r_in = (r_in_c > 0.0) ? r_in_c : isco_radius(c->a);
    d.t_obs = c->t_obs;
    d.ray_offset = offset;
    d.nx = c->nx;
    d.ny = c->ny;
    return d;
}

void set_outputs(KParams& P, const kgrt_outputs* o) {
    P.out = Outputs{o->status, o->steps, o->attempts, o->r_cross, o->g, o->phi_cross, o->t_cross,
                    o->intensity, o->i_bol, o->tau, o->n_cross};
}

void fill_common(KParams& P, const kgrt_model* m, const double* freqs, int32_t nfreq, const kgrt_integrator* in,
                 const kgrt_outputs* o, const kgrt_ctx* ctx) {
    P.model = m->kind;
    P.nf = (m->kind == KGRT_MODEL_TORUS || m->kind == KGRT_MODEL_GRID) ? nfreq : 0;
    for (int f = 0; f < 16; ++f) P.freqs[f] = (f < P.nf) ? freqs[f] : 0.0;
    P.r_in_cfg = m->r_in;
    P.r_out = m->r_out;
    P.spot_r_cfg = m->spot_r;
    P.spot_phi0 = m->spot_phi0;
    P.spot_cut2 = 16.0 * m->spot_size * m->spot_size;
    P.spot_inv_2s2 = (m->spot_size > 0.0) ? 1.0 / (2.0 * m->spot_size * m->spot_size) : 0.0;
    TorusParams& T = P.torus;
    T.n0 = m->n0_cgs;
    T.inv_rnorm = (m->r_norm > 0.0) ? 1.0 / m->r_norm : 0.0;
    T.n_index = m->n_index;
    T.inv_2h2 = (m->h_over_r > 0.0) ? 1.0 / (2.0 * m->h_over_r * m->h_over_r) : 0.0;
    T.T0 = m->T0_K;
    T.T_index = m->T_index;
    T.eps_B = m->eps_B;
    T.rg = kGMsun * m->mbh_msun / (kC * kC);
    T.r_emit_max = m->r_emit_max;
    T.cB = 8.0 * kPi * T.eps_B * kMp * kC * kC / 6.0;
    T.cTheta = kKb * T.T0 / (kMe * kC * kC);
    T.cInvTheta = (T.T0 > 0.0) ? 1.0 / T.cTheta : 0.0;
    T.cLnHalfInvTheta = (T.T0 > 0.0) ? std::log(0.5 * T.cInvTheta) : 0.0;
    T.cNu = 3.0 * kQe / (4.0 * kPi * kMe * kC);
    T.cNuC = T.cB * T.cNu * T.cNu * (T.cTheta * T.cTheta) * (T.cTheta * T.cTheta);
    T.cJ = kQe * kQe / (1.7320508075688772 * kC);
    T.cH = (T.T0 > 0.0) ? kH / (kKb * T.T0) : 0.0;
    T.cBnu = kC * kC / (2.0 * kH);
    for (int f = 0; f < 16; ++f) P.inv_freqs[f] = (f < P.nf && freqs[f] > 0.0) ? 1.0 / freqs[f] : 0.0;
    GridParams& G = P.grid;
    G = GridParams{};
    if (m->kind == KGRT_MODEL_GRID) {
        G.nodes = (const float4*)m->grid_dev;
        G.nr = m->grid_nr;
        G.nth = m->grid_nth;
        G.nph = m->grid_nph;
        G.r_min = m->grid_r_min;
        G.r_max = m->grid_r_max;
        G.ln_rmin = std::log(m->grid_r_min);
        G.u1_scale = (m->grid_nr - 1) / (std::log(m->grid_r_max) - std::log(m->grid_r_min));
        G.u2_scale = (m->grid_nth - 1) / kPi;
        G.u3_scale = m->grid_nph / (2.0 * kPi);
        G.inv_nph = 1.0 / m->grid_nph;
        G.ln_theta1 = std::log(kKb / (kMe * kC * kC));
        G.inv_cnu = 1.0 / T.cNu;
        G.h_mec2 = kH / (kMe * kC * kC);
    }
    P.rtol = in->rtol;
    P.hmax_frac = in->hmax_frac;
    P.horizon_delta = in->horizon_delta;
    P.max_steps = in->max_steps;
    P.flags = in->flags;
    if (o) set_outputs(P, o);
}

// Grows the ray-start workspace to hold `n` rays (capped at one chunk).
// Allocation happens here, outside any stream work, so it is never captured.
int ensure_workspace(kgrt_ctx* ctx, int64_t n) {
    const int64_t want = std::min<int64_t>(n, ctx->chunk_max);
    if (want <= ctx->rec_cap) return KGRT_OK;
    if (ctx->rec) {
        if (hipDeviceSynchronize() != hipSuccess) return fail(ctx, KGRT_E_HIP, "hipDeviceSynchronize failed");
        (void)hipFree(ctx->rec);
        ctx->rec = nullptr;
        ctx->rec_cap = 0;
    }
    if (hipMalloc(&ctx->rec, (size_t)want * kRecFields * sizeof(double)) != hipSuccess) {
        ctx->rec = nullptr;
        return fail(ctx, KGRT_E_NOMEM, "cannot allocate the ray-start workspace");
    }
    ctx->rec_cap = want;
    return KGRT_OK;
}

// Where one trace's kernels run: workspace, counter and launch shape.
struct LaunchEnv {
    double* rec;
    int64_t rec_cap;
    unsigned long long* counter;
    kgrt_launch launch;
    int num_cus;
    int64_t limit;  // trace only the first `limit` rays (autotuner sampling); < 0 = all
};

template <int MODEL, int NF>
int launch_one(kgrt_ctx* ctx, const LaunchEnv& env, KParams P, hipStream_t st) {
    const int block = (env.launch.block == 64 || env.launch.block == 128) ? env.launch.block : 256;
    auto kern = trace_kernel<MODEL, NF>;
    const size_t shmem = acc_lds_bytes<NF>(block);
    int per_cu = env.launch.blocks_per_cu;
    if (per_cu <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, shmem) != hipSuccess || per_cu <= 0)
            per_cu = 1;
        if (RayCountResidency<NF>::value && Transfer<MODEL>::value) {
            // the residency of two waves per SIMD when three would leave too few rays per lane;
            // decided on the whole plan, also when the autotuner times a prefix of it, so the
            // residency it times is the one the plan launches
            const int64_t rays = P.nrays;
            const int two_waves = std::max(1, (2 * 4 * 64) / block);  // blocks per CU at two waves per SIMD
            if (per_cu > two_waves && rays < (int64_t)kMinRaysPerLane * env.num_cus * per_cu * block)
                per_cu = two_waves;
        }
    }
    P.counter = env.counter;
    P.naive = (env.launch.mode == KGRT_LAUNCH_ONE_RAY_PER_THREAD) ? 1 : 0;
    P.refill_min = (env.launch.refill_min >= 1 && env.launch.refill_min <= 64) ? env.launch.refill_min
                                                                                : DefaultRefill<MODEL, NF>::value;
    const int64_t total = (env.limit >= 0) ? std::min<int64_t>(env.limit, P.nrays) : P.nrays;
    const int64_t cap = env.rec_cap;
    for (int64_t base = 0; base < total; base += cap) {
        const int64_t count = std::min<int64_t>(cap, total - base);
        const int64_t need = (count + block - 1) / block;
        const int grid = P.naive ? (int)need
                                 : (int)std::max<int64_t>(1, std::min<int64_t>(need, (int64_t)env.num_cus * per_cu));
        const int sgrid = (int)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, (int64_t)env.num_cus * 16));
        hipLaunchKernelGGL(reset_counter, dim3(1), dim3(1), 0, st, env.counter);
        hipLaunchKernelGGL(start_kernel, dim3(sgrid), dim3(256), 0, st, P, base, count, env.rec, cap);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(block), shmem, st, P, base, count, (const double*)env.rec, cap);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(ctx, KGRT_E_HIP, std::string("kernel launch failed: ") + hipGetErrorString(e));
    }
    return KGRT_OK;
}

int dispatch_env(kgrt_ctx* ctx, const LaunchEnv& env, const KParams& P, hipStream_t st) {
    if (P.model == KGRT_MODEL_DISK_IMAGES) return launch_one<KGRT_MODEL_DISK_IMAGES, 1>(ctx, env, P, st);
    if (P.model == KGRT_MODEL_HOT_SPOT) return launch_one<KGRT_MODEL_HOT_SPOT, 1>(ctx, env, P, st);
    if (P.model == KGRT_MODEL_GRID) {
        if (P.nf <= 1) return launch_one<KGRT_MODEL_GRID, 1>(ctx, env, P, st);
        if (P.nf <= 2) return launch_one<KGRT_MODEL_GRID, 2>(ctx, env, P, st);
        if (P.nf <= 4) return launch_one<KGRT_MODEL_GRID, 4>(ctx, env, P, st);
        if (P.nf <= 8) return launch_one<KGRT_MODEL_GRID, 8>(ctx, env, P, st);
        return launch_one<KGRT_MODEL_GRID, 16>(ctx, env, P, st);
    }
    if (P.model != KGRT_MODEL_TORUS) return launch_one<KGRT_MODEL_THIN_DISK, 1>(ctx, env, P, st);
    if (P.nf <= 1) return launch_one<KGRT_MODEL_TORUS, 1>(ctx, env, P, st);
    if (P.nf <= 2) return launch_one<KGRT_MODEL_TORUS, 2>(ctx, env, P, st);
    if (P.nf <= 4) return launch_one<KGRT_MODEL_TORUS, 4>(ctx, env, P, st);
    if (P.nf <= 8) return launch_one<KGRT_MODEL_TORUS, 8>(ctx, env, P, st);
    return launch_one<KGRT_MODEL_TORUS, 16>(ctx, env, P, st);
}

int dispatch(kgrt_ctx* ctx, const KParams& P, hipStream_t st) {
    const int rc = ensure_workspace(ctx, P.nrays);
    if (rc != KGRT_OK) return rc;
    const LaunchEnv env{ctx->rec, ctx->rec_cap, ctx->counter, ctx->launch, ctx->num_cus, -1};
    return dispatch_env(ctx, env, P, st);
}

template <int MODEL, int NF>
int kernel_info(int block, kgrt_kernel_info* out) {
    auto kern = trace_kernel<MODEL, NF>;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, (const void*)kern) != hipSuccess) return KGRT_E_HIP;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, acc_lds_bytes<NF>(block)) != hipSuccess)
        return KGRT_E_HIP;
    out->vgprs = fa.numRegs;
    out->scratch_bytes = (int32_t)fa.localSizeBytes;
    out->blocks_per_cu = per_cu;
    out->waves_per_simd = per_cu * (block / 64) / 4;  // four SIMDs per compute unit
    return KGRT_OK;
}

// The device address of this device's copy of the no-alloc scratch, looked up
// once per device (the caller has made `device` current). NULL if the lookup
// failed; the allocation-free entry point then reports the error.
double* noalloc_scratch(int device) {
    static std::mutex mu;
    static double* addr[256] = {};
    static bool tried[256] = {};
    if (device < 0 || device >= 256) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!tried[device]) {
        tried[device] = true;
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(kgrt::scratch)) == hipSuccess) addr[device] = (double*)p;
        else (void)hipGetLastError();  // clear the failed lookup's error
    }
    return addr[device];
}

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = (prev == dev) || hipSetDevice(dev) == hipSuccess;
        if (!ok) (void)hipGetLastError();  // leave no sticky error behind for the caller's runtime
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

int kgrt_version(void) { return 200; }

const char* kgrt_strerror(int code) {
    switch (code) {
        case KGRT_OK: return "ok";
        case KGRT_E_INVALID_ARG: return "invalid argument";
        case KGRT_E_HIP: return "HIP runtime error";
        case KGRT_E_NOMEM: return "out of memory";
        case KGRT_E_NO_DEVICE: return "no usable GPU";
        case KGRT_E_UNSUPPORTED: return "unsupported request";
        default: return "unknown error";
    }
}

const char* kgrt_last_error(const kgrt_ctx* ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int kgrt_kernel_info_get(kgrt_ctx* ctx, int32_t model, int32_t nfreq, int32_t block, kgrt_kernel_info* out) {
    if (!ctx || !out) return KGRT_E_INVALID_ARG;
    if (block == 0) block = 256;
    if (block != 64 && block != 128 && block != 256) return fail(ctx, KGRT_E_INVALID_ARG, "block must be 64, 128 or 256");
    if (model < KGRT_MODEL_GEODESIC || model > KGRT_MODEL_GRID) return fail(ctx, KGRT_E_INVALID_ARG, "unknown model");
    if ((model == KGRT_MODEL_TORUS || model == KGRT_MODEL_GRID) && (nfreq < 1 || nfreq > 16))
        return fail(ctx, KGRT_E_INVALID_ARG, "nfreq must be 1..16");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    int rc;
    if (model == KGRT_MODEL_DISK_IMAGES) rc = kernel_info<KGRT_MODEL_DISK_IMAGES, 1>(block, out);
    else if (model == KGRT_MODEL_HOT_SPOT) rc = kernel_info<KGRT_MODEL_HOT_SPOT, 1>(block, out);
    else if (model == KGRT_MODEL_GRID) {
        if (nfreq <= 1) rc = kernel_info<KGRT_MODEL_GRID, 1>(block, out);
        else if (nfreq <= 2) rc = kernel_info<KGRT_MODEL_GRID, 2>(block, out);
        else if (nfreq <= 4) rc = kernel_info<KGRT_MODEL_GRID, 4>(block, out);
        else if (nfreq <= 8) rc = kernel_info<KGRT_MODEL_GRID, 8>(block, out);
        else rc = kernel_info<KGRT_MODEL_GRID, 16>(block, out);
    } else if (model != KGRT_MODEL_TORUS) rc = kernel_info<KGRT_MODEL_THIN_DISK, 1>(block, out);
    else if (nfreq <= 1) rc = kernel_info<KGRT_MODEL_TORUS, 1>(block, out);
    else if (nfreq <= 2) rc = kernel_info<KGRT_MODEL_TORUS, 2>(block, out);
    else if (nfreq <= 4) rc = kernel_info<KGRT_MODEL_TORUS, 4>(block, out);
    else if (nfreq <= 8) rc = kernel_info<KGRT_MODEL_TORUS, 8>(block, out);
    else rc = kernel_info<KGRT_MODEL_TORUS, 16>(block, out);
    return rc == KGRT_OK ? KGRT_OK : fail(ctx, rc, "kernel attribute query failed");
}

int kgrt_check_args(const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                    const kgrt_integrator* integ) {
    std::string msg;
    return check(msg, cam, model, freqs_hz, nfreq, integ);
}

int kgrt_ctx_create(int device, kgrt_ctx** out) {
    if (!out) return KGRT_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return KGRT_E_NO_DEVICE;
    if (device < 0 || device >= n) return KGRT_E_NO_DEVICE;
    auto* ctx = new (std::nothrow) kgrt_ctx();
    if (!ctx) return KGRT_E_NOMEM;
    ctx->device = device;
    DeviceGuard g(device);
    if (!g.ok) { delete ctx; return KGRT_E_NO_DEVICE; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return KGRT_E_HIP; }
    ctx->num_cus = prop.multiProcessorCount;
    ctx->scratch = noalloc_scratch(device);
    if (hipMalloc(&ctx->counter, sizeof(unsigned long long)) != hipSuccess) { delete ctx; return KGRT_E_NOMEM; }
    *out = ctx;
    return KGRT_OK;
}

int kgrt_ctx_destroy(kgrt_ctx* ctx) {
    if (!ctx) return KGRT_OK;
    {
        DeviceGuard g(ctx->device);
        if (ctx->counter) (void)hipFree(ctx->counter);
        if (ctx->rec) (void)hipFree(ctx->rec);
    }
    delete ctx;
    return KGRT_OK;
}

int kgrt_ctx_set_launch(kgrt_ctx* ctx, const kgrt_launch* l) {
    if (!ctx) return KGRT_E_INVALID_ARG;
    if (!l) { ctx->launch = kgrt_launch{}; return KGRT_OK; }
    if (!(l->block == 0 || l->block == 64 || l->block == 128 || l->block == 256 || l->block == 512))
        return fail(ctx, KGRT_E_INVALID_ARG, "launch.block must be 0, 64, 128, 256 or 512");
    if (l->block == 512) return fail(ctx, KGRT_E_UNSUPPORTED, "launch.block 512 exceeds the kernel's launch bounds");
    if (l->blocks_per_cu < 0 || l->blocks_per_cu > 64) return fail(ctx, KGRT_E_INVALID_ARG, "launch.blocks_per_cu must be in [0, 64]");
    if (l->refill_min < 0 || l->refill_min > 64) return fail(ctx, KGRT_E_INVALID_ARG, "launch.refill_min must be in [0, 64]");
    if (l->mode != KGRT_LAUNCH_PERSISTENT && l->mode != KGRT_LAUNCH_ONE_RAY_PER_THREAD)
        return fail(ctx, KGRT_E_INVALID_ARG, "launch.mode must be KGRT_LAUNCH_PERSISTENT or KGRT_LAUNCH_ONE_RAY_PER_THREAD");
    ctx->launch = *l;
    return KGRT_OK;
}

int kgrt_ctx_num_cus(const kgrt_ctx* ctx) { return ctx ? ctx->num_cus : 0; }

int kgrt_trace(kgrt_ctx* ctx, const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
               const kgrt_integrator* integ, const kgrt_outputs* out, void* stream) {
    if (!ctx) return KGRT_E_INVALID_ARG;
    if (!cam) return fail(ctx, KGRT_E_INVALID_ARG, "camera is NULL");
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "outputs is NULL");
    std::string msg;
    int rc = check(msg, cam, model, freqs_hz, nfreq, integ);
    if (rc != KGRT_OK) return fail(ctx, rc, msg);
    const int64_t n = (int64_t)cam->nx * (int64_t)cam->ny;
    if (n == 0) return KGRT_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    KParams P{};
    P.image0 = make_image(cam, model, integ->horizon_delta, 0);
    P.images = nullptr;
    P.nimg = 1;
    P.list_mode = 0;
    P.nrays = n;
    fill_common(P, model, freqs_hz, nfreq, integ, out, ctx);
    return dispatch(ctx, P, (hipStream_t)stream);
}

int kgrt_trace_noalloc(kgrt_ctx* ctx, const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz,
                       int32_t nfreq, const kgrt_integrator* integ, const kgrt_outputs* out, void* stream) {
    if (!ctx) return KGRT_E_INVALID_ARG;
    if (!cam) return fail(ctx, KGRT_E_INVALID_ARG, "camera is NULL");
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "outputs is NULL");
    std::string msg;
    int rc = check(msg, cam, model, freqs_hz, nfreq, integ);
    if (rc != KGRT_OK) return fail(ctx, rc, msg);
    const int64_t n = (int64_t)cam->nx * (int64_t)cam->ny;
    if (n > KGRT_NOALLOC_MAX_RAYS)
        return fail(ctx, KGRT_E_INVALID_ARG, "kgrt_trace_noalloc: the image has " + std::to_string(n) +
                                                 " rays, more than the scratch holds (KGRT_NOALLOC_MAX_RAYS = " +
                                                 std::to_string((long long)KGRT_NOALLOC_MAX_RAYS) + ")");
    if (!ctx->scratch) return fail(ctx, KGRT_E_HIP, "kgrt_trace_noalloc: no device address for the scratch array");
    if (n == 0) return KGRT_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    KParams P{};
    P.image0 = make_image(cam, model, integ->horizon_delta, 0);
    P.images = nullptr;
    P.nimg = 1;
    P.list_mode = 0;
    P.nrays = n;
    fill_common(P, model, freqs_hz, nfreq, integ, out, ctx);
    // the same kernels as kgrt_trace, on the static scratch: the counter is cleared by a
    // kernel and the start records are written before they are read, on `stream`
    const LaunchEnv env{ctx->scratch + kNoAllocLead, KGRT_NOALLOC_MAX_RAYS, (unsigned long long*)ctx->scratch,
                        ctx->launch, ctx->num_cus, -1};
    return dispatch_env(ctx, env, P, (hipStream_t)stream);
}

int kgrt_trace_rays_dev(kgrt_ctx* ctx, const double* rays_dev, const int64_t* n_dev, int64_t n_max, double r_obs,
                        double phi_obs_deg, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                        const kgrt_integrator* integ, const kgrt_outputs* out, void* stream);

int kgrt_trace_rays(kgrt_ctx* ctx, const double* rays_dev, int64_t n, double r_obs, double phi_obs_deg,
                    const kgrt_model* model, const double* freqs_hz, int32_t nfreq, const kgrt_integrator* integ,
                    const kgrt_outputs* out, void* stream) {
    return kgrt_trace_rays_dev(ctx, rays_dev, nullptr, n, r_obs, phi_obs_deg, model, freqs_hz, nfreq, integ, out,
                               stream);
}

int kgrt_trace_rays_dev(kgrt_ctx* ctx, const double* rays_dev, const int64_t* n_dev, int64_t n, double r_obs,
                        double phi_obs_deg, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                        const kgrt_integrator* integ, const kgrt_outputs* out, void* stream) {
    if (!ctx) return KGRT_E_INVALID_ARG;
    if (n < 0) return fail(ctx, KGRT_E_INVALID_ARG, "n must be >= 0");
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "outputs is NULL");
    if (!(is_finite(r_obs) && r_obs > 20.0)) return fail(ctx, KGRT_E_INVALID_ARG, "r_obs must be finite and > 20");
    if (!is_finite(phi_obs_deg)) return fail(ctx, KGRT_E_INVALID_ARG, "phi_obs_deg must be finite");
    std::string msg;
    int rc = check(msg, nullptr, model, freqs_hz, nfreq, integ);
    if (rc != KGRT_OK) return fail(ctx, rc, msg);
    if (n == 0) return KGRT_OK;
    if (!rays_dev) return fail(ctx, KGRT_E_INVALID_ARG, "rays_dev is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    KParams P{};
    P.images = nullptr;
    P.nimg = 1;
    P.list_mode = 1;
    P.rays4 = rays_dev;
    P.nrays = n;
    P.count_dev = n_dev;
    const double pho = phi_obs_deg * 3.14159265358979323846 / 180.0;
    P.list_r_obs = r_obs;
    P.list_phi_obs = pho;
    P.list_sin_p = std::sin(pho);
    P.list_cos_p = std::cos(pho);
    fill_common(P, model, freqs_hz, nfreq, integ, out, ctx);
    return dispatch(ctx, P, (hipStream_t)stream);
}

}  // extern "C"

struct kgrt_plan {
    kgrt_ctx* ctx = nullptr;
    int device = 0;  // the context's device, kept so that destroying the plan never reads ctx
    KParams P{};
    ImageDesc* images = nullptr;
    double* rec = nullptr;
    int64_t rec_cap = 0;
    unsigned long long* counter = nullptr;
    kgrt_launch launch{};
    hipStream_t capture_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    kgrt_outputs graph_out{};
    kgrt_launch graph_launch{};
};

namespace {

void drop_graph(kgrt_plan* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

bool same_outputs(const kgrt_outputs& a, const kgrt_outputs& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }
bool same_launch(const kgrt_launch& a, const kgrt_launch& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

int plan_enqueue(kgrt_plan* p, const kgrt_outputs* out, hipStream_t st, int64_t limit) {
    KParams P = p->P;
    set_outputs(P, out);
    const LaunchEnv env{p->rec, p->rec_cap, p->counter, p->launch, p->ctx->num_cus, limit};
    return dispatch_env(p->ctx, env, P, st);
}

}  // namespace

extern "C" {

int kgrt_plan_create(kgrt_ctx* ctx, const kgrt_camera* cams, int32_t nimg, const kgrt_model* model,
                     const double* freqs_hz, int32_t nfreq, const kgrt_integrator* integ, kgrt_plan** out) {
    if (!ctx) return KGRT_E_INVALID_ARG;
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nimg < 1 || !cams) return fail(ctx, KGRT_E_INVALID_ARG, "a plan needs nimg >= 1 cameras");
    std::string msg;
    for (int32_t k = 0; k < nimg; ++k) {
        const int rc = check(msg, &cams[k], model, freqs_hz, nfreq, integ);
        if (rc != KGRT_OK) return fail(ctx, rc, "camera " + std::to_string(k) + ": " + msg);
    }
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    std::vector<ImageDesc> tab(nimg);
    int64_t total = 0;
    for (int32_t k = 0; k < nimg; ++k) {
        tab[k] = make_image(&cams[k], model, integ->horizon_delta, total);
        total += (int64_t)cams[k].nx * (int64_t)cams[k].ny;
    }
    auto* p = new (std::nothrow) kgrt_plan();
    if (!p) return fail(ctx, KGRT_E_NOMEM, "plan allocation failed");
    p->ctx = ctx;
    p->device = ctx->device;
    p->launch = ctx->launch;
    KParams& P = p->P;
    fill_common(P, model, freqs_hz, nfreq, integ, nullptr, ctx);
    P.image0 = tab[0];
    P.nimg = nimg;
    P.list_mode = 0;
    P.nrays = total;
    // Start records for the whole plan, so that one persistent launch covers every ray and the
    // grid drains once (88 B per ray: 1.9 GB for 256 images of up to 512^2, 24 GB for 64 of
    // 2048^2); if that much is not available, chunks of the context's size.
    int64_t cap = std::max<int64_t>(1, total);
    bool ok = hipMalloc(&p->images, sizeof(ImageDesc) * nimg) == hipSuccess;
    if (ok && hipMalloc(&p->rec, (size_t)cap * kRecFields * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();  // clear the failed allocation's error
        cap = std::max<int64_t>(1, std::min<int64_t>(total, ctx->chunk_max));
        ok = hipMalloc(&p->rec, (size_t)cap * kRecFields * sizeof(double)) == hipSuccess;
    }
    ok = ok && hipMalloc(&p->counter, sizeof(unsigned long long)) == hipSuccess &&
         hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipMemcpy(p->images, tab.data(), sizeof(ImageDesc) * nimg, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
        kgrt_plan_destroy(p);
        return fail(ctx, KGRT_E_NOMEM, "plan workspace allocation failed");
    }
    p->rec_cap = cap;
    P.images = p->images;
    *out = p;
    return KGRT_OK;
}

int64_t kgrt_plan_num_rays(const kgrt_plan* plan) { return plan ? plan->P.nrays : 0; }

int kgrt_plan_set_launch(kgrt_plan* plan, const kgrt_launch* l) {
    if (!plan) return KGRT_E_INVALID_ARG;
    kgrt_ctx* ctx = plan->ctx;
    if (!l) {
        plan->launch = ctx->launch;
        return KGRT_OK;
    }
    const kgrt_launch keep = ctx->launch;
    const int rc = kgrt_ctx_set_launch(ctx, l);  // same validation
    if (rc == KGRT_OK) plan->launch = ctx->launch;
    ctx->launch = keep;
    return rc;
}

int kgrt_plan_launch(kgrt_plan* plan, const kgrt_outputs* out, uint32_t flags, void* stream) {
    if (!plan) return KGRT_E_INVALID_ARG;
    kgrt_ctx* ctx = plan->ctx;
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "outputs is NULL");
    if (flags & ~KGRT_PLAN_GRAPH) return fail(ctx, KGRT_E_INVALID_ARG, "unknown plan flags");
    if (plan->P.nrays == 0) return KGRT_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    if (!(flags & KGRT_PLAN_GRAPH)) return plan_enqueue(plan, out, st, -1);
    if (!plan->exec || !same_outputs(plan->graph_out, *out) || !same_launch(plan->graph_launch, plan->launch)) {
        drop_graph(plan);
        if (hipStreamBeginCapture(plan->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(ctx, KGRT_E_HIP, "hipStreamBeginCapture failed");
        const int rc = plan_enqueue(plan, out, plan->capture_stream, -1);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(plan->capture_stream, &graph);
        if (rc != KGRT_OK || e != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc != KGRT_OK ? rc : fail(ctx, KGRT_E_HIP, "hipStreamEndCapture failed");
        }
        plan->graph = graph;
        if (hipGraphInstantiate(&plan->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            drop_graph(plan);
            return fail(ctx, KGRT_E_HIP, "hipGraphInstantiate failed");
        }
        plan->graph_out = *out;
        plan->graph_launch = plan->launch;
    }
    if (hipGraphLaunch(plan->exec, st) != hipSuccess) return fail(ctx, KGRT_E_HIP, "hipGraphLaunch failed");
    return KGRT_OK;
}

int kgrt_plan_autotune(kgrt_plan* plan, const kgrt_outputs* out, void* stream, kgrt_launch* best) {
    if (!plan) return KGRT_E_INVALID_ARG;
    kgrt_ctx* ctx = plan->ctx;
    if (!out) return fail(ctx, KGRT_E_INVALID_ARG, "outputs is NULL");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, KGRT_E_HIP, "hipSetDevice failed");
    hipStream_t st = (hipStream_t)stream;
    const int64_t sample = std::min<int64_t>(plan->P.nrays, 524288);
    if (sample == 0) {
        if (best) *best = plan->launch;
        return KGRT_OK;
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(ctx, KGRT_E_HIP, "hipEventCreate failed");
    const kgrt_launch base = plan->launch;
    kgrt_launch winner = base;
    float best_ms = 1e30f;
    int rc = KGRT_OK;
    // candidates: the persistent kernel (many rays per lane, refilled from the queue) at every
    // block size, residency and refill granularity, and one ray per thread (a lane traces a
    // single ray) at every block size
    std::vector<kgrt_launch> cand;
    for (int block : {64, 128, 256}) {
        // blocks per CU: the occupancy rule (0), then two and three waves per SIMD explicitly
        const int waves2 = std::max(1, 2 * 4 * 64 / block), waves3 = std::max(1, 3 * 4 * 64 / block);
        for (int per_cu : {0, waves2, waves3})
            for (int refill : {1, 16, 64}) cand.push_back(kgrt_launch{block, per_cu, refill, KGRT_LAUNCH_PERSISTENT});
        cand.push_back(kgrt_launch{block, 0, 1, KGRT_LAUNCH_ONE_RAY_PER_THREAD});
    }
    for (const kgrt_launch& c : cand) {
        plan->launch = c;
        rc = plan_enqueue(plan, out, st, sample);  // warm-up
        if (rc != KGRT_OK) break;
        (void)hipEventRecord(e0, st);
        rc = plan_enqueue(plan, out, st, sample);
        (void)hipEventRecord(e1, st);
        if (rc != KGRT_OK || hipEventSynchronize(e1) != hipSuccess) {
            rc = (rc != KGRT_OK) ? rc : fail(ctx, KGRT_E_HIP, "autotune timing failed");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            winner = plan->launch;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->launch = (rc == KGRT_OK) ? winner : base;
    if (best) *best = plan->launch;
    return rc;
}

int kgrt_plan_destroy(kgrt_plan* plan) {
    if (!plan) return KGRT_OK;
    DeviceGuard g(plan->device);
    if (plan->capture_stream) (void)hipStreamSynchronize(plan->capture_stream);
    drop_graph(plan);
    if (plan->capture_stream) (void)hipStreamDestroy(plan->capture_stream);
    if (plan->images) (void)hipFree(plan->images);
    if (plan->rec) (void)hipFree(plan->rec);
    if (plan->counter) (void)hipFree(plan->counter);
    delete plan;
    return KGRT_OK;
}

int kgrt_trace_batch(kgrt_ctx* ctx, const kgrt_camera* cams, int32_t nimg, const kgrt_model* model,
                     const double* freqs_hz, int32_t nfreq, const kgrt_integrator* integ, const kgrt_outputs* out,
                     void* stream) {
    kgrt_plan* p = nullptr;
    int rc = kgrt_plan_create(ctx, cams, nimg, model, freqs_hz, nfreq, integ, &p);
    if (rc != KGRT_OK) return rc;
    rc = kgrt_plan_launch(p, out, 0u, stream);
    if (rc == KGRT_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        rc = fail(ctx, KGRT_E_HIP, "hipStreamSynchronize failed");
    kgrt_plan_destroy(p);
    return rc;
}

}  // extern "C"
