/* kgrt.h -- C ABI of the MI355X Kerr geodesic ray tracer with radiative transfer.
 *
 * Implements the method of Pu, Yun, Younsi & Yoon (2016), "Odyssey": rays are
 * traced backwards in time from a flat image plane (section 2.2, Eqs. (18)-(26))
 * through Kerr spacetime (Eq. (1)) by integrating the six first-order
 * equations of section 2.1 (Eqs. (4)-(5), (9), (12), (14), (15)) with an
 * adaptive fifth-order Runge-Kutta scheme, while the optical depth and the
 * specific intensity of section 2.3 (Eqs. (30)-(31)) are accumulated step by
 * step along each ray.
 *
 * Conventions
 *   - Units G = c = M = 1 (section 2.1). Lengths and the affine parameter are in M.
 *   - All array arguments named *_dev are device pointers of the current HIP
 *     device of the context; all struct arguments are host pointers and are
 *     read during the call only.
 *   - Every trace call is asynchronous and ordered on `stream` (a hipStream_t,
 *     NULL = the null stream). Nothing is synchronised implicitly.
 *   - The caller owns every input and output buffer; the library owns only the
 *     scratch of its context (a work-queue counter and batch tables).
 *   - Two calls on one context race if they run concurrently on different
 *     streams (they share the work-queue counter): use one context per stream.
 *   - Return value: KGRT_OK (0) or a negative KGRT_E_* code; kgrt_last_error()
 *     then holds a message. Problems of single rays never fail a call: they are
 *     reported in the per-ray status word.
 */
#ifndef KGRT_H
#define KGRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define KGRT_OK 0
#define KGRT_E_INVALID_ARG -1  /* an argument is out of its documented range */
#define KGRT_E_HIP -2          /* a HIP runtime call failed */
#define KGRT_E_NOMEM -3        /* device or host allocation failed */
#define KGRT_E_NO_DEVICE -4    /* no usable GPU, or the device index is invalid */
#define KGRT_E_UNSUPPORTED -5  /* a valid request this build does not implement */

/* Per-ray status bits (int32 status output). */
#define KGRT_CAPTURED 1            /* reached r <= r_+ (1 + horizon_delta) */
#define KGRT_ESCAPED 2             /* p_r > 0 and r > r_obs */
#define KGRT_CROSSED 4             /* a first equatorial crossing was recorded */
#define KGRT_DISK_HIT 8            /* ...and it lies on the thin disk [r_in, r_out] */
#define KGRT_MAXSTEPS 16           /* stopped at max_steps accepted steps */
#define KGRT_UNDERFLOW 32          /* step size fell below 1e-12 max(1, r) */
#define KGRT_NONFINITE 64          /* non-finite state or unusable start point */
#define KGRT_FALLBACK 128          /* (surrogate) ray was re-integrated */
#define KGRT_REFINE_UNCONVERGED 256 /* crossing Newton refinement hit its iteration cap */
#define KGRT_SPOT_HIT 512          /* (hot spot) the ray entered the spot and ended there */

/* Emission models. */
#define KGRT_MODEL_GEODESIC 0   /* geometry only: capture flag and first crossing */
#define KGRT_MODEL_THIN_DISK 1  /* geometrically thin Keplerian disk, j = r^-3 (section 4.3) */
#define KGRT_MODEL_TORUS 2      /* thermal-synchrotron torus (section 4.5 emissivity) */
#define KGRT_MODEL_DISK_IMAGES 3 /* the thin disk of section 4.3 made optically thick and followed through
                                    every equatorial crossing: the ray ends at the first crossing on the
                                    disk, which gives the direct image and the higher-order (lensed)
                                    images of sections 4.2-4.3; the crossing outputs and intensities
                                    are those of that crossing, n_cross counts the crossings up to it */
#define KGRT_MODEL_HOT_SPOT 4   /* the orbiting hot spot of section 4.4 (Eq. (36)), optically thick: the ray
                                   ends where it first enters the spot, seen at the emission time
                                   t_obs - Delta t (camera.t_obs); r_cross, phi_cross, t_cross, g,
                                   intensity (g^3 j) and i_bol (g^4 j) describe that entry point */
#define KGRT_MODEL_GRID 5       /* thermal-synchrotron plasma read from a simulation snapshot on a
                                   (ln r, theta, phi) grid (the GRMHD data of section 6, sampled along each
                                   ray): the transfer of Eqs. (30)-(31) with the emissivity of
                                   Eqs. (37)-(39) as for the torus; outputs as for the torus */

/* Integrator flags. */
#define KGRT_STOP_AT_CROSSING 1u /* terminate each ray at its first equatorial crossing */

/* ---------------------------------------------------------------- structs */

/* Observer and image plane (section 2.2). Pixel (i, j), 0 <= i < nx, 0 <= j < ny,
 * sits at the cell centre x = x_min + (i + 1/2)(x_max - x_min)/nx,
 * y = y_min + (j + 1/2)(y_max - y_min)/ny; its output index is j*nx + i. */
typedef struct kgrt_camera {
    double a;            /* black-hole spin a/M, |a| < 1 */
    double incl_deg;     /* inclination theta_obs in degrees, 0 < incl < 180 */
    double phi_obs_deg;  /* azimuth phi_obs in degrees (finite) */
    double r_obs;        /* observer distance in M, r_obs > 10 r_+ (the paper uses 1000) */
    int32_t nx, ny;      /* image size, >= 0 (0 => nothing to trace) */
    double x_min, x_max; /* image-plane extent in M, x_min < x_max */
    double y_min, y_max; /* y_min < y_max */
    double t_obs;        /* observer (coordinate) time of the image, finite; only the hot spot depends
                            on it (section 4.4: light received at t_obs left the spot at t_obs - Delta t) */
} kgrt_camera;

/* Emission/absorption model. */
typedef struct kgrt_model {
    int32_t kind;        /* KGRT_MODEL_* */
    int32_t reserved;    /* must be 0 */
    /* thin disk (section 4.3): inner edge r_in (<= 0 selects r_ISCO(a)), outer edge r_out */
    double r_in, r_out;
    /* torus: n_e = n0 (r/r_norm)^-n_index exp(-z^2/(2 (h_over_r r)^2)), z = r cos(theta);
     * T_e = T0 (r/r_norm)^-T_index; B^2/(8 pi) = eps_B n_e m_p c^2 / (6 r);
     * thermal synchrotron j_nu of Eqs. (37)-(39) per steradian, Kirchhoff absorption;
     * black-hole mass mbh_msun sets r_g; emission only for r_capture < r <= r_emit_max. */
    double n0_cgs, r_norm, n_index, h_over_r, T0_K, T_index, eps_B, mbh_msun, r_emit_max;
    /* hot spot (section 4.4): the centre orbits the equator at Boyer-Lindquist radius spot_r (<= 0
     * selects r_ISCO(a)) with the Keplerian Omega = 1/(spot_r^3/2 + a), at azimuth
     * spot_phi0 + Omega t (radians) at coordinate time t; the spot is the region z > 0,
     * d < 4 spot_size in the pseudo-Cartesian coordinates of section 2.2 (d the distance from the
     * centre), its emissivity exp(-d^2 / (2 spot_size^2)) (Eq. (36), arbitrary units); its matter
     * moves rigidly with the centre (u = u^t (1, 0, 0, Omega), the zero-angular-momentum observer
     * where that is not timelike). spot_size > 0. */
    double spot_r, spot_size, spot_phi0;
    /* gridded plasma (KGRT_MODEL_GRID; section 6): grid_dev is a DEVICE array of float32 values
     * grid_dev[((i * grid_nth + j) * grid_nph + k) * 4 + q], owned by the caller and read during the
     * trace, on the nodes
     *   ln r_i = ln grid_r_min + i (ln grid_r_max - ln grid_r_min) / (grid_nr - 1),  0 <= i < grid_nr,
     *   theta_j = j pi / (grid_nth - 1),  0 <= j < grid_nth,
     *   phi_k = 2 pi k / grid_nph,  0 <= k < grid_nph (periodic in phi),
     * with q = 0: ln n_e (n_e in cm^-3), 1: ln T_e (K), 2: ln B (G), 3: the angular velocity Omega
     * (1/M) of the plasma, which moves on circles, u = u^t (1, 0, 0, Omega) (the zero-angular-
     * momentum observer where that is not timelike). Values between nodes: trilinear interpolation
     * in (ln r, theta, phi), theta clamped to [0, pi]. No plasma outside [grid_r_min, grid_r_max]
     * or at or inside the capture radius. The snapshot is frozen while light crosses it. mbh_msun
     * sets r_g as for the torus; the other torus fields are ignored. grid_nr >= 2, grid_nth >= 2,
     * grid_nph >= 1, grid_nr * grid_nth * grid_nph < 2^31, 0 < grid_r_min < grid_r_max, grid_dev
     * 16-byte aligned (one node, four floats, is read as one 16-byte load),
     * grid_reserved = 0; the other models ignore these fields (grid_dev may be NULL). */
    const float* grid_dev;
    int32_t grid_nr, grid_nth, grid_nph, grid_reserved;
    double grid_r_min, grid_r_max;
} kgrt_model;

/* Adaptive Runge-Kutta controls (section 2.1). */
typedef struct kgrt_integrator {
    double rtol;          /* relative tolerance of the error control, 1e-14 <= rtol <= 1e-2 */
    double hmax_frac;     /* step cap |h| <= hmax_frac * r, 0 < hmax_frac <= 1 */
    double horizon_delta; /* capture radius r_+ (1 + horizon_delta), 0 < delta <= 0.5 */
    int32_t max_steps;    /* accepted-step cap per ray, >= 1 */
    uint32_t flags;       /* KGRT_STOP_AT_CROSSING */
} kgrt_integrator;

/* Per-ray outputs: device arrays of n = number of rays entries (frequency-major
 * [nfreq][n] where noted). A NULL pointer means "do not write". */
typedef struct kgrt_outputs {
    int32_t* status;    /* [n] KGRT_* status bits */
    int32_t* steps;     /* [n] accepted RK steps */
    int32_t* attempts;  /* [n] attempted RK steps (accepted + rejected) */
    double* r_cross;    /* [n] Boyer-Lindquist r at the first equatorial crossing, 0 if none */
    double* g;          /* [n] redshift nu_obs/nu_emit of a Keplerian emitter there (Eq. (2)), 0 if none */
    double* phi_cross;  /* [n] Boyer-Lindquist phi there (accumulated, not wrapped), 0 if none */
    double* t_cross;    /* [n] coordinate time there (negative: traced backwards), 0 if none */
    double* intensity;  /* thin disk: [n] g^3 r_c^-3 on the disk, else 0;
                           torus: [nfreq][n] observed I_nu, erg s^-1 cm^-2 Hz^-1 sr^-1 */
    double* i_bol;      /* thin disk: [n] g^4 r_c^-3 on the disk, else 0 */
    double* tau;        /* torus: [nfreq][n] optical depth along the ray */
    int32_t* n_cross;   /* KGRT_MODEL_DISK_IMAGES: [n] equatorial crossings outside the capture radius
                           up to the end of the ray (the image order of a disk hit is n_cross - 1);
                           not written by the other models */
} kgrt_outputs;

/* Launch modes. */
#define KGRT_LAUNCH_PERSISTENT 0          /* persistent grid, idle lanes refilled from a ray queue */
#define KGRT_LAUNCH_ONE_RAY_PER_THREAD 1  /* one ray per thread, no queue: the paper's mapping (section 3,
                                             Fig. 1), kept as the in-house baseline */

/* Launch shape of the integrator kernel. Zeros select defaults. */
typedef struct kgrt_launch {
    int32_t block;          /* threads per block: 64, 128 or 256 (default 256) */
    int32_t blocks_per_cu;  /* resident blocks per compute unit (default: occupancy limit) */
    int32_t refill_min;     /* refill a wave only when at least this many lanes are idle (1..64; default
                               64, and 1 for eight and more frequencies) */
    int32_t mode;           /* KGRT_LAUNCH_* (default persistent) */
} kgrt_launch;

/* Plan launch flags. */
#define KGRT_PLAN_GRAPH 1u  /* replay the plan's kernels as one captured hipGraph */

typedef struct kgrt_ctx kgrt_ctx;
typedef struct kgrt_plan kgrt_plan;

/* -------------------------------------------------------------- context */

/* Creates a context on HIP device `device` and allocates its scratch.
 * Returns KGRT_E_NO_DEVICE when no GPU is present or the index is invalid. */
int kgrt_ctx_create(int device, kgrt_ctx** out);
/* Destroys a context (NULL is a no-op). Waits for nothing: the caller must
 * make sure no call on it is still running. */
int kgrt_ctx_destroy(kgrt_ctx* ctx);
/* Sets the default launch shape used by later calls (NULL restores defaults). */
int kgrt_ctx_set_launch(kgrt_ctx* ctx, const kgrt_launch* launch);
/* Number of compute units of the context's device. */
int kgrt_ctx_num_cus(const kgrt_ctx* ctx);

/* Launch facts of the integrator kernel the library would run for `model`
 * and `nfreq` (torus: 1..16; others: ignored) at `block` threads per block
 * (64, 128 or 256; 0 = 256), as the runtime reports them for the compiled
 * code: VGPRs per lane, scratch (spill) bytes per lane, resident blocks per
 * compute unit and the resulting waves per SIMD. */
typedef struct kgrt_kernel_info {
    int32_t vgprs, scratch_bytes, blocks_per_cu, waves_per_simd;
} kgrt_kernel_info;
int kgrt_kernel_info_get(kgrt_ctx* ctx, int32_t model, int32_t nfreq, int32_t block, kgrt_kernel_info* out);

/* Validates a request without touching a GPU (the trace calls run the same
 * checks first). cam may be NULL (ray-list mode), freqs_hz is a host array. */
int kgrt_check_args(const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                    const kgrt_integrator* integ);

/* ---------------------------------------------------------------- tracing */

/* Traces one image: one ray per pixel from the image plane of `cam` (section 2.2)
 * until capture, escape or the step cap, with the chosen model.
 * freqs_hz: host array of nfreq observing frequencies (torus: 1 <= nfreq <= 16,
 * each finite and > 0; other models: ignored). Outputs have n = nx*ny entries. */
int kgrt_trace(kgrt_ctx* ctx, const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz,
               int32_t nfreq, const kgrt_integrator* integ, const kgrt_outputs* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): kgrt_trace with the
 * same kernels and results, but its scratch (the work-queue counter and the
 * 88-byte start record of each ray) lives in a static device array of the
 * library instead of the context's workspace, so the call allocates nothing.
 * The array holds KGRT_NOALLOC_MAX_RAYS rays (about 23 MB, held on each device
 * the library runs on until the process ends); an image with more rays
 * (nx * ny > KGRT_NOALLOC_MAX_RAYS) is rejected with KGRT_E_INVALID_ARG.
 * Every call on one device shares that device's array: calls that overlap in
 * time on one device (different streams, threads or contexts) race and give
 * undefined results; calls ordered on one stream are safe (the counter is
 * cleared by a kernel at the start of each call). Returns KGRT_E_HIP if the
 * array's device address could not be obtained when the context was created.
 * Arguments, outputs and other errors as kgrt_trace. */
#define KGRT_NOALLOC_MAX_RAYS 262144
int kgrt_trace_noalloc(kgrt_ctx* ctx, const kgrt_camera* cam, const kgrt_model* model, const double* freqs_hz,
                       int32_t nfreq, const kgrt_integrator* integ, const kgrt_outputs* out, void* stream);

/* Traces a list of independent rays, each with its own spin, inclination and
 * image-plane point: rays_dev is a device array [n][4] of (a, incl_deg, x, y);
 * r_obs and phi_obs are shared. n >= 0 (0 is a no-op). Outputs have n entries. */
int kgrt_trace_rays(kgrt_ctx* ctx, const double* rays_dev, int64_t n, double r_obs, double phi_obs_deg,
                    const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                    const kgrt_integrator* integ, const kgrt_outputs* out, void* stream);

/* ------------------------------------------------------------ batches */

/* A plan holds many images of uneven size, spin and inclination (one model,
 * one frequency set, one integrator) traced together in one persistent launch.
 * This generalises the paper's per-image tracing (section 3) to scene
 * batches. The rays of image k occupy output indices
 * [offset_k, offset_k + nx_k ny_k), offsets the prefix sums of the image sizes
 * in the order given; torus outputs are [nfreq][total rays].
 * kgrt_plan_create validates every camera (as kgrt_trace does; empty images are
 * allowed), uploads the image table and allocates the plan's workspace
 * (synchronously): an 88-byte start record per ray of the whole plan, so that
 * one launch covers all its rays; if that allocation fails, records for
 * chunks of 2^22 rays traced one launch after another. The plan keeps a
 * pointer to ctx; destroy plans first. */
int kgrt_plan_create(kgrt_ctx* ctx, const kgrt_camera* cams, int32_t nimg, const kgrt_model* model,
                     const double* freqs_hz, int32_t nfreq, const kgrt_integrator* integ, kgrt_plan** out);
/* Total number of rays (sum of image sizes). */
int64_t kgrt_plan_num_rays(const kgrt_plan* plan);
/* Launches the plan on `stream` (asynchronous). With KGRT_PLAN_GRAPH the
 * kernels are captured once into a hipGraph (on a stream private to the plan)
 * and replayed; a new capture happens when the output pointers or the launch
 * shape change. Two launches of one plan must not overlap in time. */
int kgrt_plan_launch(kgrt_plan* plan, const kgrt_outputs* out, uint32_t flags, void* stream);
/* Times candidate launch shapes on the plan's first <= 524288 rays: the
 * persistent kernel (many rays per lane) at block 64/128/256, residency (the
 * occupancy rule, decided on the whole plan, or two or three waves per SIMD)
 * and refill granularity 1, 16 or 64, and one ray per thread at block 64/128/256.
 * The fastest is kept for later launches and written to *best if best !=
 * NULL. Synchronous: it waits for `stream`. Outputs of the sampled rays are
 * overwritten. */
int kgrt_plan_autotune(kgrt_plan* plan, const kgrt_outputs* out, void* stream, kgrt_launch* best);
/* Sets the plan's launch shape explicitly (NULL = context default). */
int kgrt_plan_set_launch(kgrt_plan* plan, const kgrt_launch* launch);
/* Releases the plan (waits for its private stream; the caller must make sure
 * no launch of it is still running on other streams). NULL is a no-op. */
int kgrt_plan_destroy(kgrt_plan* plan);

/* One-shot batch: plan, launch, wait for `stream`, destroy. */
int kgrt_trace_batch(kgrt_ctx* ctx, const kgrt_camera* cams, int32_t nimg, const kgrt_model* model,
                     const double* freqs_hz, int32_t nfreq, const kgrt_integrator* integ, const kgrt_outputs* out,
                     void* stream);

/* ------------------------------------------------------------- spectra */

/* Flux density of each image at each frequency, the spectra of section 4:
 * F_nu = sum over the image's pixels of I_nu times the solid angle of one
 * pixel. The intensities are laid out as the torus outputs of a plan,
 * intensity[f * total + i] for frequency f < nfreq and ray i < total, and
 * image k owns rays [offsets[k], offsets[k + 1]) (a plan's offsets are the
 * prefix sums of its image sizes). Writes
 *   flux[k * nfreq + f] = domega[k] * sum_{i in image k} intensity[f * total + i]
 * (erg s^-1 cm^-2 Hz^-1 for intensities in erg s^-1 cm^-2 Hz^-1 sr^-1 and
 * domega in sr, see kgrt_pixel_solid_angle).
 * Arguments: device arrays intensity [nfreq][total] (read; may be NULL when
 * total == 0), offsets [nimg + 1] int64 and domega [nimg] (read), flux
 * [nimg][nfreq] (written); the caller owns all of them. Each image's range is
 * clamped to [0, total] on the device, so offsets outside it read nothing
 * (an empty or reversed range gives 0). Every sum is taken in a fixed order
 * (per-thread strided partial sums, then a fixed tree), so repeated calls give
 * identical results. Asynchronous on `stream`. Returns KGRT_E_INVALID_ARG for
 * nimg < 0 or > 65535, nfreq < 1, total < 0 or a NULL array that would be
 * read or written; nimg == 0 does nothing. */
int kgrt_image_spectra(const double* intensity_dev, int64_t total, int32_t nfreq, const int64_t* offsets_dev,
                       const double* domega_dev, int32_t nimg, double* flux_dev, void* stream);
/* Solid angle in sr of one pixel of cam seen from distance_cm (section 2.2:
 * the image plane is flat, in units of M = r_g = G M_bh / c^2 with M_bh =
 * mbh_msun solar masses): dx dy (r_g / distance_cm)^2 with dx, dy the pixel
 * pitch in M. Host function. Returns -1 for a NULL camera, an empty image, a
 * non-positive or non-finite extent, mass or distance. */
double kgrt_pixel_solid_angle(const kgrt_camera* cam, double mbh_msun, double distance_cm);

/* Spectrum of the Novikov-Thorne disk of section 4.3 seen in traced images of
 * the thin disk (KGRT_MODEL_THIN_DISK or KGRT_MODEL_DISK_IMAGES outputs):
 * every pixel with KGRT_DISK_HIT is a blackbody at the effective temperature
 * of its crossing radius, sigma T^4 = 3 G M Mdot f(r) / (8 pi R^3) (Eq. (35),
 * R = r r_g, f of Page & Thorne (1974) for zero torque at the ISCO of the
 * image's spin), observed with its redshift g, so
 *   flux[k * nfreq + f] = domega[k] * sum over image k's disk pixels of
 *                         g^3 B_nu(T(r_c), nu_f / g)   (erg s^-1 cm^-2 Hz^-1).
 * Arguments: device arrays r_cross, g [total] f64 and status [total] i32 (a
 * plan's outputs), offsets [nimg + 1] int64, domega [nimg] and spin [nimg]
 * f64 (read), flux [nimg][nfreq] (written); freqs_hz is a HOST array of nfreq
 * observed frequencies, 1 <= nfreq <= 32; mbh_msun > 0 and mdot_gs >= 0 (g/s).
 * Sums in a fixed order (per-thread partial sums, then a fixed tree).
 * Asynchronous on `stream`. Returns KGRT_E_INVALID_ARG for out-of-range sizes,
 * non-finite or non-positive frequencies, mass or accretion rate, or a NULL
 * array that would be read or written. */
int kgrt_disk_spectrum(const double* r_cross_dev, const double* g_dev, const int32_t* status_dev, int64_t total,
                       const int64_t* offsets_dev, const double* domega_dev, const double* spin_dev, int32_t nimg,
                       double mbh_msun, double mdot_gs, const double* freqs_hz, int32_t nfreq, double* flux_dev,
                       void* stream);

/* Spectrogram of images of the hot spot (section 4.4, Fig. 7): for each image
 * k (a frame at its observer time) and energy-shift bin b,
 *   out[k * nbins + b] = domega[k] * sum of i_bol[i] over the rays i of image k
 *                        with g_edges[b] <= g[i] < g_edges[b + 1],
 * i.e. the flux of a line emitted at one rest-frame energy E0, binned by the
 * observed energy g E0 (i_bol = g^4 j per pixel, the frequency-integrated
 * intensity). Summed over the bins it is the frame's point of the lightcurve
 * (Fig. 8). Arguments: device arrays i_bol [total] and g [total] (a plan's
 * outputs), offsets [nimg + 1] int64 and domega [nimg] (as for
 * kgrt_image_spectra, ranges clamped to [0, total]), out [nimg][nbins]
 * (written); g_edges is a HOST array of nbins + 1 increasing finite edges,
 * 1 <= nbins <= 64. Each sum is taken in a fixed order (per-thread partial
 * histograms, then threads in order), so repeated calls agree bit for bit.
 * Asynchronous on `stream`. Returns KGRT_E_INVALID_ARG for nimg < 0 or
 * > 65535, nbins out of range, edges not increasing, total < 0 or a NULL
 * array that would be read or written. */
int kgrt_spot_spectrogram(const double* i_bol_dev, const double* g_dev, int64_t total, const int64_t* offsets_dev,
                          const double* domega_dev, int32_t nimg, const double* g_edges, int32_t nbins,
                          double* out_dev, void* stream);

/* ----------------------------------------------------------- surrogate */

/* A learned surrogate of the integrator: a perceptron 4 -> 256 -> 256 -> 256 -> 256 -> 5
 * with SiLU on the hidden layers, mapping ray features (a, cos(inclination),
 * x/15, y/15) to (capture logit, log r_c, g, sin phi_c, cos phi_c) of the first
 * equatorial crossing (section 4.3 thin-disk quantities). Weights and
 * activations are BF16 with FP32 accumulation (MFMA) on the 256x256 layers;
 * the input layer and the output head run in FP32. Parameters are one FP32
 * vector, layer by layer W[out][in] then b[out] (199941 values). */
typedef struct kgrt_mlp kgrt_mlp;
typedef struct kgrt_adam {
    float lr, beta1, beta2, eps;  /* Kingma & Ba (2015) */
} kgrt_adam;

/* Number of parameters (199941). */
int64_t kgrt_mlp_num_params(void);
/* Creates a network on the current device of ctx with workspace for batches
 * of up to max_batch samples (16 <= max_batch <= 2^24, a multiple of 16).
 * Parameters are undefined until kgrt_mlp_set_params. The network object owns
 * its parameters, Adam state, gradient and the training workspace (per-sample
 * activations and partial sums): its training and gradient calls share that
 * workspace, so calls on one object must be ordered (one stream, or streams
 * the caller synchronises). */
int kgrt_mlp_create(kgrt_ctx* ctx, int64_t max_batch, kgrt_mlp** out);
int kgrt_mlp_destroy(kgrt_mlp* mlp);
const char* kgrt_mlp_last_error(const kgrt_mlp* mlp);
/* Host FP32 parameter vector in/out (synchronous). set_params also resets Adam. */
int kgrt_mlp_set_params(kgrt_mlp* mlp, const float* params_host, int64_t n);
int kgrt_mlp_get_params(kgrt_mlp* mlp, float* params_host, int64_t n);
/* Adam state (Kingma & Ba 2015) for checkpoints: first and second moments, FP32
 * vectors of num_params entries in the parameter order (host arrays, synchronous),
 * and the number of steps taken (the t of the bias corrections 1 - beta^t).
 * set_adam rejects non-finite moments or negative second moments and step < 0;
 * call it after set_params, which resets the state. */
int kgrt_mlp_get_adam(kgrt_mlp* mlp, float* m_host, float* v_host, int64_t n, int64_t* step);
int kgrt_mlp_set_adam(kgrt_mlp* mlp, const float* m_host, const float* v_host, int64_t n, int64_t step);
/* Inference: x_dev [n][4] FP32 features -> y_dev [n][5] FP32 outputs, any n >= 0. */
int kgrt_mlp_forward(kgrt_mlp* mlp, const float* x_dev, float* y_dev, int64_t n, void* stream);
/* Loss and gradients of one batch. x_dev [*][4] features, t_dev [*][6] targets
 * (capture 0/1, log r_c, g, sin phi_c, cos phi_c, phi valid 0/1); the batch is
 * rows idx_dev[0..n) (int32, device) or rows 0..n if idx_dev is NULL;
 * 32 <= n <= max_batch, n a multiple of 32. Loss per sample:
 * BCE-with-logits(o0, t0) + 10 (o1-t1)^2 + 10 (o2-t2)^2 + t5 ((o3-t3)^2 + (o4-t4)^2),
 * averaged; written to loss_dev (one float). If grads_dev is not NULL the
 * gradient (num_params floats) is copied there. Every sum over the batch is
 * taken in a fixed order, so the same inputs give bit-identical loss and
 * gradient. */
int kgrt_mlp_loss_grads(kgrt_mlp* mlp, const float* x_dev, const float* t_dev, const int32_t* idx_dev, int64_t n,
                        float* loss_dev, float* grads_dev, void* stream);
/* One Adam step on the batch (as kgrt_mlp_loss_grads): each parameter's new
 * value is written to P and to the BF16 fragments that hold it in the same
 * launch that sums its gradient. */
int kgrt_mlp_train_step(kgrt_mlp* mlp, const float* x_dev, const float* t_dev, const int32_t* idx_dev, int64_t n,
                        const kgrt_adam* opt, float* loss_dev, void* stream);
/* Ray features (a, cos(incl), x/15, y/15) from rays_dev [n][4] = (a, incl_deg, x, y). */
int kgrt_surrogate_features(const double* rays_dev, int64_t n, float* features_dev, void* stream);
/* Training targets [n][6] from integrator outputs of the same rays (thin-disk or
 * geodesic model): rays without a recorded crossing get r_c = r_+, g = 0 and no
 * phi target. */
int kgrt_surrogate_targets(const double* rays_dev, const int32_t* status_dev, const double* r_cross_dev,
                           const double* g_dev, const double* phi_cross_dev, int64_t n, float* targets_dev,
                           void* stream);

/* Fallback policy of the surrogate render. The network's crossing radius is
 * first polished on the exact Mino-time relation of the photon's constants of
 * motion (Eqs. (7), (8), (13) of its start state: Newton's method from the
 * prediction, the radial and polar Mino times by Gauss-Legendre quadrature and
 * Carlson's R_F); that also decides whether the ray reaches the equator
 * outside the capture radius at all. A ray is re-integrated in FP64 when its
 * predicted capture probability lies in [p_lo, p_hi], when it is within
 * crit_band (M, radially in the image plane) of the image's Kerr critical
 * curve, when the polish cannot be certified (no convergence, a Mino-time leg
 * decided by less than 1e-9 relative, Q <= 0), when the polished crossing
 * radius is within edge_band (M) of a disk edge (where the intensity jumps),
 * if g_tol > 0 when the network's g output and the Keplerian g at the polished
 * radius differ by more than g_tol, and if grad_max > 0 when the predicted
 * ln r_c changes by more than grad_max per M of image-plane distance toward
 * one of its 4 neighbouring pixels (one of the two predictions within
 * edge_band of the disk; neighbours in the same network segment of up to 2^22
 * pixels). */
typedef struct kgrt_fallback {
    float p_lo, p_hi, crit_band, edge_band;  /* the package's policy: 0.05, 0.95, 0.5, 1e-4 */
    float g_tol, grad_max;                   /* 0: no check */
} kgrt_fallback;

/* The Kerr critical curve (section 4.2's shadow boundary) seen at infinity,
 * as radius from the image centre on nbins = 1024 equal polar-angle bins
 * starting at -pi (host array; the table the fallback band uses). */
int kgrt_critical_curve(double a, double incl_deg, float* radius_host, int32_t nbins);

/* Thin-disk images (section 4.3, j = r^-3, I = g^3 j) from the surrogate, with
 * fallback rays (kgrt_fallback) re-integrated by the FP64 integrator:
 * features -> network -> decode (crossing-radius polish, Keplerian g at it,
 * fallback test) -> device-built ray list -> integrator -> composite ->
 * per-image flux (each summed in a fixed order). The fallback rays of
 * consecutive images with the same r_obs and phi_obs, up to 2^26 pixels, go to
 * the integrator as one list (one launch), on a stream of the network object
 * ordered by events, while `stream` goes on with the next images (into a
 * second list); `stream` waits for every list before the flux sums, so the
 * call is ordered on `stream` like the others. The integration runs on a
 * context of the network object (its own work queue, so ctx may trace on
 * other streams meanwhile), with lanes refilled once 8 of a wave's are idle
 * (kgrt_launch.refill_min), the fastest measured for fallback lists; ctx is
 * the caller's context on the network's device. Outputs (device): intensity [total]
 * (images concatenated, pixel j*nx+i), status [total] or NULL (KGRT_FALLBACK
 * set on re-integrated rays; others carry the predicted capture/escape bit),
 * flux [nimg] or NULL (sum of intensity per image), fallback_counts [nimg] or
 * NULL. Everything, the critical-curve tables included (built on the device,
 * the same as kgrt_critical_curve's), is asynchronous on `stream`; the host
 * waits only when the workspace grows. Workspace grows on demand
 * and is kept by the network object (about 104 bytes per pixel, two lists of
 * at most 2^26 pixels' worth, plus 36 bytes per pixel of at most 2^22). */
int kgrt_surrogate_render(kgrt_ctx* ctx, kgrt_mlp* mlp, const kgrt_camera* cams, int32_t nimg,
                          const kgrt_model* disk, const kgrt_integrator* integ, const kgrt_fallback* fb,
                          double* intensity_dev, int32_t* status_dev, double* flux_dev,
                          unsigned long long* fallback_counts_dev, void* stream);

/* As kgrt_trace_rays, for lists built on the device: only the first *n_dev
 * (device int64, read by the kernels) of at most n_max rays are traced. Outputs
 * are laid out for n_max rays (torus planes [nfreq][n_max]). */
int kgrt_trace_rays_dev(kgrt_ctx* ctx, const double* rays_dev, const int64_t* n_dev, int64_t n_max, double r_obs,
                        double phi_obs_deg, const kgrt_model* model, const double* freqs_hz, int32_t nfreq,
                        const kgrt_integrator* integ, const kgrt_outputs* out, void* stream);

/* Error strings. kgrt_last_error returns the context's last message ("" if none). */
const char* kgrt_strerror(int code);
const char* kgrt_last_error(const kgrt_ctx* ctx);
/* ABI version (major*10000 + minor*100 + patch). */
int kgrt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KGRT_H */
