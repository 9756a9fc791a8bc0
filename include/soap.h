/*
 * soap.h - C ABI of libsoap: disk-integrated spectrum synthesis of an active
 * star on one MI355X (gfx950), following Zhao & Dumusque (2023), "SOAP-GPU:
 * Efficient Spectral Modelling of Stellar Activity Using Graphical
 * Processing Units".
 *
 * Pipeline per call (every step runs in HIP kernels of this library):
 *   soap_grid_init       disk grid, limb darkening, rotation shift per disk
 *                        column, quiet integrated spectrum (section 2.1,
 *                        Algorithm 1, Eqs. 6 and 9-11)
 *   soap_active_spectra  per rotation phase: region positions, InfoMap owner
 *                        per cell, per-column weights, shifted and summed
 *                        differences, final spectra (section 3.3,
 *                        Algorithm 5, Eqs. 1-4; chromatic contrast of
 *                        section 4.3.1)
 *   soap_ccf_rv          CCF against a line mask and Gaussian fit, RV = fitted
 *                        mean (section 4.1)
 *
 * Conventions shared by every entry point
 *   - Every call returns a soap_status; no C++ exception crosses the ABI.
 *   - Arguments are validated before anything is enqueued.  A call that
 *     fails validation leaves the context unchanged and usable; the message
 *     is kept in the context (soap_last_error) until the next failing call.
 *   - Input arrays are read during the call (host arrays are copied before
 *     the call returns); the caller keeps ownership of everything it passes.
 *     Output arrays are allocated by the caller.
 *   - Device pointers must be HIP device memory on the device that was
 *     current at soap_grid_init.  "*_on_device = 0" means a host pointer; the
 *     call then synchronises its stream before returning.  With device
 *     outputs the call only enqueues work on the context's stream.
 *   - Floating-point arrays of spectra and fluxes are float in SOAP_PREC_FP32
 *     contexts and double in SOAP_PREC_FP64 contexts.
 *   - A context is used by one host thread at a time.
 *   - Every device allocation of the library counts against the cap set by
 *     the environment variable SOAP_MAX_DEVICE_BYTES (bytes; unset, empty or
 *     0 = no cap), read at each allocation.  An allocation that would take
 *     the bytes the process holds past it fails as SOAP_ERR_OOM, with the
 *     cap and the bytes held in the message; a value that is not a byte
 *     count refuses every allocation.  soap_device_bytes reports the bytes
 *     held.
 */
#ifndef SOAP_H
#define SOAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SOAP_ABI_VERSION 4

typedef enum {
  SOAP_OK = 0,
  SOAP_ERR_ARG = -1,         /* invalid argument (message says which)          */
  SOAP_ERR_OOM = -2,         /* device or pinned host allocation failed         */
  SOAP_ERR_HIP = -3,         /* a HIP runtime call failed (message has the text) */
  SOAP_ERR_STATE = -4,       /* call not valid in the context's current state   */
  SOAP_ERR_NOCONV = -5,      /* reserved: fit did not converge (per-RV flag)    */
  SOAP_ERR_UNSUPPORTED = -6  /* valid but beyond a stated implementation limit  */
} soap_status;

/* surface types: index into soap_star_desc.spectra */
enum { SOAP_QUIET = 0, SOAP_SPOT = 1, SOAP_FACULA = 2 };

/* effect of active regions, section 2.1:
 *   TOT   Eq. 3: active cells contribute C * S'_active
 *   FLUX  Eq. 1: active cells contribute C * S'_quiet
 *   BCONV Eq. 2: active cells contribute S'_active          */
enum { SOAP_EFFECT_TOT = 0, SOAP_EFFECT_FLUX = 1, SOAP_EFFECT_BCONV = 2 };

/* arithmetic of the synthesis:
 *   FP64  everything in double
 *   FP32  float spectra, interpolation and per-pixel accumulation; float
 *         per-lane column sums with Kahan compensation; double for the sum
 *         over the disk (column sums -> tap weights), the quiet spectrum and
 *         the final per-pixel combine; the CCF sums and the fit in double    */
enum { SOAP_PREC_FP64 = 0, SOAP_PREC_FP32 = 1 };

/* contrast of active regions (section 4.3.1):
 *   SCALAR  soap_region.contrast, one number per region
 *   PLANCK  per pixel B_lambda(T_act) / B_lambda(T_eff), T_act = T_eff - dT_spot
 *           for spots and T_eff + dT_f(mu_b) for faculae, with
 *           dT_f(mu) = c0 + c1 mu + c2 mu^2 evaluated at the mu bin; it
 *           multiplies the spectrum after the Doppler shift
 *   ARRAY   per pixel and mu bin, given by the caller in
 *           soap_star_desc.contrast (section 4.3.3, the SED and limb-brightening
 *           factors of Eqs. 12-14: LB(mu_b) x SED_active / SED_quiet); it
 *           multiplies the shifted active spectrum at the output pixel     */
enum { SOAP_CONTRAST_SCALAR = 0, SOAP_CONTRAST_PLANCK = 1, SOAP_CONTRAST_ARRAY = 2 };

typedef struct soap_ctx soap_ctx;

/* Star description.  Disk: n_grid x n_grid cells with centres
 * x_i = -1 + (2i+1)/n_grid (same for y); a cell is on the disk when
 * x^2 + y^2 < 1; mu = sqrt(1 - x^2 - y^2); weight (2/n_grid)^2 * I(mu) with
 * I(mu) = 1 - ld_u1 (1-mu) - ld_u2 (1-mu)^2; line-of-sight velocity
 * vsini_kms * x (receding for x > 0) under solid-body rotation (diff_rot
 * below for differential rotation).  Wavelength grid: log-uniform,
 * ln(lambda_m / Angstrom) = ln_lambda0 + m * dln_lambda, m = 0..n_pix-1.
 * Local spectra: spectra[t] holds n_mu rows of n_pix samples, row b for the
 * mu bin mu_bins[b]; a cell takes the row of the closest mu bin (ties to the
 * lower index).  spectra[SOAP_QUIET] is required; spectra[SOAP_SPOT] and
 * spectra[SOAP_FACULA] are required only if regions of that type are used
 * (NULL otherwise).                                                          */
typedef struct {
  int32_t n_grid;            /* 2 .. 4096                                   */
  int32_t n_mu;              /* 1 .. 64                                     */
  int64_t n_pix;             /* >= 2 * max shift + 4                        */
  double vsini_kms;          /* |vsini| < 0.1 c                             */
  double incl_deg;           /* inclination of the rotation axis, 0 .. 180  */
  double ld_u1, ld_u2;       /* quadratic limb darkening                    */
  double ln_lambda0;         /* ln(lambda_0 / Angstrom)                     */
  double dln_lambda;         /* > 0                                         */
  const double* mu_bins;     /* host, [n_mu], strictly decreasing in (0, 1] */
  const void* spectra[3];    /* [n_mu][n_pix] row-major, float or double    */
  int32_t spectra_on_device; /* 1: spectra are device pointers              */
  int32_t precision;         /* SOAP_PREC_*                                 */
  int32_t contrast_mode;     /* SOAP_CONTRAST_*                             */
  int32_t reserved0;
  double teff_k;             /* PLANCK mode: quiet effective temperature    */
  double dt_spot_k;          /* PLANCK mode: spot temperature deficit       */
  double dt_fac_coef[3];     /* PLANCK mode: facula dT_f(mu) coefficients   */
  const void* contrast[3];   /* ARRAY mode: [n_mu][n_pix] per active type,
                                same float type and location as spectra;
                                contrast[SOAP_QUIET] must be NULL (the quiet
                                SED is part of the quiet spectra) and
                                contrast[t] is required where spectra[t] is
                                given; finite values.  NULL in other modes.  */
  double diff_rot;           /* differential rotation (section 3.4), |x| < 1:
                                omega(theta) = omega_0 (1 + diff_rot
                                sin^2 theta), theta the latitude; 0 = solid
                                body.  A cell's velocity becomes
                                vsini_kms x (1 + diff_rot sin^2 theta) with
                                sin theta = y sin i + mu cos i, and a region
                                advances 360 deg x phase x (1 + diff_rot
                                sin^2 lat) in longitude.  With it, n_mu times
                                the shift range (2 max|s| + 4) is at most 512 */
} soap_star_desc;

/* One circular active region (section 2.1 region parameters).  Its centre
 * sits at latitude lat_deg and longitude lon_deg + 360 deg * phase (times
 * 1 + diff_rot sin^2 lat_deg under differential rotation); the cap
 * has angular radius asin(radius).  Regions are written into the disk map in
 * list order, so the last listed region covering a cell owns it
 * (section 3.3).  contrast is the scalar I_active / I_quiet used in
 * SOAP_CONTRAST_SCALAR mode (ignored in PLANCK mode).                        */
typedef struct {
  int32_t type;              /* SOAP_SPOT or SOAP_FACULA                    */
  int32_t reserved0;
  double lat_deg;            /* -90 .. 90                                   */
  double lon_deg;
  double radius;             /* sin(alpha), 0 < radius < 1                  */
  double contrast;           /* > 0 (scalar mode)                           */
} soap_region;

/* CCF line mask.  Line l at rest wavelength exp(ln_lambda[l]) with weight
 * weight[l] has, at trial velocity v_k = v0_kms + k dv_kms (k < n_v), a hole
 * spanning the Doppler-shifted (Eq. 6) wavelengths of v_k -/+ half_width_kms.
 * CCF_k = sum_l weight[l] sum_m F_m |pixel_m intersect hole| / dln_lambda,
 * pixel m covering ln(lambda) in [ln_lambda0 + (m - 1/2) dln, + (m + 1/2) dln)
 * and only existing pixels contributing.                                     */
typedef struct {
  int64_t n_lines;           /* 1 .. 1<<20                                  */
  const double* ln_lambda;   /* host, [n_lines]                             */
  const double* weight;      /* host, [n_lines]                             */
  double half_width_kms;     /* > 0, hole at most 8 pixels wide             */
  double v0_kms;
  double dv_kms;             /* > 0                                         */
  int32_t n_v;               /* 4 .. 768; the grid (with holes) spans at most
                                508 pixels                                  */
  int32_t reserved0;
} soap_mask;

/* Result of the Gaussian fit c0 - amp exp(-(v - rv)^2 / (2 sigma^2)) of one
 * CCF (section 4.1: RV = the fitted mean).  status:
 *   0  converged;
 *   1  iteration limit reached;
 *   2  degenerate CCF: a non-finite sample, or no depth (max - min at most
 *      1e-12 of max);
 *   3  failed: no damped step lowers chi^2 from a point that is not a
 *      minimum (no step was ever accepted, the sums are singular or not
 *      finite, or the undamped Newton step there is not of rounding size).
 * Every non-zero status means the RV is not a fitted mean.                   */
typedef struct {
  double rv_kms;
  double fwhm_kms;           /* 2 sqrt(2 ln 2) |sigma|                      */
  double c0;
  double amp;
  double sigma_kms;
  double chi2;               /* sum of squared residuals                    */
  int32_t iters;
  int32_t status;
} soap_rv;

/* Creates a context for one star: copies the description and spectra to the
 * device, computes the per-column Doppler shift, interpolation weights
 * (Eqs. 6, 9-11 on the log grid), the contrast arrays (PLANCK mode) and the
 * quiet integrated spectrum of Algorithm 1, all on `hip_stream` (a
 * hipStream_t; NULL = the null stream).  The device copies of the spectra,
 * contrast arrays and the quiet spectrum are then checked on the device:
 * a non-finite value is SOAP_ERR_ARG for device inputs and SOAP_ERR_HIP
 * (a corrupted upload) for host inputs, which are checked on the host first.
 * SOAP_ERR_UNSUPPORTED when the limb-darkened disk weight, sum of
 * (2/n_grid)^2 |I(mu)| over the cells, reaches 15.9 (the range of the
 * fixed-point tap sums).  The context owns all device workspace until
 * soap_destroy.  On error *out is set to NULL.                              */
soap_status soap_grid_init(const soap_star_desc* desc, void* hip_stream, soap_ctx** out);

/* Copies the quiet integrated spectrum (Algorithm 1) to out[n_pix].          */
soap_status soap_quiet_spectrum(soap_ctx* ctx, void* out, int32_t out_on_device);

/* Integrated spectra of the star with active regions at each phase
 * (Algorithm 5, Eqs. 1-4): flux[n_phases][n_pix], row-major.  regions and
 * phases are host arrays (n_regions 0 .. 64, n_phases 1 .. 1<<20); phase is
 * in rotations (longitude advances 360 deg per unit).  Types present in
 * regions must have spectra.  In SCALAR mode with contrasts other than one
 * (flux and total effects), SOAP_ERR_UNSUPPORTED when the disk weight times
 * the largest contrast reaches 15.9 (the fixed-point range of the sums).    */
soap_status soap_active_spectra(soap_ctx* ctx, const soap_region* regions, int32_t n_regions,
                                const double* phases, int32_t n_phases, int32_t effect,
                                void* flux, int32_t flux_on_device);

/* Many activity configurations of one star in one pass of the kernels
 * (Algorithm 5 per phase, each phase with its own region list): job j has
 * regions[region_offsets[j] .. region_offsets[j+1]) (0 .. 64 of them) and
 * phases[phase_offsets[j] .. phase_offsets[j+1]) (at least one); its spectra
 * are rows phase_offsets[j] .. of flux[total phases][n_pix].  offsets are
 * host arrays of n_jobs + 1 entries starting at 0; at most 2^22 regions and
 * 2^20 phases in all.  Every row equals, bit for bit, what
 * soap_active_spectra gives for that job's regions at that phase.           */
soap_status soap_active_spectra_jobs(soap_ctx* ctx, const soap_region* regions, const int32_t* region_offsets,
                                     const double* phases, const int32_t* phase_offsets, int32_t n_jobs,
                                     int32_t effect, void* flux, int32_t flux_on_device);

/* Size evolution of an active region (section 4.2.1): a linear growing
 * phase, a linear decaying phase, or growth and decay shaped as an
 * asymmetric Gaussian.  Sizes are in millionths of the solar hemisphere
 * (MSH); time t = phase x prot_days.  With d = t - t0_days:
 *   NONE          A = size0_msh
 *   LINEAR_GROWTH A = size0_msh + rate_msh_day d for d >= 0, size0_msh before
 *   LINEAR_DECAY  A = max(0, size0_msh - rate_msh_day d) for d >= 0,
 *                 size0_msh before
 *   ASYM_GAUSS    A = size0_msh exp(-d^2 / (2 w^2)), w = sigma (1 + asym_per_day d),
 *                 sigma = fwhm_days / (2 sqrt(2 ln 2)); A = 0 where w <= 0
 *                 (asym_per_day > 0: fast growth, slow decay)
 * A region of A MSH is a cap covering the fraction f = A 1e-6 of the
 * hemisphere, 1 - cos(alpha) = f, so its radius is sin(alpha) =
 * sqrt(f (2 - f)); a region of size 0 is absent at that time.               */
enum { SOAP_EVOLVE_NONE = 0, SOAP_EVOLVE_LINEAR_GROWTH = 1, SOAP_EVOLVE_LINEAR_DECAY = 2,
       SOAP_EVOLVE_ASYM_GAUSS = 3 };
typedef struct {
  int32_t mode;              /* SOAP_EVOLVE_*                               */
  int32_t reserved0;
  double t0_days;            /* start (linear) or peak (Gaussian) time      */
  double size0_msh;          /* size at t0, > 0, below 1e6 (the hemisphere) */
  double rate_msh_day;       /* linear modes: growth / decay rate, >= 0     */
  double fwhm_days;          /* ASYM_GAUSS: full width at half maximum, > 0 */
  double asym_per_day;       /* ASYM_GAUSS: asymmetry factor                */
} soap_evolution;

/* Size in MSH of a region following `law` at time t_days (NaN for an
 * invalid law).                                                             */
double soap_evolution_size(const soap_evolution* law, double t_days);

/* Integrated spectra of a star whose active regions change size with time
 * (section 4.2.1 with Algorithm 5): region r follows laws[r]; at phase p its
 * radius is the cap radius of its size at t = phases[p] x prot_days (the
 * region's own radius field is ignored), and regions of size 0 are left out.
 * Arguments and flux layout as in soap_active_spectra; prot_days > 0.  Every
 * row equals what soap_active_spectra gives for that phase's region list.   */
soap_status soap_active_spectra_evolving(soap_ctx* ctx, const soap_region* regions, const soap_evolution* laws,
                                         int32_t n_regions, const double* phases, int32_t n_phases,
                                         double prot_days, int32_t effect, void* flux, int32_t flux_on_device);

/* Resolution lowering (the last step of Algorithms 2 and 5: each final
 * spectrum is lowered to the spectrograph's resolution).  The line-spread
 * function is a Gaussian of full width at half maximum lambda / resolution,
 * sigma = 1 / (resolution dln 2 sqrt(2 ln 2)) pixels on the log-uniform grid;
 * the kernel is that Gaussian sampled at whole pixels |k| <= ceil(4 sigma)
 * and normalised to sum 1, and out[m] = sum_k w_k in[clamp(m - k)] (end
 * values held).  in and out are [n_spec][n_pix] in the context's float type,
 * both host or both device memory (on_device), and must not overlap.
 * SOAP_ERR_UNSUPPORTED when the kernel would reach more than 32 pixels each
 * side.  Enqueues only for device memory.                                    */
soap_status soap_instrument_lsf(soap_ctx* ctx, const void* in, void* out, int64_t n_spec, double resolution,
                                int32_t on_device);

/* Makes later soap_active_spectra, soap_active_spectra_jobs and
 * soap_active_spectra_evolving calls on ctx return their spectra lowered to
 * `resolution` as soap_instrument_lsf does (the synthesis goes to a context
 * workspace first); 0 switches the lowering off (the default).  Batches
 * (soap_batch_*) are not affected.                                           */
soap_status soap_set_instrument(soap_ctx* ctx, double resolution);

/* CCF of n_spec spectra flux[n_spec][n_pix] (the context's grid and float
 * type) against `mask`, then a Gaussian fit per CCF (section 4.1).
 * ccf_out[n_spec][n_v] (double, may be NULL) and rv_out[n_spec] (may be
 * NULL) are host or device memory as flagged.  On the first call with a new
 * mask (the context compares against the last one) the line positions, the
 * hole edges per velocity and the batches of nearby lines are built on the
 * host and uploaded; lines whose holes at every velocity fall outside the
 * spectrum add nothing and are left out of the tables.  SOAP_ERR_UNSUPPORTED
 * when a line's holes over the grid reach more than 512 pixels (the velocity
 * span plus the pixels a hole can touch).                                   */
soap_status soap_ccf_rv(soap_ctx* ctx, const void* flux, int32_t flux_on_device, int64_t n_spec,
                        const soap_mask* mask, double* ccf_out, int32_t ccf_on_device,
                        soap_rv* rv_out, int32_t rv_on_device);

/* soap_ccf_rv without any allocation, for callers that cannot allocate
 * (work under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same CCF and fit, bit for bit, as soap_ccf_rv on the same
 * flux; flux, ccf_out (may be NULL) and rv_out (may be NULL) are device
 * memory.  The partial CCFs of the line blocks, and the CCF rows when
 * ccf_out is NULL, go to a file-scope device array of 32 MiB that the
 * library holds on every device it runs on until the process ends:
 * n_spec n_v (e ceil(n_lines / 32) + 8 [ccf_out == NULL]) bytes, e the size
 * of the context's float type, n_lines the mask lines whose reads reach the
 * spectrum (see soap_ccf_rv), the first part rounded up to 256, must fit,
 * else SOAP_ERR_UNSUPPORTED.  The mask
 * must be the one the context already holds (the last one given to
 * soap_ccf_rv), else SOAP_ERR_STATE; nothing is uploaded.  Every call on a
 * device shares that device's array: calls that overlap on one device (other
 * streams, other contexts) race.  Enqueues only; calls no hipMalloc, hipFree
 * or host allocation of pinned memory.                                       */
soap_status soap_ccf_rv_noalloc(soap_ctx* ctx, const void* flux, int64_t n_spec, const soap_mask* mask,
                                double* ccf_out, soap_rv* rv_out);

/* Fits the CCFs of spectra written as a quiet part plus a linear
 * combination of basis spectra, without forming the spectra: the CCF
 * (section 4.1) is linear in the flux, so for F_i = F_0 + sum_k coef[i][k] B_k
 *   CCF(F_i) = base[v] + sum_k coef[i][k] basis[k][v]
 * with base = CCF(F_0) and basis[k] = CCF(B_k) on the context's current mask
 * velocity grid (the last mask given to soap_ccf_rv, which must exist).
 * The sum runs in double in increasing k, then each row is fitted as in
 * soap_ccf_rv.  All arrays are device memory: coef[n][k] float,
 * base[n_v] and basis[k][n_v] double, ccf_out[n][n_v] double (may be NULL),
 * rv_out[n] (may be NULL).  n 1 .. 1<<24, k 1 .. 4096.  Enqueues only.     */
soap_status soap_ccf_linear_rv(soap_ctx* ctx, const float* coef, int64_t n, int32_t k, const double* base,
                               const double* basis, double* ccf_out, soap_rv* rv_out);

/* Surrogate RVs with their gate in one pass, one sample per wave:
 *   rv_out[i], rv_kms[i]: the fit of the CCF of the ensemble-mean prediction
 *     coef[i] (the same CCF and fit as soap_ccf_linear_rv);
 *   err_kms[i] = calib x the sample standard deviation over the members of
 *     the first-order RV change their predictions cause: the fitted
 *     parameters move by H^-1 J^T dy for a CCF change dy (H the Hessian of
 *     half the squared residual sum at the fit, J the model's Jacobian), so
 *     member e moves the RV by h . (members[e][i] - coef[i]) with
 *     h = basis (J H^-1 e_rv);
 *   fallback[i] = 1 when err_kms[i] >= threshold_kms or the fit did not
 *     converge (err_kms is then +inf), else 0.
 * coef[n][k], members[n_ens][n][k] float; base[n_v] double, or with
 * base_index (int32 [n], may be NULL) one base row per sample,
 * base[base_index[i]][n_v] of n_base rows (several stars sharing the basis;
 * a sample whose index is outside [0, n_base) gets status 2 and goes to the
 * fallback); basis[k][n_v]
 * double; all on the context's mask grid (which must exist); outputs device
 * arrays (rv_out and err_kms may be NULL).  n 1 .. 1<<24, n_ens 2 .. 16.
 * Enqueues only, after growing a context workspace (16 n_v + 4 bytes per
 * sample, waiting for the stream) when a call has more samples than any
 * before.                                                                    */
soap_status soap_surrogate_rv(soap_ctx* ctx, const float* coef, const float* members, int64_t n, int32_t n_ens,
                              int32_t k, const double* base, const int32_t* base_index, int32_t n_base,
                              const double* basis, double calib, double threshold_kms, soap_rv* rv_out,
                              double* rv_kms, double* err_kms, int32_t* fallback);

/* Shape of the shift-and-sum kernel and its tuner.  A block of four waves
 * covers a tile of pixels for one chunk of `phases_per_chunk` phases: 8
 * (tiles of 2048 pixels) or 16 (1024 pixels) in FP32, 4 (1024 pixels) or 8
 * (512 pixels) in FP64; the first of each pair is the default.  More phases
 * per chunk read each source window once for more phases (fewer loads per
 * tap), fewer keep more pixels per lane (fewer empty phase slots where
 * regions are visible for only part of a chunk).  Phases per chunk is the
 * layout of the tap tables that the next soap_active_spectra call builds.
 * Every wave keeps `depth` (2 or 3) windows of source samples in flight
 * (the loads of the next depth - 1 windows are issued before the current one
 * is consumed).  `order` picks how each XCD walks its (tile, chunk) items:
 * 0 = chunks with the most windows first, 1 = tile by tile (all chunks of a
 * tile together).  Every shape gives the same result bit for bit (each
 * pixel adds the non-zero taps of its phase in the same window order, and a
 * tap slot that is zero adds exactly zero); only the time differs.          */
typedef struct {
  int32_t depth;
  int32_t order;
  int32_t phases_per_chunk;
  int32_t from_cache;        /* 1: taken from the cache file, not timed     */
  double apply_us;           /* measured time of one launch of the choice   */
  int32_t n_tried;           /* shapes timed                                */
  int32_t reserved;
  char key[128];             /* cache key of the workload shape             */
} soap_tune;

/* Sets the shape used by later calls on ctx; SOAP_ERR_ARG for a depth other
 * than 2 or 3, an order other than 0 or 1, or phases per chunk other than
 * the two of the context's precision (0 = the default one).                 */
soap_status soap_set_apply_shape(soap_ctx* ctx, int32_t depth, int32_t order, int32_t phases_per_chunk);

/* Runs soap_active_spectra on the given workload (arguments as there) once
 * per phases-per-chunk value, times every (depth, order) shape on each
 * call's tap lists (10 launches each, HIP events on the context's stream)
 * and keeps the fastest for later calls.  With cache_path (may be NULL) the
 * choice is looked up first under a key made of the precision, table mode,
 * and the power-of-two buckets of the pixel count, phase count and windows
 * per chunk (default layout), plus the shift range and the mu-bin count; a
 * timed choice is written back.  On error the context keeps its previous
 * phases per chunk.  Waits for the stream.                                  */
soap_status soap_autotune(soap_ctx* ctx, const soap_region* regions, int32_t n_regions, const double* phases,
                          int32_t n_phases, int32_t effect, const char* cache_path, soap_tune* out);

/* Batch of activity configurations over many stars, replayed as one HIP
 * graph.  Configuration i is star ctxs[i] (contexts may repeat) with regions
 * regions[region_offsets[i] .. region_offsets[i+1]) (0 .. 64) at phases
 * phases[phase_offsets[i] .. phase_offsets[i+1]) (at least one); its spectra
 * go to flux[i], a device array [phases of i][n_pix of its star] in the
 * star's float type.  Stars may differ in grid size, pixel count, mu bins,
 * precision and contrast mode.  soap_batch_create validates everything,
 * uploads the parameters, allocates each configuration's tables and
 * captures every configuration's kernels (Algorithm 5 per phase: region
 * parameters, weights, tap lists, shift-and-sum with the context's current
 * apply shape, one launch per group of configurations sharing precision,
 * table mode, phases per chunk and depth) into one graph spread over four
 * parallel branches;
 * soap_batch_run then enqueues the whole batch with a single graph launch on
 * hip_stream.  Every output row equals what soap_active_spectra gives for
 * that configuration, bit for bit.  The contexts and flux arrays must
 * outlive the batch and not be used by other work while a run is in flight;
 * flux arrays must not overlap.  On error *out is NULL and
 * soap_batch_last_error(NULL) has the message (per thread).                 */
typedef struct soap_batch soap_batch;
soap_status soap_batch_create(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                              const int32_t* region_offsets, const double* phases, const int32_t* phase_offsets,
                              int32_t effect, void* const* flux, void* hip_stream, soap_batch** out);
/* The same batch with the CCF and Gaussian fit of every configuration's
 * spectra added to the graph (section 4.1): mask as for soap_ccf_rv (it is
 * set on every context, and the batch keeps its own copy of each context's
 * mask tables); ccf (may be NULL, or hold NULLs) device arrays
 * [phases of i][n_v] double; rv (may be NULL, or hold NULLs) device arrays of
 * soap_rv per phase.  The CCF and fit of configuration i read flux[i] after
 * its shift-and-sum (work-list launches over every configuration sharing a
 * mask layout); every row equals soap_ccf_rv on that flux, bit for bit.
 * Mask errors are those of soap_ccf_rv.                                      */
soap_status soap_batch_create_rv(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                                 const int32_t* region_offsets, const double* phases, const int32_t* phase_offsets,
                                 int32_t effect, void* const* flux, const soap_mask* mask, double* const* ccf,
                                 soap_rv* const* rv, void* hip_stream, soap_batch** out);
/* The configurations of soap_batch_create (same arguments and checks) run
 * once, without a graph: the same work-list launches enqueued on
 * hip_stream, then the call waits for the stream.  For many small
 * configurations over many stars (one call instead of one per star).  The
 * device arena is kept by the library between calls (reused, grown when a
 * call needs more) and calls are serialised on it.  It does not wait for
 * the contexts' own streams: the tables it reads are complete when
 * soap_grid_init returns.  Errors as for soap_batch_create; the message is
 * soap_batch_last_error(NULL).                                              */
soap_status soap_active_spectra_multi(soap_ctx* const* ctxs, int32_t n_cfg, const soap_region* regions,
                                      const int32_t* region_offsets, const double* phases,
                                      const int32_t* phase_offsets, int32_t effect, void* const* flux,
                                      void* hip_stream);
soap_status soap_batch_run(soap_batch* batch);
int64_t soap_batch_n_spectra(const soap_batch* batch);
const char* soap_batch_last_error(const soap_batch* batch);
void soap_batch_destroy(soap_batch* batch);

/* Per-stage GPU time and traffic bookkeeping, for benchmarks.  With
 * profiling on, every stage kernel of soap_active_spectra and soap_ccf_rv is
 * bracketed by HIP events on the context's stream; soap_profile_read waits
 * for the stream and returns the summed stage times since the last
 * soap_profile_enable(ctx, 1), plus the number of distinct local spectra and
 * contrast arrays the last soap_active_spectra read (its touched inputs).   */
typedef struct {
  double weights_ms;         /* region weights + InfoMap + column sums      */
  double compact_ms;         /* slab sums and tap lists                     */
  double apply_ms;           /* shift-and-sum of the final spectra          */
  double ccf_ms;             /* CCF partial sums per block of mask lines    */
  double gfit_ms;            /* fixed-order sum of the partials + fits      */
  double lsf_ms;             /* resolution lowering                         */
  int64_t active_calls;
  int64_t ccf_calls;
  int64_t src_arrays;        /* last apply: distinct local spectra read     */
  int64_t con_arrays;        /* last apply: distinct contrast arrays read   */
  int64_t last_phases;       /* last apply: number of phases                */
  /* last apply's arithmetic per output pixel, summed over its phases and
   * windows: non-zero taps (one FMA each per pixel), window offsets with any
   * non-zero tap (one FMA each to form the difference), and the FMAs the
   * kernel issues (4 per (offset, four-phase group) with a non-zero tap,
   * plus 8 difference FMAs per window)                                     */
  int64_t taps_nonzero;
  int64_t taps_offsets;
  int64_t fma_issued;
} soap_profile;

soap_status soap_profile_enable(soap_ctx* ctx, int32_t on);
soap_status soap_profile_read(soap_ctx* ctx, soap_profile* out);

/* Waits for all work the context enqueued.                                   */
soap_status soap_sync(soap_ctx* ctx);

/* Frees the context and its workspace (waits for its work first).  NULL is a
 * no-op.                                                                      */
void soap_destroy(soap_ctx* ctx);

/* Message of the last failing call on ctx ("" if none); with ctx == NULL, the
 * message of the last failing soap_grid_init in this thread.  Valid until the
 * next call on the same context.                                             */
const char* soap_last_error(const soap_ctx* ctx);

/* Static name of a status code.                                               */
const char* soap_status_string(soap_status status);

/* SOAP_ABI_VERSION of the built library.                                      */
int32_t soap_abi_version(void);

/* Bytes of device memory the library holds in this process now (contexts,
 * batches, surrogates and their workspaces; the fixed array of the
 * allocation-free entry point is not an allocation and is not counted).
 * Needs no device.                                                          */
uint64_t soap_device_bytes(void);

/* ---- learned surrogate --------------------------------------------------
 * Simulations at scale feed data-driven activity models (PCA of line-profile
 * time series, neural networks on CCFs: section 1; section 5 invites such
 * methods to train and test on simulated spectral series).  The surrogate
 * stands in for the synthesis of one spectrum: a small ensemble of MLPs maps
 * the parameters x[n_in] of a configuration (active region, phase) to the
 * normalised PCA coefficients of its difference from the quiet spectrum,
 * and the ensemble spread of the resulting RVs decides which samples go back
 * to the full synthesis.
 *
 * Network of each member: SiLU(x W1 + b1) -> SiLU(. W2 + b2) -> . W3 + b3,
 * W1 [n_in][hidden], W2 [hidden][hidden], W3 [hidden][n_out].  FP32 master
 * parameters; the products run in BF16 on the matrix cores with FP32
 * accumulation.  Loss: mean over batch and outputs of the squared error.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
 * Parameter vectors in the natural layout: W1, b1, W2, b2, W3, b3, each
 * row-major, soap_surrogate_n_params floats per member.  Members start from
 * Glorot-uniform weights drawn with SplitMix64 from (seed, member) and zero
 * biases.  Every kernel adds in a fixed order: results repeat bit for bit.
 * One surrogate is used by one host thread at a time; all its work runs on
 * `hip_stream` (NULL = the null stream).                                    */
typedef struct soap_surrogate soap_surrogate;

/* n_in 1 .. 32; hidden and n_out multiples of 32 in [32, 4096];
 * n_ensemble 1 .. 16.  On error *out is NULL.                                */
soap_status soap_surrogate_create(int32_t n_in, int32_t hidden, int32_t n_out, int32_t n_ensemble,
                                  uint64_t seed, void* hip_stream, soap_surrogate** out);

/* Parameters per member in the natural layout (-1 for NULL).                 */
int64_t soap_surrogate_n_params(const soap_surrogate* s);

/* One Adam step of every member on the same batch: x[batch][n_in] and
 * targets y[batch][n_out], device float arrays; batch a multiple of 32 in
 * [32, 1<<20].  loss_out (host, may be NULL) receives the members' mean loss
 * before the step and makes the call wait for the stream.                   */
soap_status soap_surrogate_train_step(soap_surrogate* s, const float* x, const float* y, int32_t batch, float lr,
                                      float* loss_out);

/* Forward pass of every member: coef[batch][n_out] = ensemble mean,
 * members[n_ensemble][batch][n_out] = each member's output (may be NULL).
 * Device float arrays; batch a multiple of 16 in [16, 1<<20].  Enqueues
 * only.                                                                      */
soap_status soap_surrogate_predict(soap_surrogate* s, const float* x, int32_t batch, float* coef, float* members);

/* Copy one member's parameters, or its gradients from the last train step
 * (before that step's update), to / from a host array of n_params floats.
 * These wait for the stream.                                                 */
soap_status soap_surrogate_get_params(const soap_surrogate* s, int32_t member, float* out);
soap_status soap_surrogate_set_params(soap_surrogate* s, int32_t member, const float* in);
soap_status soap_surrogate_get_grads(const soap_surrogate* s, int32_t member, float* out);

/* Checkpoint of parameters, Adam moments and step count; load requires a
 * surrogate of the same shape and restores it bit for bit.                  */
soap_status soap_surrogate_save(const soap_surrogate* s, const char* path);
soap_status soap_surrogate_load(soap_surrogate* s, const char* path);

/* Message of the last failing call on s.                                     */
const char* soap_surrogate_last_error(const soap_surrogate* s);

/* Frees s (waits for its stream).  NULL is a no-op.                          */
void soap_surrogate_destroy(soap_surrogate* s);

/* Projection onto a PCA basis: coef[i][j] = sum_p (d[i][p] - m_i[p]) V[p][j]
 * for i < n, j < k, in FP32, with m_i = mean[0 .. n_pix), or, with
 * mean_index (int32 [n], may be NULL), row mean_index[i] of mean
 * [n_mean][n_pix] (a per-star centre; a row whose index is outside
 * [0, n_mean) gets NaN coefficients).  d rows have stride ld >= n_pix
 * floats; all arrays are device memory.  n 1 .. 2^25, k 1 .. 4096.
 * Enqueues on hip_stream.                                                    */
soap_status soap_pca_project(const float* d, int64_t n, int64_t n_pix, int64_t ld, const float* mean,
                             const int32_t* mean_index, int32_t n_mean, const float* V, int32_t k, float* coef,
                             void* hip_stream);

/* Network inputs of n samples from their raw descriptions, on the device:
 * raw[i] = (spot latitude deg, longitude deg, radius R*, contrast, rotation
 * phase, T_eff K, inclination deg, v sin i km/s) (double [n][8]); x[i] =
 * 12 floats: latitude / 60 deg, sine and cosine of the rotated longitude
 * (longitude + 360 deg x phase), the spot centre on the sky (x; y along the
 * projected axis; z towards the observer), radius, contrast, T_eff,
 * inclination and v sin i each centred and scaled over their sampled ranges
 * ((r - 0.055) / 0.045, (c - 0.6) / 0.3, (T - 5500) / 1000, (i - 60) / 30,
 * (v - 3) / 2), and 1.  n 1 .. 2^26.  Enqueues on hip_stream.              */
soap_status soap_surrogate_features(const double* raw, int64_t n, float* x, void* hip_stream);

/* Ensemble gate.  rv[(1 + n_ens) n] (device) holds the fits of the
 * ensemble-mean prediction (rows 0 .. n-1) and then of member e (rows
 * (1 + e) n ..).  For sample i: rv_kms[i] = the mean prediction's RV,
 * err_kms[i] = calib * the sample standard deviation of the members' RVs,
 * fallback[i] = 1 when err_kms[i] >= threshold_kms or any of its fits did
 * not converge, else 0 (threshold 0 sends every sample to the full
 * synthesis).  n_ens 2 .. 16; device outputs (err_kms may be NULL).
 * Enqueues on hip_stream.                                                    */
soap_status soap_surrogate_gate(const soap_rv* rv, int64_t n, int32_t n_ens, double calib, double threshold_kms,
                                double* rv_kms, double* err_kms, int32_t* fallback, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SOAP_H */
