/*
 * jam.h - C ABI of the MI355X (gfx950) library for the cylindrically aligned
 * Jeans Anisotropic Model (JAM) projected second moment of a
 * Multi-Gaussian-Expansion (MGE) galaxy with a central black hole, followed
 * by PSF convolution and luminosity-weighted binning, and its adjoint.
 *
 * What is computed (paper Sect. 2.4 and App. A):
 *   - the light MGE, eq. (sb_mge_2D), and the mass MGE, eq. (smd_mge), are
 *     deprojected at inclination i (App. A, requires cos^2 i < q'^2_min);
 *   - the line-of-sight luminosity-weighted second moment, eq. (VLos), of a
 *     cylindrically aligned, per-Gaussian anisotropic Jeans solution in the
 *     potential of the mass MGE plus a BH Gaussian (sigma_BH, q' = 1);
 *   - convolution of I v_los^2 and of I with the kinematic PSF and their
 *     ratio summed over every bin (unnumbered equation before eq. (Vrms)),
 *     giving v_rms^2 per bin; v_rms = sqrt of that (eq. (Vrms)) is left to
 *     the caller.
 *
 * Units: lengths on the sky in arcsec, distance in Mpc, masses in Msun,
 * Sigma0 in Msun/pc^2, luminous amplitudes in any unit (they cancel),
 * inclination in radians (pi/2 = edge-on), output in (km/s)^2.
 * Anisotropy beta_k per luminous Gaussian: 1 - v_z^2 / v_R^2 for the
 * cylindrically aligned model, 1 - v_theta^2 / v_r^2 for the spherically
 * aligned one (jam_options.alignment).
 *
 * Memory: every pointer is a HOST pointer unless its comment says DEVICE.
 * Arrays are contiguous, float64 unless stated, row-major.  The library
 * launches its kernels asynchronously on the caller's HIP stream (passed as
 * void*, a hipStream_t); results are ready when that stream is.  Calls on
 * one context must not overlap in time (one stream at a time); separate
 * contexts are independent.
 *
 * Reproducibility: every sum runs in a fixed order (or in integers), so
 * outputs and gradients are bitwise identical across calls with the same
 * inputs, batch composition and numerator schedule (the schedule is fixed
 * by the options, except that the autotuner may time its way to another
 * one in a new context unless it reads the same tune_cache file); there is
 * no non-deterministic fast path to switch off.
 *
 * Errors: every call returns a jam_status; on anything but JAM_OK nothing
 * was launched unless stated, and jam_last_error() returns a message
 * (thread-local, valid until the next call on the same thread).
 */
#ifndef JAM_H
#define JAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct jam_ctx jam_ctx;

typedef enum {
  JAM_OK = 0,
  JAM_E_INVALID_ARG = 1,   /* a size, pointer or geometry value is invalid        */
  JAM_E_DEPROJECTION = 2,  /* per model: cos^2 i >= q'^2_min (App. A)             */
  JAM_E_NONPHYSICAL = 3,   /* per model: beta_k >= 1, negative mass or amplitude  */
  JAM_E_WORKSPACE = 4,     /* workspace missing or smaller than required          */
  JAM_E_DEVICE = 5,        /* a HIP runtime call or kernel launch failed          */
  JAM_E_UNSUPPORTED = 6    /* option or size outside what this library supports   */
} jam_status;

/* One galaxy model's fixed description (what a sampler does not vary).
 * All arrays are HOST memory and are deep-copied by jam_create.
 *
 * Light MGE, eq. (sb_mge_2D): n_lum >= 1 Gaussians of dispersion
 *   lum_sigma[k] > 0 [arcsec] along the projected major axis, apparent axis
 *   ratio 0 < lum_q[k] <= 1 and default peak lum_I0[k] >= 0.
 * Mass MGE, eq. (smd_mge): n_mass >= 0 Gaussians (mass_sigma, mass_q as
 *   above, default peak mass_S0[j] >= 0 in Msun/pc^2); the BH is appended as
 *   one more mass Gaussian of dispersion bh_sigma > 0 [arcsec], q' = 1.
 * Sky: nx x ny pixels of side pixsize [arcsec]; pixel (ix, iy) is centred at
 *   (xc + (ix - (nx-1)/2) pixsize, yc + (iy - (ny-1)/2) pixsize) with the
 *   galaxy at the origin and x along the major axis; each pixel is split
 *   into supersample x supersample sub-pixels.
 * PSF: psf_n x psf_n kernel (psf_n odd), row-major, sampled on the
 *   sub-pixel grid; it is used as given (normalise it to unit sum).
 * Bins: bin_index[iy * nx + ix] in [-1, n_bins), -1 = excluded; every bin
 *   must own at least one pixel.  Sub-pixels inherit their pixel's bin.
 * Quadrature: n_u in [1, 1024] Gauss-Legendre nodes on u in [0, 1].       */
typedef struct {
  int32_t n_lum;
  const double *lum_sigma, *lum_q, *lum_I0;
  int32_t n_mass;
  const double *mass_sigma, *mass_q, *mass_S0;
  double bh_sigma;
  double distance_mpc;
  int32_t nx, ny;
  double pixsize, xc, yc;
  int32_t supersample;
  int32_t psf_n;
  const double *psf;
  int32_t n_bins;
  const int32_t *bin_index;
  int32_t n_u;
} jam_geometry;

/* form: 0 = automatic, 1 = per-pixel VALU quadrature kernels only,
 *       2 = separable matrix-core (MFMA) kernels.
 * autotune (form 0 only): 1 = when a batch composition is first prepared,
 *       time the candidate numerator schedules (kernel variant, 64x64-tile
 *       pairing threshold, terms per work item, per-item or persistent launch)
 *       on it with fixed valid parameters and keep the fastest; results are
 *       cached per composition, and in the text file tune_cache if not NULL
 *       (read at jam_create, rewritten after each tuning).
 * launch: 0 = one workgroup per work item, dispatched by the hardware;
 *       1 = persistent grid whose workgroups pull work items from a device
 *       queue (largest first).
 * graph: 1 = record each prepared composition's evaluation (and adjoint) as
 *       a HIP graph on first use and replay it while the call's pointers are
 *       unchanged (re-recorded when they change).
 * alignment: 0 = cylindrically aligned velocity ellipsoid (beta_k = 1 -
 *       v_z^2 / v_R^2 per luminous Gaussian; closed-form line-of-sight
 *       integral); 1 = spherically aligned (eqs. J1, J2 of Sect. 2.4; beta_k
 *       = 1 - v_theta^2 / v_r^2), solved along the characteristics of the
 *       Jeans equations into a 128 x 24 polar table of the intrinsic moments
 *       per model and integrated along the line of sight (64 nodes);
 *       autotune and launch do not apply.  The forward takes the
 *       tracer-independent potential sums G, G_theta at the characteristic
 *       nodes from a per-model grid (512 x 512 points asinh-spaced in R and
 *       z, a matrix-core contraction over the (j, u) terms, 4-point Lagrange
 *       interpolation; within 3.4e-7 of the direct sums on the IFU-scale
 *       model); with form = 1 it sums the terms at every node instead.  The
 *       adjoint differentiates the same grid model (with form = 1, the
 *       direct sums); when jam_vjp recomputes V it takes it from the
 *       forward path (bitwise equal to jam_eval's V).  The grid's term
 *       sensitivities spread the point cotangents onto the grid as 64-bit
 *       fixed-point integers, so gradients stay bitwise reproducible.
 *       jam_vjp / jam_vjp_chi2 run the
 *       model's own adjoint (recomputing the moment table in one pass with
 *       the cotangent-free sums of its adjoint; the table cotangent is
 *       summed as 64-bit fixed-point integers at a per-model power-of-two
 *       scale, so gradients are bitwise reproducible) and need a larger
 *       workspace (jam_workspace_size).                                     */
typedef struct {
  int32_t form;
  int32_t autotune;
  const char *tune_cache;
  int32_t launch;
  int32_t graph;
  int32_t alignment;
} jam_options;

/* A batch of n >= 1 models.  geom_idx is HOST memory (n entries, each a
 * geometry index given to jam_create).  Everything else is DEVICE memory:
 * inc[n] (radians), mass_scale[n] (multiplies every mass Gaussian but the
 * BH), m_bh[n] (Msun); beta packed model after model, n_lum(geometry) values
 * each; lum_I0 / mass_S0 packed the same way, or NULL to use the geometry
 * defaults.                                                                   */
typedef struct {
  int32_t n;
  const int32_t *geom_idx;
  const double *inc;
  const double *mass_scale;
  const double *m_bh;
  const double *beta;
  const double *lum_I0;
  const double *mass_S0;
} jam_batch;

/* Gradients of sum_b cot_b v_rms^2_b, DEVICE memory packed like jam_batch
 * (inc, mass_scale, m_bh: n each; beta, lum_I0: sum n_lum; mass_S0:
 * sum n_mass).  Any pointer may be NULL to skip that output.                 */
typedef struct {
  double *inc, *mass_scale, *m_bh, *beta, *lum_I0, *mass_S0;
} jam_grads;

/* Create a context owning device copies of n_geom geometries (validated on
 * the host; JAM_E_INVALID_ARG names the first bad field).  opt may be NULL.
 * Allocates device memory; uses the current HIP device.                      */
jam_status jam_create(int32_t n_geom, const jam_geometry *geoms,
                      const jam_options *opt, jam_ctx **out);

/* Release everything the context owns (NULL is ignored).  The caller must
 * ensure no work using the context is still running.                        */
void jam_destroy(jam_ctx *ctx);

/* Sizes of a batch composition: total packed bins (length of the vrms2
 * output and of the cotangent), total luminous and mass Gaussians (lengths
 * of the packed beta / lum_I0 and mass_S0 arrays).  Any output may be NULL.  */
jam_status jam_batch_sizes(const jam_ctx *ctx, int32_t n, const int32_t *geom_idx,
                           int64_t *n_bins_total, int64_t *n_lum_total,
                           int64_t *n_mass_total);

/* Device workspace, in bytes, that jam_eval_batch (with_vjp = 0) or jam_vjp
 * (with_vjp = 1) needs for this composition.                                 */
jam_status jam_workspace_size(jam_ctx *ctx, int32_t n, const int32_t *geom_idx,
                              int32_t with_vjp, size_t *bytes);

/* Build (or find) the device-side work lists of a batch composition ahead of
 * time.  The first evaluation of a new composition does this itself, which
 * allocates and copies; once prepared, evaluations of that composition
 * neither allocate nor copy and may be captured in a HIP graph.             */
jam_status jam_prepare(jam_ctx *ctx, int32_t n, const int32_t *geom_idx);

/* Forward model for a batch: vrms2 (DEVICE, sum n_bins doubles, model after
 * model) receives v_rms^2 per bin; status (DEVICE int32[n], may be NULL)
 * receives JAM_OK, JAM_E_DEPROJECTION or JAM_E_NONPHYSICAL per model, whose
 * bins are then NaN (other models are unaffected).  ws: DEVICE workspace of
 * ws_bytes >= jam_workspace_size(..., 0).                                    */
jam_status jam_eval_batch(jam_ctx *ctx, const jam_batch *batch, double *vrms2,
                          int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Same as jam_eval_batch for exactly one model (batch->n must be 1).       */
jam_status jam_eval(jam_ctx *ctx, const jam_batch *one, double *vrms2,
                    int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Allocation-free forward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and outputs as jam_eval_batch (vrms2, status
 * as there), with the workspace taken from a fixed device array inside the
 * library (64 MiB; each GPU the library runs on holds one copy until the
 * process ends) instead of a caller's buffer.  It calls no allocating
 * routine and records no graph: the composition must have been prepared on
 * this context (jam_prepare or an earlier call that built it), else
 * JAM_E_INVALID_ARG; a composition whose forward workspace
 * (jam_workspace_size(..., 0)) exceeds 64 MiB gets JAM_E_WORKSPACE.  All
 * calls on one GPU share the array, which keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other contexts, other
 * threads) race and must be serialised by the caller.                       */
jam_status jam_eval_batch_noalloc(jam_ctx *ctx, const jam_batch *batch, double *vrms2,
                                  int32_t *status, void *stream);

/* Unconvolved sky maps on the padded sub-pixel grid of every model:
 * N = int rho_* v_los^2 dz' (numerator of eq. (VLos)) and I (eq.
 * (sb_mge_2D)), each DEVICE, nyp x nxp doubles per model, model after model,
 * with nxp = nx*supersample + psf_n - 1 (likewise nyp); N / I is the
 * per-pixel v_los^2 of eq. (VLos).  Workspace as for jam_eval_batch.         */
jam_status jam_eval_maps(jam_ctx *ctx, const jam_batch *batch, double *N_map,
                         double *I_map, int32_t *status, void *ws, size_t ws_bytes,
                         void *stream);

/* Adjoint: gradients of sum_b cot_b v_rms^2_b with respect to inclination,
 * beta_k, mass scale, BH mass, lum_I0 and mass_S0.  vrms2 is the forward
 * output for the same batch (DEVICE), or NULL to have it recomputed; cot is
 * DEVICE, packed like vrms2.  Nothing from the forward is kept: intermediates
 * are recomputed.  Models with a non-OK status get NaN gradients.  The
 * spherically aligned model runs its own adjoint (jam_options.alignment).
 * ws_bytes >= jam_workspace_size(..., 1).                                    */
jam_status jam_vjp(jam_ctx *ctx, const jam_batch *batch, const double *vrms2,
                   const double *cot, jam_grads *grads, void *ws, size_t ws_bytes,
                   void *stream);

/* Observed kinematics of geometry `geom` for the goodness of fit of eq.
 * (chi2_dyn): vrms_obs (HOST, n_bins doubles, km/s) and the covariance of
 * their measurement errors, cov (HOST, n_bins x n_bins doubles, row-major,
 * (km/s)^2, symmetric positive definite).  The library factors cov (FP64
 * Cholesky), keeps vrms_obs and cov^-1 on the device and owns them until
 * jam_destroy or the next call for the same geometry.  A set-up call: it
 * allocates and waits for the device, so it must not overlap evaluations.
 * JAM_E_INVALID_ARG for a bad index, NULL arrays, non-finite values, an
 * asymmetric or non-positive-definite cov; JAM_E_UNSUPPORTED above 4096
 * bins.                                                                      */
jam_status jam_set_kinematics(jam_ctx *ctx, int32_t geom, const double *vrms_obs,
                              const double *cov);

/* chi^2 of eq. (chi2_dyn) per model from v_rms^2 per bin (eq. (Vrms)):
 * chi2_m = r^T cov^-1 r with r_b = vrms_obs_b - sqrt(vrms2_b), in FP64.
 * vrms2: DEVICE, packed as jam_eval_batch writes it; chi2: DEVICE double[n];
 * dchi2 (DEVICE, packed like vrms2, may be NULL) receives d chi2_m / d
 * vrms2_b = -(cov^-1 r)_b / sqrt(vrms2_b).  A model with any vrms2_b <= 0 or
 * NaN gets NaN in chi2 and dchi2.  Every model's geometry needs kinematics
 * (jam_set_kinematics), else JAM_E_INVALID_ARG before any launch.           */
jam_status jam_chi2(jam_ctx *ctx, const jam_batch *batch, const double *vrms2,
                    double *chi2, double *dchi2, void *stream);

/* Forward model and chi^2 in one call: chi2 (DEVICE double[n]); vrms2
 * (DEVICE, packed, may be NULL to keep it in the workspace) and status as in
 * jam_eval_batch.  ws_bytes >= jam_workspace_size(..., 0).                  */
jam_status jam_eval_chi2(jam_ctx *ctx, const jam_batch *batch, double *chi2, double *vrms2,
                         int32_t *status, void *ws, size_t ws_bytes, void *stream);

/* Adjoint of the chi^2: gradients of sum_m cot_m chi2_m (cot: DEVICE
 * double[n]) with respect to the parameters of jam_vjp.  vrms2 is the
 * forward output for the same batch (DEVICE, packed), or NULL to have the
 * forward recomputed; d chi2 / d vrms2 is formed in the workspace and fed to
 * the adjoint of jam_vjp.  ws_bytes >= jam_workspace_size(..., 1).          */
jam_status jam_vjp_chi2(jam_ctx *ctx, const jam_batch *batch, const double *vrms2,
                        const double *cot, jam_grads *grads, void *ws, size_t ws_bytes,
                        void *stream);

/* One-dimensional multi-Gaussian expansion of radial profiles by the
 * integral transform of Sect. 3.2 (eq. integral_transfer) evaluated with the
 * Euler algorithm.  Each of n_prof profiles is a sum of n_comp cored power
 * laws F(R) = sum_c a_c (R^2 + c_c^2)^(-p_c) of the elliptical radius R
 * (this covers the paper's Chameleon and dPIE profiles, p = 1/2 pairs, its
 * softened power law, p = (gamma - 1) / 2, and the p = 3/2 basis of its
 * eNFW); comp is DEVICE double[n_prof][n_comp][3] = (a, c, p) with c >= 0.
 * sigma (HOST, n_sigma strictly increasing positive values, equally spaced
 * in log) are the Gaussians' dispersions; euler_p is the Euler order P
 * (2P + 1 profile evaluations per Gaussian).  amp (DEVICE
 * double[n_prof][n_sigma]) receives the peak amplitudes A_n of
 * F(R) ~ sum_n A_n exp(-R^2 / (2 sigma_n^2)) (trapezoid weights in
 * log sigma).  Used as lum_I0 / mass_S0 of a geometry whose Gaussians have
 * these dispersions and a common axis ratio.  Limits: n_comp <= 64,
 * n_sigma <= 64, 1 <= euler_p <= 20, n_prof <= 2^24; JAM_E_INVALID_ARG
 * otherwise.  Asynchronous on `stream`; no allocation.                     */
jam_status jam_mge1d(int32_t n_prof, int32_t n_comp, const double *comp, int32_t n_sigma,
                     const double *sigma, int32_t euler_p, double *amp, void *stream);

/* Adjoint of jam_mge1d: grad (DEVICE double[n_prof][n_comp][3]) receives
 * sum_n cot[prof][n] d amp[prof][n] / d (a, c, p) for cot (DEVICE
 * double[n_prof][n_sigma]), e.g. the lum_I0 / mass_S0 gradients of jam_vjp.
 * Same arguments and limits as jam_mge1d.                                   */
jam_status jam_mge1d_vjp(int32_t n_prof, int32_t n_comp, const double *comp, int32_t n_sigma,
                         const double *sigma, int32_t euler_p, const double *cot, double *grad,
                         void *stream);

/* Radially varying orbital anisotropy (Sect. 6: tangential near the centre,
 * radial outside).  For each model m of the batch (only batch->n and
 * batch->geom_idx are read) prof (DEVICE double[n][4]) holds a logistic
 * profile in log r, (beta_0, beta_inf, r_a [arcsec], alpha):
 *   beta(r) = beta_0 + (beta_inf - beta_0) / (1 + (r_a / r)^alpha),
 * and beta (DEVICE, packed like jam_batch.beta) receives it sampled at every
 * tracer Gaussian's dispersion, beta_k = beta(sigma'_k) (the Jeans solutions
 * take one constant anisotropy per Gaussian).  A model whose r_a or alpha is
 * not positive and finite gets NaN, which jam_eval_batch reports as
 * JAM_E_NONPHYSICAL.  Prepares the batch composition's plan if needed;
 * asynchronous on `stream`; no other allocation.                            */
jam_status jam_beta_logistic(jam_ctx *ctx, const jam_batch *batch, const double *prof, double *beta,
                             void *stream);

/* Adjoint of jam_beta_logistic: grad (DEVICE double[n][4]) receives
 * sum_k cot_k d beta_k / d (beta_0, beta_inf, r_a, alpha) for cot (DEVICE,
 * packed like beta; e.g. the beta gradient of jam_vjp); NaN for an invalid
 * profile.  Fixed-order sums.                                               */
jam_status jam_beta_logistic_vjp(jam_ctx *ctx, const jam_batch *batch, const double *prof,
                                 const double *cot, double *grad, void *stream);

/* Kernel timing, for measurement.  enable = 1 clears the record and starts
 * bracketing every launch of the quadrature (numerator) kernel and of the
 * adjoint sensitivity kernel with HIP events on the caller's stream;
 * enable = 0 stops, waits for the recorded events and returns the summed
 * durations in ms and the launch counts (any output may be NULL).  At most
 * 4096 launches of each are recorded; later ones are not timed.            */
jam_status jam_timing(jam_ctx *ctx, int32_t enable, double *numerator_ms,
                      int64_t *numerator_launches, double *sens_ms, int64_t *sens_launches);

/* Schedule chosen for a batch composition (prepares it if needed):
 * info[0..8] = numerator rule (0 per-pixel, 1 MFMA), 64x64-tile threshold,
 * slice length per item ((k, j) pairs, or units of 64 terms), launch mode,
 * numerator work items, numerator workgroups launched, adjoint work items,
 * adjoint workgroups launched, numerator kernel (0 per-pixel k_num_pix,
 * 1 matrix-core tiles k_num_mfma, 2 whole-map matrix core k_num_map,
 * 3 spherical moments k_sph_moments).  info holds 9 int32 (host memory). */
jam_status jam_plan_info(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, int32_t *info);

/* Host utility: the n-node Gauss-Legendre rule on [0, 1] that the library
 * uses (nodes ascending), written to host arrays of n doubles.              */
jam_status jam_gauss_legendre(int32_t n, double *nodes, double *weights);

/* Message of the last non-OK status on this thread ("" if none).          */
const char *jam_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* JAM_H */
