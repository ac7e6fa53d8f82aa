// Internal structures shared by the host runtime (jam_host.cpp) and the
// gfx950 kernels (jam_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace jam {

// Device description of one geometry; every pointer is into the context's
// device arena.  The sky maps depend on x'^2 and y'^2 only, so the library
// works on the distinct |x'| values of the padded sub-pixel columns (xs) and
// the distinct |y'| values of its rows (ys); ux/uy map a padded column/row to
// its distinct value.  A "unique pixel" is p = iy * n_ux + ix.
struct GeomDev {
  int K, J1, n_u, T;          // luminous, mass incl. BH, u-nodes, K*J1*n_u terms
  int n_ux, n_uy, n_pix;      // distinct |x'|, |y'|, n_ux*n_uy
  int n_bins;
  int nxp, nyp;               // padded sub-pixel grid
  int pad0, pad1;
  double s_pc;                // pc per arcsec at the geometry's distance
  double bh_sigma;            // arcsec
  const double *lum_sigma, *lum_q, *lum_I0;     // [K]
  const double *mass_sigma, *mass_q, *mass_S0;  // [J1-1]
  const double *u, *w;                          // Gauss-Legendre on [0,1], [n_u]
  const double *xs, *ys;                        // [n_ux], [n_uy]
  const int *ux, *uy;                           // [nxp], [nyp]
  // Bin weights: v_rms^2_b = sum_p W[b,p] N[p] / sum_p W[b,p] I[p] where
  // W[b,p] = sum over field sub-pixels q of bin b and padded sub-pixels
  // mapping to unique pixel p of psf[q - padded]; stored both by bin (for the
  // forward) and by unique pixel (for the adjoint).
  const int *bin_ptr, *bin_pix;  const double *bin_w;   // [n_bins+1], [nnz]
  const int *pix_ptr, *pix_bin;  const double *pix_w;   // [n_pix+1],  [nnz]
  // Spherically aligned model: polar table radii r_i = exp(sph_lnr0 + i
  // sph_dlnr), i < kSphNR; the 8-node Gauss-Legendre rule on [-1, 1] of the
  // composite quadratures.
  double sph_lnr0, sph_dlnr, sph_sig_max;
  double gl8_x[8], gl8_w[8];
};

// Spherically aligned model: polar table of kSphNR radii x kSphNT angles on
// [0, pi/2] of (A_r, A_theta, A_phi); composite rules of kSphSeg segments of
// 8 Gauss-Legendre nodes for the r' and line-of-sight integrals.
constexpr int kSphNR = 128;
constexpr int kSphNT = 24;
constexpr int kSphSeg = 8;
constexpr int kSphNodes = 8 * kSphSeg;   // 64
// (j, u) terms of the spherical potential integrals, padded to whole groups
// of 64; the per-model term region holds that many float4 plus as many floats.
__host__ __device__ inline int sph_terms_padded(int J1, int n_u) {
  return (J1 * n_u + 63) / 64 * 64;
}

// One model of a prepared batch; offsets into packed inputs/outputs and into
// the caller's workspace regions.
struct ModelDev {
  int geom;          // geometry index
  int lum_off;       // into packed beta / lum_I0
  int mass_off;      // into packed mass_S0
  int out_off;       // into packed vrms2 / cot
  int n_slices;      // split of the term range in the numerator kernels
  int n_xt, n_yt;    // 32x32 blocks covering the unique-pixel map (partial maps are
                     // stored padded to 32 n_xt x 32 n_yt per slice)
  int form;          // 1 per-pixel VALU, 2 separable MFMA (wave tiles), 3 separable MFMA
                     // on a map of one 32x32 block with terms computed in place (no term
                     // table), 4 separable MFMA with one workgroup per whole map
  int n_sens_parts;  // partial sensitivity blocks summed by the chain kernel
  int part_f32;      // 1: the split-term partial maps are FP32 (whole-map numerator)
  int sgrid_slices;  // spherical forward: term slices of the potential grid (0: no grid)
  int64_t gauss_off; // doubles, per-Gaussian derived quantities
  int64_t term_off;  // float4 entries, term table (cylindrical: padded_terms(T) entries,
                     // zero past T)
  int64_t pix_off;   // doubles, unique-pixel maps (N, I, lambda)
  int64_t part_off;  // doubles, split-term partial numerators
  int64_t map_off;   // doubles, padded full maps (jam_eval_maps)
  int64_t sens_off;  // doubles, per-term adjoint sensitivities + chain rows
  int64_t bin_off;   // doubles, per-bin sums [Nb | Ib]
  int64_t sph_off;   // doubles, spherical moment table [kSphNR][kSphNT][3]
  int64_t sbp_off;   // doubles, surface-brightness adjoint partials [K][sb items]
  int64_t sgrid_off; // floats, spherical forward potential grid
                     // [sgrid_slices][kSphGridN][kSphGridN][2] (slice 0 holds the sums)
  int64_t sgrid6_off;// floats, the adjoint's grid [sgrid_slices][kSphGridN][kSphGridN][8]
  int64_t sgcot_off; // doubles, the adjoint's grid cotangent (sph_gcot_size)
};
// Entries of a cylindrical model's term table: T rounded up to a multiple of
// 32, so that kernels reading whole chunks of 32 terms stay inside it.
__host__ __device__ inline int64_t padded_terms(int T) { return ((int64_t)T + 31) / 32 * 32; }
// Surface-brightness tiles: kSbRows rows x 64 columns of the unique-pixel map.
constexpr int kSbRows = 8;
__host__ __device__ inline int sb_tiles(int n_ux, int n_uy) {
  return ((n_uy + kSbRows - 1) / kSbRows) * ((n_ux + 63) / 64);
}

// Observed kinematics of one geometry for the chi^2 of eq. (chi2_dyn):
// v_rms per bin and the inverse covariance of their errors (row-major,
// n_bins x n_bins).  Both NULL until set.
struct KinDev {
  const double *vobs, *prec;
};
constexpr int kChi2MaxBins = 4096;
constexpr int kSensTerms = 2048;  // terms per matrix-core sensitivity item

// Constants of the one-dimensional MGE transform (Euler inversion), passed
// by value: nodes beta_k = beta_re + i beta_im[k] and signed weights eta[k]
// (k < n_terms = 2P + 1); per Gaussian n < n_sigma its sigma^2 and the
// factor turning sum_k eta_k Re F(sigma chi_k) into its peak amplitude.
constexpr int kMgeMaxTerms = 41;
constexpr int kMgeMaxSigma = 64;
constexpr int kMgeMaxComp = 64;
struct MgeConst {
  int n_terms, n_sigma;
  double beta_re;
  double beta_im[kMgeMaxTerms];
  double eta[kMgeMaxTerms];
  double sigma2[kMgeMaxSigma];
  double scale[kMgeMaxSigma];
};

// A unit of work of one kernel: model m and up to three kernel-specific
// indices (pixel block, tile, slice, bin, ...).
struct Item {
  int m, a, b, c;
};

// Per-model parameters as the caller passed them (device pointers).
struct ParamsDev {
  const double *inc, *mass_scale, *m_bh, *beta, *lum_I0, *mass_S0;
};

struct GradsDev {
  double *inc, *mass_scale, *m_bh, *beta, *lum_I0, *mass_S0;
};

// Layout of the per-model derived table written by the set-up kernel
// (doubles, at gauss_off): for luminous k: alpha = 1/(2 sigma^2),
// alphaq = alpha / q^2, nu0 (peak density), b = 1/(1-beta); for mass j
// (incl. BH): r = 1/(2 sigma^2), e2 = 1 - q^2, Kp = sqrt(2/pi) G M/(s sigma);
// then sin^2 i, cos^2 i.
__host__ __device__ inline int64_t gauss_size(int K, int J1) { return 4 * K + 3 * J1 + 2; }

// Kernel launchers (jam_kernels.hip).  All asynchronous on `st`.
// Set-up + term table + surface brightness of the cylindrical model in one
// launch: items (m, 0, 0, 0) set-up, (m, term block, 0, 1) terms from the
// parameters, (m, row tile, column tile, 2) surface brightness, (m, term
// block, 0, 3) terms from the Gaussian table of an earlier launch_setup
// (fused: kinds 0, 1, 2; otherwise kinds 2, 3); also zeroes queues[0..1]
// (may be NULL).
void launch_prologue(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                     double *gauss, int *st_ws, int32_t *st_out, int *queues, float4 *terms,
                     double *pix, bool fused, hipStream_t st);
// Also zeroes the two work-queue counters queues[0..1] (may be NULL).
void launch_setup(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, double *gauss,
                  int *st_ws, int32_t *st_out, int *queues, hipStream_t st);
// Items (m, block of 8 unique-pixel rows, block of 64 columns).
void launch_sb(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
               double *pix, hipStream_t st);
// Numerator over a work list of workgroup items.  mfma = false: per-pixel
// VALU form, items (m, 256-pixel block, slice).  mfma = true: matrix-core
// form, items (m, tile origin in 32-blocks x | y << 16, slice, variant 2..5 =
// tile of (1,1), (2,1), (1,2), (2,2) blocks of 32x32; variant 6 = a map of
// one 32x32 block whose terms are computed from the Gaussian table `gauss`
// instead of read from `terms`).  queue != NULL: persistent grid of `grid`
// workgroups pulling items from the counter; else `grid` workgroups striding
// over the list.
void launch_num(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                const float4 *terms, const double *gauss, const int *st_ws, double *part,
                int *queue, int grid, bool mfma, hipStream_t st);
// Whole-map matrix-core numerator (maps of exactly kMapBlocks x kMapBlocks
// blocks of 32x32): items (m, 0, slice, 7), one workgroup per item (queue as
// launch_num); FP32 partial maps.
constexpr int kMapBlocks = 7;
void launch_num_map(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                    const float4 *terms, const int *st_ws, double *part, int *queue, int grid,
                    hipStream_t st);
int occupancy_num(bool mfma);   // resident numerator workgroups per CU
int occupancy_sens();   // resident sensitivity workgroups per CU
// Items (m, 64-pixel block).
void launch_reduce(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                   const double *part, double *pix, hipStream_t st);
// FP32 partial maps (whole-map numerator): items (m, block of 256 positions
// of the padded partial layout).
void launch_reduce_f32(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                       const double *part, double *pix, hipStream_t st);
// Bin items: the first n_wave are (m, first bin, 1) items of up to 4 bins,
// one per wave; the rest (m, bin, 0) items of one bin each.
void launch_bins(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, int n_wave,
                 const double *pix, const int *st_ws, double *vrms2, double *binws,
                 hipStream_t st);
void launch_maps(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                 const double *pix, const int *st_ws, double *N_map, double *I_map,
                 hipStream_t st);
void launch_bins_adjoint(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                         const double *vrms2, const double *cot, const double *binws,
                         const int *st_ws, double *pix, hipStream_t st);
// Sensitivities, variant in Item::c: 0 per-pixel VALU (m, 256-term block),
// 1 MFMA (m, 32-row x tile, tile of kSensTerms terms); queue as launch_num.
void launch_sens(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                 const float4 *terms, const double *pix, const int *st_ws, double *sens,
                 int *queue, int grid, hipStream_t st);
// Wide matrix-core sensitivities: items (m, part p | tiles << 16 for the 1-4
// consecutive 32-row x tiles 4p.., first 32-term group, end group); one
// workgroup of kWideWaves waves per CU, wave w taking the item's groups w,
// w + kWideWaves, ...; queue as launch_sens (the second counter).
constexpr int kWideWaves = 8;
void launch_sens_wide(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                      const float4 *terms, const double *pix, const int *st_ws, double *sens,
                      int *queue, int grid, hipStream_t st);
// sens region per model: n_sens_parts blocks of [S0 | S1 | Sg] (T doubles
// each), then the chain rows [K][J1][3].  Chain items (m, k, jb) for
// jb < ceil(J1 / 4), one mass Gaussian per wave.  The per-pixel kernel
// writes one block; the MFMA kernel one block per 32-row x tile (items
// (m, x tile, 256-term tile)).
void launch_chain(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                  double *sens, const int *st_ws, hipStream_t st);
// Small-map models (unique-pixel map within one 32x32 block): sensitivities
// and chain in one pass, items (m, first tracer | end tracer << 16); writes
// the chain rows (the model has no partial sensitivity blocks,
// n_sens_parts = 0).  An item holds at most kSmallAdjTracers tracers; the
// form needs at most kSmallAdjMass mass Gaussians (BH included).
constexpr int kSmallAdjTerms = 1024;
constexpr int kSmallAdjTracers = 64;
constexpr int kSmallAdjMass = 256;
void launch_adj_small(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                      const double *pix, const int *st_ws, double *sens, hipStream_t st);
void launch_grads(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, double *sens,
                  const double *sbp, const int *st_ws, GradsDev out, hipStream_t st);
// Spherically aligned model.  Terms: items (m, block of 256 terms), the
// model's FP32 (j, u) coefficients into its term region.  Moments: items (m,
// table point i_r * kSphNT + i_theta), one workgroup each, writing A_r,
// A_theta, A_phi into the model's table.  Numerator: items (m, 64-pixel
// block), the line-of-sight integral of the projected table into the
// unique-pixel N map.
void launch_sph_terms(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                      const double *gauss, const int *st_ws, float4 *terms, hipStream_t st);
// Items (m, group of four table points), a wave per point.  With sgrid !=
// NULL the moments take G and G_theta at the characteristic nodes from the
// model's potential grid instead of summing the terms there.
void launch_sph_moments(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                        const double *gauss, const float4 *terms, const int *st_ws,
                        const float *sgrid, double *table, hipStream_t st);
// Potential grid of the spherical model: the tracer-free (j, u) sums G and
// G_theta (forward), or those and their four coefficient-weighted sums for
// the R'^2, z'^2 derivatives (adjoint), on kSphGridN x kSphGridN points
// asinh-spaced in R and in z, as FP32 matrix-core contractions over the
// terms.  Items (m, 64 x 64 tile, term slice) write slice partials; with more
// than one slice the reduce items (m, block of 1024 floats) sum them in order
// into slice 0.
constexpr int kSphGridN = 512;
constexpr int kSphGridTile = 64;
constexpr int kSphGridTiles = (kSphGridN / kSphGridTile) * (kSphGridN / kSphGridTile);
void launch_sph_grid(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                     const double *gauss, const float4 *terms, const int *st_ws, float *sgrid,
                     bool adjoint, hipStream_t st);
void launch_sph_grid_reduce(const ModelDev *m, const Item *it, int n_it, const int *st_ws,
                            float *sgrid, bool adjoint, hipStream_t st);
void launch_sph_num(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                    const double *gauss, const int *st_ws, const double *table, double *pix,
                    hipStream_t st);
// Surface-brightness adjoint, after the bin adjoint has filled lambda_I:
// items (m, row tile, column tile) as launch_sb; sbp[m][k][tile] = sum over
// the tile of lambda_I exp(-x^2 / 2 sigma'^2 - y^2 / 2 sigma'^2 q'^2).
void launch_sb_adjoint(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                       const int *st_ws, const double *pix, double *sbp, hipStream_t st);
// Adjoint of the spherically aligned model, after the bin adjoint has filled
// lambda_N and lambda_I: zero the table cotangents (block per model), the
// line-of-sight adjoint (items (m, 64-pixel block)), the characteristic
// integrals' adjoint (items as launch_sph_moments), the term-major
// sensitivities over point ranges (items (m, 256-term tile, range)) and over
// the table points (items (m, 256-term tile)), the per-term chain (items (m,
// 256-term tile)), and the per-model gradients (block per model; they read
// the surface-brightness partials sbp).
// The moment table together with the cotangent-free node sums of its
// adjoint (SphAdj::jac, gphi), for the adjoint's forward pass; with sgrid6
// != NULL the six node sums come from the model's adjoint grid.
void launch_sph_moments_jac(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                            const double *gauss, const float4 *terms, const int *st_ws,
                            const float *sgrid6, double *table, double *sens, hipStream_t st);
// With sgcot != NULL the term sensitivities go through the potential grid
// (items it_pcot (m, point item), it_pfix (m, 1024 grid points), it_sgs (m,
// 32-term block, row part)) instead of the point-range items it_sens.
void launch_sph_adjoint(const GeomDev *g, const ModelDev *m, int n, const Item *it_los,
                        int n_los, const Item *it_cell, int n_cell, const Item *it_sens,
                        int n_sens, const Item *it_tile, int n_tile, const Item *it_pcot,
                        int n_pcot, const Item *it_pfix, int n_pfix, const Item *it_sgs,
                        int n_sgs, ParamsDev p, const double *gauss, const float4 *terms,
                        const int *st_ws, const double *table, const double *pix,
                        const double *sbp, double *sens, double *sgcot, GradsDev out,
                        hipStream_t st);
// Adjoint of the spherically aligned model.  Per model, in the sensitivity
// region (doubles): the table cotangent [kSphNR*kSphNT][3], per (tracer,
// cell) rows (d/dbeta, d/dalphaq, d/dnu0) [K][cells][3], line-of-sight
// partials (d/di at fixed node scale, d/d node scale) per 64-pixel block,
// per-term sensitivities per point range [n_rng][Tp][6] and of the cell
// points per 256-cell part [kSphCellParts][Tp][3], per-term chain values
// (d/de2, d/dKp) [Tp][2], the table
// cotangent's fixed-point scale [1], the cotangent-free node sums of the
// characteristic integrals' adjoint per (tracer, cell) [K][cells][8] and
// G_phi per cell [cells].  n_rng is ModelDev::n_sens_parts.
constexpr int kSphCells = kSphNR * kSphNT;
// The cell sensitivities come in parts of 256 cells, summed in order.
constexpr int kSphCellParts = kSphCells / 256;
static_assert(kSphCellParts * 256 == kSphCells, "whole 256-cell parts");
struct SphAdj {
  double *dtab, *rows, *losp, *sparts, *cparts, *tchain, *dscale, *jac, *gphi;
};
__host__ __device__ inline int64_t sph_adj_size(int K, int n_pix, int Tp, int n_rng) {
  return 3LL * kSphCells + 3LL * kSphCells * K + 2LL * ((n_pix + 63) / 64) +
         6LL * n_rng * Tp + (3LL * kSphCellParts + 2) * Tp + 1 + 8LL * kSphCells * K + kSphCells;
}
__host__ __device__ inline SphAdj sph_adj_layout(double *base, int K, int n_pix, int Tp,
                                                 int n_rng) {
  SphAdj a;
  a.dtab = base;
  a.rows = a.dtab + 3LL * kSphCells;
  a.losp = a.rows + 3LL * kSphCells * K;
  a.sparts = a.losp + 2LL * ((n_pix + 63) / 64);
  a.cparts = a.sparts + 6LL * n_rng * Tp;
  a.tchain = a.cparts + 3LL * kSphCellParts * Tp;
  a.dscale = a.tchain + 2LL * Tp;
  a.jac = a.dscale + 1;
  a.gphi = a.jac + 8LL * kSphCells * K;
  return a;
}
// Points of one model's characteristic integrals: (cell, tracer, node).
__host__ __device__ inline int64_t sph_points(int K) { return (int64_t)kSphCells * K * kSphNodes; }
// Point ranges of the term-major sensitivity pass: about 2^17 points each,
// at most 64, each a whole number of 256-point chunks.
__host__ __device__ inline int sph_ranges(int K) {
  const int64_t r = (sph_points(K) + 131071) / 131072;
  return (int)(r < 1 ? 1 : (r > 64 ? 64 : r));
}
__host__ __device__ inline int64_t sph_range_len(int K, int n_rng) {
  const int64_t per = (sph_points(K) + n_rng - 1) / n_rng;
  return (per + 255) / 256 * 256;
}
// Term-major sensitivities through the potential grid: the point
// cotangents are spread onto the grid tile by tile.  Point items of
// kSphPtsItem points (items (m, q)) count their points per grid tile (tiles
// of kSphTileB x kSphTileB stencil base cells), a per-model scan turns the
// counts into positions, the point items write their point indices sorted
// by tile, and items (m, q) over kSphPtsItem consecutive entries of that
// list accumulate each tile's stencils in LDS and add them to the grid.
// The fixed-point grid is converted in items (m, block of 1024 grid
// points); the contraction runs in items (m, 32-term block, row part) over
// kSphIParts parts of the grid rows, which are the sensitivities' ranges.
// Workspace per model: sph_gcot_size doubles.
constexpr int kSphPtsItem = 16384;
constexpr int kSphIParts = 4;
constexpr int kSphTileB = 32;
constexpr int kSphTilesAx = (kSphGridN - 2 + kSphTileB - 1) / kSphTileB;
constexpr int kSphTiles = kSphTilesAx * kSphTilesAx;
__host__ __device__ inline int sph_pitems(int K) {
  return (int)((sph_points(K) + kSphPtsItem - 1) / kSphPtsItem);
}
// Doubles: fixed-point grid [N][N][2], FP32 grid [N][N][2], bound partials
// [items][2] and the two scales; then int32: per (item, tile) list
// positions [items][kSphTiles], tile offsets [kSphTiles + 1], a consistency
// flag and the point list [points]; then one byte per point, its tile.
static_assert(kSphTiles <= 256, "a tile index fits one byte");
__host__ __device__ inline int64_t sph_gcot_ints(int K) {
  return (int64_t)sph_pitems(K) * kSphTiles + kSphTiles + 2 + sph_points(K);
}
__host__ __device__ inline int64_t sph_gcot_size(int K) {
  return 3LL * kSphGridN * kSphGridN + 2LL * sph_pitems(K) + 2 + (sph_gcot_ints(K) + 1) / 2 +
         (sph_points(K) + 7) / 8;
}

// Logistic radial anisotropy profile prof[m][0..3] = (beta_0, beta_inf, r_a,
// alpha) sampled at every tracer Gaussian's sigma into the packed beta, and
// its adjoint grad[m][0..3] from the packed cotangent of beta.
void launch_beta_logistic(const GeomDev *g, const ModelDev *m, int n, const double *prof,
                          double *beta, hipStream_t st);
void launch_beta_logistic_vjp(const GeomDev *g, const ModelDev *m, int n, const double *prof,
                              const double *cot, double *grad, hipStream_t st);
// One-dimensional MGE of n_prof profiles, each a sum of n_comp cored power
// laws (a, c, p) = comp[prof][comp][0..2]: amp[prof][n] (device).
void launch_mge1d(int n_prof, int n_comp, const double *comp, const MgeConst &k, double *amp,
                  hipStream_t st);
// grad[prof][comp][0..2] = sum_n cot[prof][n] d amp[prof][n] / d (a, c, p).
void launch_mge1d_vjp(int n_prof, int n_comp, const double *comp, const MgeConst &k,
                      const double *cot, double *grad, hipStream_t st);
// chi^2 per model from V (packed per bin); chi2 and dV may be NULL.  dV gets
// cot[m] * d chi^2_m / dV_b (cot NULL: 1).  st_ws may be NULL.
void launch_chi2(const GeomDev *g, const ModelDev *m, int n, const KinDev *kin, const double *V,
                 const int *st_ws, double *chi2, const double *cot, double *dV, hipStream_t st);

}  // namespace jam
