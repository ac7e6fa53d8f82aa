// gfx950 kernels of the JAM-cyl forward model and its adjoint.
//
// The numerator map of eq. (VLos) is, per sky point (x', y'),
//   N = sum_{k,j,n} exp(-c1 x'^2 - gamma y'^2) (C0 + C1 x'^2),
// one term per luminous Gaussian k, mass Gaussian j (BH last) and
// Gauss-Legendre node u_n (the u-integral of the deprojected-MGE potential);
// the term coefficients follow from the App. A deprojection and the
// cylindrically aligned Jeans solution.  Derivation per term, with
// alpha = 1/(2 sigma_k^2), r = 1/(2 sigma_j^2), h = 1 - e_j^2 u^2:
//   c1 = alpha + r u^2,  A = alpha/q_k^2 + r u^2 / h,
//   a = c1 sin^2 i + A cos^2 i,  gamma = c1 A / a,
//   g = nu0 K r u^2 / (A h^{3/2})   (nu v_z^2 amplitude),
//   w = 2 nu0 K r u^2 / h^{1/2}      (nu R^-1 dPhi/dR amplitude),
//   P = (cos^2 i + b sin^2 i) g,  Q = sin^2 i (w - 2 c1 b g),
//   C0 = w_n sqrt(pi/a) P,  C1 = w_n sqrt(pi/a) Q,
// with nu0 the deprojected peak density (App. A), K = sqrt(2/pi) G M/(s sigma_j)
// and b = 1/(1 - beta_k).
//
// Precision: the set-up and term coefficients are FP64 and stored as FP32
// (with log2(e) folded into the exponent coefficients for v_exp_f32); the
// integrand sums run in FP32 per (k, j) group of u-nodes and are folded into
// FP64 accumulators; the surface brightness, bin sums and the final division
// are FP64.
#include "jam_internal.h"

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <type_traits>

namespace jam {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kLog2e = 1.44269504088896340736;
// G in pc (km/s)^2 / Msun: IAU nominal GM_sun over (1 pc in m) * 1e6, with
// 1 pc = 648000/pi au and the IAU au.
constexpr double kGMsun = 1.3271244e20;
constexpr double kAu = 149597870700.0;

__device__ inline double grav_const() { return kGMsun / (kAu * 648000.0 / kPi * 1.0e6); }

__device__ inline float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// Split-term partial maps are stored per slice on the unique-pixel map padded
// to whole 32x32 blocks and transposed (y fastest): element (x, y) at
// x * 32 n_yt + y, 32 n_xt * 32 n_yt doubles per slice.  A wave's MFMA tile
// then stores 32 consecutive y values per instruction.
__device__ inline int64_t part_slice_size(const ModelDev &md) {
  return (int64_t)(32 * md.n_xt) * (32 * md.n_yt);
}
__device__ inline int64_t part_index(const ModelDev &md, const GeomDev &g, int q) {
  return (int64_t)(q % g.n_ux) * (32 * md.n_yt) + q / g.n_ux;
}

// Deterministic block sum of one double over a 256-thread block.
__device__ double block_sum256(double v, double *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Eight wave sums at once, in a fixed order: three halving exchanges (lanes
// 32 apart swap halves of the eight values, then 16 apart, then 8 apart)
// leave each lane a partial of value lane / 8, and three butterflies over
// the lane's group of eight finish it.  Returns the full sum of value
// lane / 8 in every lane of group lane / 8 (10 exchanges instead of 48).
__device__ inline double wave_sum8(const double (&v)[8], int lane) {
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double w[4], x[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = h5 ? v[i + 4] : v[i], send = h5 ? v[i] : v[i + 4];
    w[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = h4 ? w[i + 2] : w[i], send = h4 ? w[i] : w[i + 2];
    x[i] = keep + __shfl_xor(send, 16, 64);
  }
  const double keep = h3 ? x[1] : x[0], send = h3 ? x[0] : x[1];
  double y = keep + __shfl_xor(send, 8, 64);
  y += __shfl_xor(y, 4, 64);
  y += __shfl_xor(y, 2, 64);
  y += __shfl_xor(y, 1, 64);
  return y;
}

// ---------------------------------------------------------------------------
// Set-up: App. A deprojection and per-Gaussian derived quantities (FP64),
// per-model validity.
// ---------------------------------------------------------------------------
// One model's set-up; every thread of the block calls it (block-wide ORs).
__device__ void setup_item(const GeomDev *__restrict__ geoms, const ModelDev *__restrict__ models,
                           int m, const ParamsDev &p, double *__restrict__ gauss,
                           int *__restrict__ st_ws, int32_t *__restrict__ st_out) {
  const ModelDev md = models[m];
  const GeomDev g = geoms[md.geom];
  double *tab = gauss + md.gauss_off;
  const double inc = p.inc[m];
  const double si = sin(inc), ci = cos(inc);
  const double si2 = si * si, ci2 = ci * ci;
  const double ml = p.mass_scale[m];
  const double mbh = p.m_bh[m];
  const double G = grav_const();
  const double s = g.s_pc;
  int bad_dep = !(si > 0.0) || !isfinite(inc);
  int bad_phys = !(ml >= 0.0) || !(mbh >= 0.0) || !isfinite(ml) || !isfinite(mbh);
  const int K = g.K, J = g.J1 - 1;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double qo = g.lum_q[k], sig = g.lum_sigma[k];
    const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
    const double beta = p.beta[md.lum_off + k];
    if (!(qo * qo > ci2)) bad_dep = 1;
    if (!(beta < 1.0) || !(I0 >= 0.0) || !isfinite(I0)) bad_phys = 1;
    const double q = sqrt(fmax(qo * qo - ci2, 0.0)) / si;
    const double alpha = 0.5 / (sig * sig);
    tab[k] = alpha;
    tab[K + k] = alpha / (q * q);
    tab[2 * K + k] = qo * I0 / (sqrt(2.0 * kPi) * sig * q);
    tab[3 * K + k] = 1.0 / (1.0 - beta);
  }
  double *mt = tab + 4 * K;
  for (int j = threadIdx.x; j < J + 1; j += blockDim.x) {
    double r, e2, Kp;
    if (j < J) {
      const double qo = g.mass_q[j], sig = g.mass_sigma[j];
      const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
      if (!(qo * qo > ci2)) bad_dep = 1;
      if (!(S0 >= 0.0) || !isfinite(S0)) bad_phys = 1;
      const double q = sqrt(fmax(qo * qo - ci2, 0.0)) / si;
      const double M = ml * 2.0 * kPi * S0 * (s * sig) * (s * sig) * qo;
      r = 0.5 / (sig * sig);
      e2 = 1.0 - q * q;
      Kp = sqrt(2.0 / kPi) * G * M / (s * sig);
    } else {
      r = 0.5 / (g.bh_sigma * g.bh_sigma);
      e2 = 0.0;
      Kp = sqrt(2.0 / kPi) * G * mbh / (s * g.bh_sigma);
    }
    mt[j] = r;
    mt[g.J1 + j] = e2;
    mt[2 * g.J1 + j] = Kp;
  }
  if (threadIdx.x == 0) {
    mt[3 * g.J1] = si2;
    mt[3 * g.J1 + 1] = ci2;
  }
  const int any_dep = __syncthreads_or(bad_dep);
  const int any_phys = __syncthreads_or(bad_phys);
  if (threadIdx.x == 0) {
    const int code = any_dep ? 2 : (any_phys ? 3 : 0);
    st_ws[m] = code;
    if (st_out) st_out[m] = code;
  }
}

__global__ void __launch_bounds__(64) k_setup(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models, int n,
                                              ParamsDev p, double *__restrict__ gauss,
                                              int *__restrict__ st_ws, int32_t *__restrict__ st_out,
                                              int *__restrict__ queues) {
  // Work-queue counters of the kernels that follow on the stream.
  if (queues && blockIdx.x == 0 && threadIdx.x < 2) queues[threadIdx.x] = 0;
  for (int m = blockIdx.x; m < n; m += gridDim.x)
    setup_item(geoms, models, m, p, gauss, st_ws, st_out);
}

// Surface-brightness adjoint: the derivative of sum_p lambda_I[p] I[p] with
// respect to I0_k, per tile of kSbRows rows x 64 columns (the forward's
// items): lane = column, waves split the Gaussians; FP64, wave sums; the
// per-tile partials are summed by the gradient kernels in tile order.
__global__ void __launch_bounds__(256) k_sb_adj(const GeomDev *__restrict__ geoms,
                                                const ModelDev *__restrict__ models,
                                                const Item *__restrict__ items, int n_it,
                                                const int *__restrict__ st_ws,
                                                const double *__restrict__ pix,
                                                double *__restrict__ sbp) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;
    const int y0 = it.a * kSbRows;
    const int ix = it.b * 64 + lane;
    const bool vx = ix < g.n_ux;
    const double x = vx ? g.xs[ix] : 0.0;
    const double *lamI = pix + md.pix_off + 3 * (int64_t)g.n_pix;
    double lam[kSbRows], yy[kSbRows];
#pragma unroll
    for (int r = 0; r < kSbRows; ++r) {
      const bool v = vx && y0 + r < g.n_uy;
      const double y = y0 + r < g.n_uy ? g.ys[y0 + r] : 0.0;
      yy[r] = y * y;
      lam[r] = v ? lamI[(int64_t)(y0 + r) * g.n_ux + ix] : 0.0;
    }
    const int tile = it.a * ((g.n_ux + 63) / 64) + it.b;
    const int n_tiles = sb_tiles(g.n_ux, g.n_uy);
    for (int k = wave; k < g.K; k += 4) {
      const double sig = g.lum_sigma[k], qo = g.lum_q[k];
      const double a = 1.0 / (2.0 * sig * sig), ay = a / (qo * qo);
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < kSbRows; ++r) acc += lam[r] * exp(-ay * yy[r]);
      acc = wave_sum(acc * exp(-a * x * x));
      if (lane == 0) sbp[md.sbp_off + (int64_t)k * n_tiles + tile] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Term table: FP64 coefficients of every (k, j, n) term, stored as FP32
// (-c1 log2e, -gamma log2e, C0, C1).  Term t = (k * J1 + j) * n_u + n.
// ---------------------------------------------------------------------------
// FP64 reciprocal and reciprocal square root: the hardware approximations
// refined by two Newton steps (a few FP64 ulp; the coefficients they feed are
// stored as FP32).  Arguments are positive and finite.
__device__ inline double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double rsq64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

constexpr double kSqrtPi = 1.77245385090551602730;

__device__ inline void term_coeffs(double alpha, double alphaq, double nu0, double b, double r,
                                   double e2, double Kp, double si2, double ci2, double u,
                                   double wq, double &c1, double &gam, double &C0, double &C1) {
  const double u2 = u * u;
  const double h = fma(-e2, u2, 1.0);
  const double ru2 = r * u2;
  c1 = alpha + ru2;
  const double rh = rcp64(h);
  const double A = fma(ru2, rh, alphaq);
  const double a = fma(c1, si2, A * ci2);
  gam = c1 * A * rcp64(a);
  const double base = nu0 * Kp * ru2;
  const double rsh = rsq64(h);
  const double gg = base * rcp64(A) * rh * rsh;
  const double ww = 2.0 * base * rsh;
  const double P = (ci2 + b * si2) * gg;
  const double Q = si2 * (ww - 2.0 * c1 * b * gg);
  const double f = wq * kSqrtPi * rsq64(a);
  C0 = f * P;
  C1 = f * Q;
}

// Term t = (k * J1 + j) * n_u + n of a model from its Gaussian table (the
// set-up's output), as the term table stores it.
__device__ inline float4 term_of(const GeomDev &g, const double *__restrict__ tab, int t) {
  const int n = t % g.n_u, kj = t / g.n_u;
  const int j = kj % g.J1, k = kj / g.J1;
  const double *mt = tab + 4 * g.K;
  double c1, gam, C0, C1;
  term_coeffs(tab[k], tab[g.K + k], tab[2 * g.K + k], tab[3 * g.K + k], mt[j], mt[g.J1 + j],
              mt[2 * g.J1 + j], mt[3 * g.J1], mt[3 * g.J1 + 1], g.u[n], g.w[n], c1, gam, C0, C1);
  return make_float4((float)(-c1 * kLog2e), (float)(-gam * kLog2e), (float)C0, (float)C1);
}


// The per-(k, j) quantities of the set-up straight from the parameters (its
// formulas and operation order), for kernels that run beside the set-up:
// v = (alpha, alphaq, nu0, b, r, e2, Kp, si2, ci2).
__device__ inline void pair_from_params(const GeomDev &g, const ModelDev &md, int m,
                                        const ParamsDev &p, int k, int j, double *v) {
  const double inc = p.inc[m];
  const double si = sin(inc), ci = cos(inc);
  const double si2 = si * si, ci2 = ci * ci;
  const double qo = g.lum_q[k], sig = g.lum_sigma[k];
  const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
  const double q = sqrt(fmax(qo * qo - ci2, 0.0)) / si;
  const double alpha = 0.5 / (sig * sig);
  v[0] = alpha;
  v[1] = alpha / (q * q);
  v[2] = qo * I0 / (sqrt(2.0 * kPi) * sig * q);
  v[3] = 1.0 / (1.0 - p.beta[md.lum_off + k]);
  const double G = grav_const(), sp = g.s_pc;
  if (j < g.J1 - 1) {
    const double qoj = g.mass_q[j], sj = g.mass_sigma[j];
    const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
    const double qj = sqrt(fmax(qoj * qoj - ci2, 0.0)) / si;
    const double M = p.mass_scale[m] * 2.0 * kPi * S0 * (sp * sj) * (sp * sj) * qoj;
    v[4] = 0.5 / (sj * sj);
    v[5] = 1.0 - qj * qj;
    v[6] = sqrt(2.0 / kPi) * G * M / (sp * sj);
  } else {
    v[4] = 0.5 / (g.bh_sigma * g.bh_sigma);
    v[5] = 0.0;
    v[6] = sqrt(2.0 / kPi) * G * p.m_bh[m] / (sp * g.bh_sigma);
  }
  v[7] = si2;
  v[8] = ci2;
}

// ---------------------------------------------------------------------------
// Surface brightness, eq. (sb_mge_2D), FP64, on the unique-pixel map, using
// its separability: I(x, y) = sum_k I0_k exp(-x^2/2s_k^2) exp(-y^2/2s_k^2q_k^2).
// Item (m, block of 8 rows, block of 256 columns): the row factors are
// computed once per workgroup, the column factor once per thread and k.
// pix region per model: [N | I | lambda_N | lambda_I], n_pix doubles each.
// ---------------------------------------------------------------------------

// Item (m, block of 8 rows, block of 64 columns); lane = column, wave w takes
// luminous Gaussians k = w, w + 4, ...; the four partial sums are combined in
// a fixed order.
// One surface-brightness tile; every thread of the block calls it.
__device__ void sb_item(const Item &it, const ModelDev &md, const GeomDev &g, const ParamsDev &p,
                        double *__restrict__ pix, double (*red)[kSbRows][64]) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int y0 = it.a * kSbRows;
  const int ix = it.b * 64 + lane;
  const bool vx = ix < g.n_ux;
  const double x = vx ? g.xs[ix] : 0.0;
  double yy[kSbRows];
#pragma unroll
  for (int r = 0; r < kSbRows; ++r) {
    const double y = y0 + r < g.n_uy ? g.ys[y0 + r] : 0.0;
    yy[r] = y * y;
  }
  double acc[kSbRows];
#pragma unroll
  for (int r = 0; r < kSbRows; ++r) acc[r] = 0.0;
  for (int k = wave; k < g.K; k += 4) {
    const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
    const double sig = g.lum_sigma[k], qo = g.lum_q[k];
    const double a = 1.0 / (2.0 * sig * sig);
    const double fx = I0 * exp(-a * x * x);
    const double ay = a / (qo * qo);
#pragma unroll
    for (int r = 0; r < kSbRows; ++r) acc[r] += fx * exp(-ay * yy[r]);
  }
  if (wave > 0)
#pragma unroll
    for (int r = 0; r < kSbRows; ++r) red[wave - 1][r][lane] = acc[r];
  __syncthreads();
  if (wave == 0 && vx) {
#pragma unroll
    for (int r = 0; r < kSbRows; ++r)
      if (y0 + r < g.n_uy)
        pix[md.pix_off + g.n_pix + (int64_t)(y0 + r) * g.n_ux + ix] =
            ((acc[r] + red[0][r][lane]) + red[1][r][lane]) + red[2][r][lane];
  }
  __syncthreads();
}

__global__ void __launch_bounds__(256) k_sb(const GeomDev *__restrict__ geoms,
                                            const ModelDev *__restrict__ models,
                                            const Item *__restrict__ items, int n_it, ParamsDev p,
                                            double *__restrict__ pix) {
  __shared__ double red[3][kSbRows][64];
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    sb_item(it, md, g, p, pix, red);
  }
}

// Prologue of the cylindrical model: items of four kinds (Item::c): 0 set-up
// of model m (status, Gaussian table); 1 a block of 256 FP32 terms computed
// straight from the parameters, so it needs nothing from set-up items running
// in the same launch (a model with a bad status gets meaningless terms, which
// every later kernel skips); 2 a surface-brightness tile; 3 a block of terms
// from the Gaussian table of a set-up that ran in an earlier launch (zero
// terms for a bad status).  One launch of kinds 0, 1, 2 suits a few large
// models; many small ones run the set-up first and then kinds 2 and 3, which
// avoids recomputing each (k, j) pair's set-up in every term block.
template <bool kFused>
__global__ void __launch_bounds__(256) k_prologue(const GeomDev *__restrict__ geoms,
                                                  const ModelDev *__restrict__ models,
                                                  const Item *__restrict__ items, int n_it,
                                                  ParamsDev p, double *__restrict__ gauss,
                                                  int *__restrict__ st_ws,
                                                  int32_t *__restrict__ st_out,
                                                  int *__restrict__ queues,
                                                  float4 *__restrict__ terms,
                                                  double *__restrict__ pix) {
  __shared__ double red[3][kSbRows][64];
  // per-(k, j) quantities of a term block (kind 1 only)
  __shared__ double pv[kFused ? 258 : 1][9];
  if (queues && blockIdx.x == 0 && threadIdx.x < 2) queues[threadIdx.x] = 0;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (kFused && it.c == 0) {       // uniform per block
      setup_item(geoms, models, it.m, p, gauss, st_ws, st_out);
      continue;
    }
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (it.c == 2) {
      sb_item(it, md, g, p, pix, red);
      continue;
    }
    if (!kFused) {                   // kind 3
      const int t = it.a * 256 + threadIdx.x;
      if (t < g.T)
        terms[md.term_off + t] = st_ws[it.m] == 0 ? term_of(g, gauss + md.gauss_off, t)
                                                  : make_float4(0.f, 0.f, 0.f, 0.f);
      else if (t < padded_terms(g.T))
        terms[md.term_off + t] = make_float4(0.f, 0.f, 0.f, 0.f);
      continue;
    }
    // kind 1: the (k, j) pairs of this block's 256 terms, once each, then
    // the terms
    const int t0 = it.a * 256;
    const int kj0 = t0 / g.n_u, kj1 = (min(t0 + 256, g.T) - 1) / g.n_u;
    for (int q = threadIdx.x; q <= kj1 - kj0; q += 256)
      pair_from_params(g, md, it.m, p, (kj0 + q) / g.J1, (kj0 + q) % g.J1, pv[q]);
    __syncthreads();
    const int t = t0 + threadIdx.x;
    if (t < g.T) {
      const int n = t % g.n_u;
      const double *v = pv[t / g.n_u - kj0];
      double c1, gam, C0, C1;
      term_coeffs(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], g.u[n], g.w[n], c1, gam,
                  C0, C1);
      terms[md.term_off + t] =
          make_float4((float)(-c1 * kLog2e), (float)(-gam * kLog2e), (float)C0, (float)C1);
    } else if (t < padded_terms(g.T)) {
      terms[md.term_off + t] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-pixel VALU quadrature.  Item (m, block of 256 unique pixels, slice of
// (k, j) pairs); thread = pixel.  The slice's terms are staged through LDS
// in runs of whole (k, j) pairs (at most kPixStage terms), read back as
// broadcasts (the same address in every lane); per pair the integrand is
// summed over the u-nodes in FP32 and folded into an FP64 accumulator.
// ---------------------------------------------------------------------------
constexpr int kPixStage = 1024;

__device__ __forceinline__ void num_pix_item(const Item it, const GeomDev *__restrict__ geoms,
    const ModelDev *__restrict__ models, const float4 *__restrict__ terms, const int *__restrict__ st_ws, double *__restrict__ part, float4 *stage) {
  const ModelDev md = models[it.m];
  const GeomDev g = geoms[md.geom];
  const int q = it.a * 256 + threadIdx.x;
  const bool valid = q < g.n_pix;
  float x2 = 0.f, y2 = 0.f;
  if (valid) {
    const double x = g.xs[q % g.n_ux], y = g.ys[q / g.n_ux];
    x2 = (float)(x * x);
    y2 = (float)(y * y);
  }
  const int n_pairs = g.K * g.J1;
  const int per = (n_pairs + md.n_slices - 1) / md.n_slices;
  const int p0 = it.b * per;
  const int p1 = min(n_pairs, p0 + per);
  const int nu = __builtin_amdgcn_readfirstlane(g.n_u);
  const int run = max(1, kPixStage / nu);   // pairs per LDS run
  double acc = 0.0;
  if (st_ws[it.m] == 0) {
    const float4 *tb = terms + md.term_off;
    for (int r0 = p0; r0 < p1; r0 += run) {
      const int r1 = min(p1, r0 + run);
      const int nt = (r1 - r0) * nu;
      __syncthreads();                 // the previous run's reads are done
      for (int e = threadIdx.x; e < nt; e += 256) stage[e] = tb[(int64_t)r0 * nu + e];
      __syncthreads();
      for (int pr = 0; pr < r1 - r0; ++pr) {
        const float4 *tp = stage + pr * nu;
        float s = 0.f;
        int n = 0;
        for (; n + 4 <= nu; n += 4) {
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const float4 c = tp[n + u];
            const float e = fast_exp2(fmaf(c.x, x2, c.y * y2));
            s = fmaf(e, fmaf(c.w, x2, c.z), s);
          }
        }
        for (; n < nu; ++n) {
          const float4 c = tp[n];
          const float e = fast_exp2(fmaf(c.x, x2, c.y * y2));
          s = fmaf(e, fmaf(c.w, x2, c.z), s);
        }
        acc += (double)s;
      }
    }
  }
  if (valid) part[md.part_off + it.b * part_slice_size(md) + part_index(md, g, q)] = acc;
}


// ---------------------------------------------------------------------------
// Separable matrix-core form.  On the unique-pixel map
//   N[x, y] = sum_t A[x, t] B[y, t],
//   A[x, t] = 2^(cx_t x^2) (C0_t + C1_t x^2),   B[y, t] = 2^(cy_t y^2),
// an exact factorisation of the same sum, evaluated as a dense FP32
// contraction over terms with v_mfma_f32_32x32x2f32.  Each 32x32 output
// block accumulates a chunk of 64 terms in FP32 and folds it into FP64.
//
// Operand layout of v_mfma_f32_32x32x2f32 (lane l): A[l % 32][l / 32],
// B[l / 32][l % 32]; accumulator r of lane l is D[i][j] with
// i = (r % 4) + 4 (l / 32) + 8 (r / 4), j = l % 32.
// ---------------------------------------------------------------------------
typedef float v16f __attribute__((ext_vector_type(16)));

__device__ inline int mfma_row(int r, int lane) { return (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2); }

constexpr int KC2 = 64;  // terms per chunk of the matrix-core numerator


// Term range of one slice, in whole chunks of `unit` terms.
__device__ inline void slice_range(int T, int n_slices, int slice, int &t0, int &t1,
                                   int unit) {
  const int chunks = (T + unit - 1) / unit;
  const int per = (chunks + n_slices - 1) / n_slices;
  t0 = min(T, slice * per * unit);
  t1 = min(T, t0 + per * unit);
}

// One workgroup, one item: an output tile of BX x BY blocks of 32x32 unique
// pixels (BX along x, BY along y) over one slice of the terms; the four
// waves take contiguous quarters of the slice in chunks of 64 terms.  Lane l
// generates the operands of its row / column l % 32 of every block for the
// term of its half-wave (A for BX rows, B for BY columns), so each generated
// value feeds BY (resp. BX) MFMAs.  A chunk's coefficients go through the
// wave's private 64-entry LDS slot (one vector load per lane, prefetched a
// chunk ahead); each chunk is summed into fresh FP32 blocks that are then
// folded into FP64 accumulators.  The four FP64 tiles are summed through LDS
// in a fixed order and wave 0 writes the slice's partial tile.
// Item (m, tile origin in 32-blocks x | y << 16, slice, variant 2..5 for
// (BX, BY) = (1,1), (2,1), (1,2), (2,2)); slices are whole 64-term chunks.
// With kGen (variant 6, maps of one 32x32 block, whose terms feed a single
// tile) each lane computes its term of the next chunk from the model's
// Gaussian table instead of loading it from the term table.
template <int BX, int BY, bool kGen>
__device__ __forceinline__ void num_tile_item(const Item it, const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models,
                                              const float4 *__restrict__ terms,
                                              const double *__restrict__ gauss,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ part, float4 *cs, int wave,
                                              double *red) {
  const int lane = threadIdx.x & 63;
  const ModelDev md = models[it.m];
  const GeomDev g = geoms[md.geom];
  const int x0 = (it.a & 0xffff) * 32, y0 = (it.a >> 16) * 32;
  const int c32 = lane & 31, kh = lane >> 5;
  // Rows/columns outside the map get an exponent offset of -inf (and x^2 = 0),
  // so their operands are exactly 0 without a per-element select; inside the
  // map the offset is 0 and fma(c, x^2, 0) rounds exactly like c * x^2.
  float x2[BX], xoff[BX], y2[BY], yoff[BY];
#pragma unroll
  for (int bx = 0; bx < BX; ++bx) {
    const int xi = x0 + 32 * bx + c32;
    x2[bx] = 0.f;
    xoff[bx] = -__builtin_inff();
    if (xi < g.n_ux) { const double x = g.xs[xi]; x2[bx] = (float)(x * x); xoff[bx] = 0.f; }
  }
#pragma unroll
  for (int by = 0; by < BY; ++by) {
    const int yi = y0 + 32 * by + c32;
    y2[by] = 0.f;
    yoff[by] = -__builtin_inff();
    if (yi < g.n_uy) { const double y = g.ys[yi]; y2[by] = (float)(y * y); yoff[by] = 0.f; }
  }
  int ts, te;
  slice_range(g.T, md.n_slices, it.b, ts, te, KC2);
  // this wave's quarter of the slice, in whole chunks
  const int n_all = (st_ws[it.m] == 0) ? (te - ts + KC2 - 1) / KC2 : 0;
  const int qn = (n_all + 3) / 4;
  const int cb = min(n_all, wave * qn), ce = min(n_all, cb + qn);
  const int n_ch = ce - cb;
  const int t0 = ts + cb * KC2, t1 = min(te, ts + ce * KC2);
  const float4 *tb = terms + md.term_off;
  const double *gt = gauss + md.gauss_off;
  auto term = [&](int t) { return kGen ? term_of(g, gt, t) : tb[t]; };
  double acc[BX][BY][16];
#pragma unroll
  for (int bx = 0; bx < BX; ++bx)
#pragma unroll
    for (int by = 0; by < BY; ++by)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[bx][by][r] = 0.0;
  float4 cnext = make_float4(0.f, 0.f, 0.f, 0.f);
  if (n_ch > 0) cnext = term(min(t0 + lane, t1 - 1));
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int ch = 0; ch < n_ch; ++ch) {
    const int tc = t0 + ch * KC2;
    cs[lane] = cnext;
    __builtin_amdgcn_wave_barrier();
    if (ch + 1 < n_ch) cnext = term(min(tc + KC2 + lane, t1 - 1));
    v16f d[BX][BY];
#pragma unroll
    for (int bx = 0; bx < BX; ++bx)
#pragma unroll
      for (int by = 0; by < BY; ++by) d[bx][by] = zero;
    if (tc + KC2 <= t1) {          // whole chunk (wave-uniform), fully unrolled
#pragma unroll
      for (int s2 = 0; s2 < KC2 / 2; ++s2) {
        const float4 c = cs[2 * s2 + kh];
        float a[BX], b[BY];
#pragma unroll
        for (int bx = 0; bx < BX; ++bx)
          a[bx] = fast_exp2(fmaf(c.x, x2[bx], xoff[bx])) * fmaf(c.w, x2[bx], c.z);
#pragma unroll
        for (int by = 0; by < BY; ++by) b[by] = fast_exp2(fmaf(c.y, y2[by], yoff[by]));
#pragma unroll
        for (int bx = 0; bx < BX; ++bx)
#pragma unroll
          for (int by = 0; by < BY; ++by)
            d[bx][by] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bx], b[by], d[bx][by], 0, 0, 0);
      }
    } else {                      // last, partial chunk of the slice
      for (int s2 = 0; s2 < KC2 / 2; ++s2) {
        const int k = 2 * s2 + kh;
        const float4 c = cs[k];
        const bool vt = tc + k < t1;
        float a[BX], b[BY];
#pragma unroll
        for (int bx = 0; bx < BX; ++bx) {
          const float v = fast_exp2(fmaf(c.x, x2[bx], xoff[bx])) * fmaf(c.w, x2[bx], c.z);
          a[bx] = vt ? v : 0.f;
        }
#pragma unroll
        for (int by = 0; by < BY; ++by) {
          const float v = fast_exp2(fmaf(c.y, y2[by], yoff[by]));
          b[by] = vt ? v : 0.f;
        }
#pragma unroll
        for (int bx = 0; bx < BX; ++bx)
#pragma unroll
          for (int by = 0; by < BY; ++by)
            d[bx][by] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bx], b[by], d[bx][by], 0, 0, 0);
      }
    }
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int bx = 0; bx < BX; ++bx)
#pragma unroll
      for (int by = 0; by < BY; ++by)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[bx][by][r] += (double)d[bx][by][r];
  }
  // fixed-order sum of the four waves' tiles: wave 0 adds those of waves
  // 3, 2 and 1 in turn through one LDS tile
  for (int src = 3; src >= 1; --src) {
    __syncthreads();
    if (wave == src) {
#pragma unroll
      for (int bx = 0; bx < BX; ++bx)
#pragma unroll
        for (int by = 0; by < BY; ++by)
#pragma unroll
          for (int r = 0; r < 16; ++r) red[((bx * BY + by) * 16 + r) * 64 + lane] = acc[bx][by][r];
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int bx = 0; bx < BX; ++bx)
#pragma unroll
        for (int by = 0; by < BY; ++by)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[bx][by][r] += red[((bx * BY + by) * 16 + r) * 64 + lane];
    }
  }
  if (wave != 0) return;
  // padded, transposed partial map: every row and column of the tile exists,
  // so the stores need no bounds checks; lanes store consecutive y
  const int ldh = 32 * md.n_yt;
  double *out = part + md.part_off + it.b * part_slice_size(md) +
                (int64_t)(x0 + 4 * kh) * ldh + y0 + c32;
#pragma unroll
  for (int bx = 0; bx < BX; ++bx)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double *o = out + (int64_t)(32 * bx + (r & 3) + 8 * (r >> 2)) * ldh;
#pragma unroll
      for (int by = 0; by < BY; ++by) o[32 * by] = acc[bx][by][r];
    }
}

// Numerator, per-pixel VALU form, over a work list of items (m, 256-pixel
// block, slice).  With a queue, every workgroup pulls the next item from a
// device counter (a persistent grid; items are ordered largest first);
// without one, workgroups stride over the list.
__global__ void __launch_bounds__(256) k_num_pix(const GeomDev *__restrict__ geoms,
                                                 const ModelDev *__restrict__ models,
                                                 const Item *__restrict__ items, int n_it,
                                                 const float4 *__restrict__ terms,
                                                 const int *__restrict__ st_ws,
                                                 double *__restrict__ part, int *queue) {
  __shared__ float4 stage[kPixStage];
  __shared__ int next;
  int i = blockIdx.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      i = next;
      __syncthreads();
    }
    if (i >= n_it) break;
    num_pix_item(items[i], geoms, models, terms, st_ws, part, stage);
    if (!queue) i += gridDim.x;
  }
}

// Numerator, matrix-core form, over a work list of workgroup items.  With a
// queue, every workgroup pulls the next item (largest first) from a device
// counter (a persistent grid); without one, workgroups stride over the list.
// Variants of different tile shapes share one launch; the register budget is
// that of the 2x2 tile (two waves per SIMD, with the MFMA accumulators in
// ordinary VGPRs).
__global__ void __launch_bounds__(256, 2) k_num_mfma(const GeomDev *__restrict__ geoms,
                                                  const ModelDev *__restrict__ models,
                                                  const Item *__restrict__ items, int n_it,
                                                  const float4 *__restrict__ terms,
                                                  const double *__restrict__ gauss,
                                                  const int *__restrict__ st_ws,
                                                  double *__restrict__ part, int *queue) {
  __shared__ __attribute__((aligned(16))) float4 cs[4][KC2];
  __shared__ double red[4 * 16 * 64];
  __shared__ int next;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int i = blockIdx.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      i = next;
      __syncthreads();
    }
    if (i >= n_it) break;
    const Item it = items[i];
    switch (it.c) {
      case 2: num_tile_item<1, 1, false>(it, geoms, models, terms, gauss, st_ws, part, cs[wave], wave, red); break;
      case 3: num_tile_item<2, 1, false>(it, geoms, models, terms, gauss, st_ws, part, cs[wave], wave, red); break;
      case 4: num_tile_item<1, 2, false>(it, geoms, models, terms, gauss, st_ws, part, cs[wave], wave, red); break;
      case 6: num_tile_item<1, 1, true>(it, geoms, models, terms, gauss, st_ws, part, cs[wave], wave, red); break;
      default: num_tile_item<2, 2, false>(it, geoms, models, terms, gauss, st_ws, part, cs[wave], wave, red); break;
    }
    if (!queue) i += gridDim.x;
  }
}

// ---------------------------------------------------------------------------
// Whole-map matrix-core numerator.  One workgroup of eight waves (two per
// SIMD) computes one slice of the terms for the model's entire unique-pixel
// map (n_xt x n_yt = 7 x 7 blocks of 32x32).  Per chunk of 32 terms the 512
// threads generate the operands of every block once (row i of A =
// 2^(cx x^2)(C0 + C1 x^2) and column i of B = 2^(cy y^2), thread i % 256
// for terms 4 (i / 256) .. + 3 of each group of eight) into LDS, double
// buffered, while the waves run the previous chunk's MFMAs.  Operand rows
// hold a chunk's 32 terms contiguously (plus 4 floats of padding), so one
// 16-byte LDS read gives a lane its value for four MFMA steps: in a group of
// eight terms, half-wave kh supplies term 4 kh + j at step j, in A and B
// alike (the contraction index is a sum, so any consistent assignment is
// exact).  Wave w owns the six consecutive row-major blocks 6w .. 6w + 5 and
// accumulates them over the whole slice in FP32 matrix-core accumulators;
// the 49th block (6, 6) is shared out by steps (wave w takes steps 2w, 2w + 1
// of every chunk) and its eight partial sums are added in wave order.  Every
// SIMD so carries 12.25 blocks, and while one of its waves waits on operand
// generation the other keeps the matrix core busy.  The slice's partial map
// is stored in FP32 and the slices are summed in FP64 by k_reduce_f32 in a
// fixed order.  Term coefficients are read straight from the term table at
// wave-uniform addresses (scalar loads), a group ahead.  Rows and columns
// past the map get exact zero operands (exponent offset -inf); terms past T
// are the table's zero padding.
// ---------------------------------------------------------------------------
constexpr int kMapC = 32;                 // terms per chunk
constexpr int kMapLd = kMapC + 4;         // floats per operand row (a chunk + padding)
constexpr int kMapWaves = 8;
constexpr int kMapThreads = 64 * kMapWaves;

struct MapLds {
  float a[2][256][kMapLd];                // [buffer][x row][term]
  float b[2][256][kMapLd];                // [buffer][y column][term]
};

template <int W>
__device__ __forceinline__ void num_map_item(const Item it, const ModelDev &md, const GeomDev &g,
                                             const float4 *__restrict__ terms,
                                             const int *__restrict__ st_ws,
                                             double *__restrict__ part, MapLds &L) {
  constexpr int NXB = kMapBlocks, NYB = kMapBlocks, NBLK = NXB * NYB;
  static_assert(32 * NXB <= 256 && 32 * NYB <= 256, "one operand row per thread");
  constexpr int NB = (NBLK - 1) / kMapWaves, Q0 = W * NB;            // owned blocks
  static_assert(NB * kMapWaves == NBLK - 1, "the last block is the shared one");
  constexpr int BX0 = Q0 / NYB, NR = (Q0 + NB - 1) / NYB - BX0 + 1;   // rows of this wave
  constexpr bool OWN_LAST_ROW = BX0 + NR == NXB;
  constexpr int NG = kMapC / 8;                                       // groups per chunk
  constexpr int SPW = kMapC / 2 / kMapWaves;     // steps of the shared block per wave
  static_assert(SPW == 2, "a wave's shared steps lie in one group");
  constexpr int QS = W * SPW / 4;                // the group holding them
  constexpr int H = W / 4;                       // generates terms 4H .. 4H + 3 of a group
  const int tid = threadIdx.x, row = tid & 255;
  const int lane = tid & 63, c32 = lane & 31, kh = lane >> 5;
  int ts, te;
  slice_range(g.T, md.n_slices, it.b, ts, te, kMapC);
  const int n_ch = (st_ws[it.m] == 0) ? (te - ts + kMapC - 1) / kMapC : 0;   // uniform
  const float4 *tb = terms + md.term_off;
  // this thread's generated row / column
  float x2 = 0.f, xoff = -__builtin_inff(), y2 = 0.f, yoff = -__builtin_inff();
  if (row < g.n_ux) { const double x = g.xs[row]; x2 = (float)(x * x); xoff = 0.f; }
  if (row < g.n_uy) { const double y = g.ys[row]; y2 = (float)(y * y); yoff = 0.f; }
  // coefficients of term 8q + 4H + k of chunk ch (only called with n_ch > 0).
  // Slices end on a multiple of 32 terms or at T, and the table is zero from
  // T to the next multiple of 32, so a whole chunk is always in the table and
  // its terms past the slice are zero; the chunk after the last one repeats it.
  auto coef = [&](int ch, int q, int k) {
    return tb[ts + min(ch, n_ch - 1) * kMapC + 8 * q + 4 * H + k];
  };
  auto gen_a = [&](float4 c) { return fast_exp2(fmaf(c.x, x2, xoff)) * fmaf(c.w, x2, c.z); };
  auto gen_b = [&](float4 c) { return fast_exp2(fmaf(c.y, y2, yoff)); };
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  v16f acc[NB], acc_s = zero;
#pragma unroll
  for (int i = 0; i < NB; ++i) acc[i] = zero;
  if (n_ch > 0) {
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      float4 c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = coef(0, q, k);
      const int k4 = 8 * q + 4 * H;
      *reinterpret_cast<float4 *>(&L.a[0][row][k4]) =
          make_float4(gen_a(c[0]), gen_a(c[1]), gen_a(c[2]), gen_a(c[3]));
      *reinterpret_cast<float4 *>(&L.b[0][row][k4]) =
          make_float4(gen_b(c[0]), gen_b(c[1]), gen_b(c[2]), gen_b(c[3]));
    }
  }
  __syncthreads();
  for (int ch = 0; ch < n_ch; ++ch) {
    const int cur = ch & 1, nxt = cur ^ 1;
    // operands of this wave's block rows (and, in group QS, of the last
    // row) and of every block column for the eight terms of group q
    float4 av[2][NR], bv[2][NYB], al[2];
    auto rd = [&](int u, int q) {
#pragma unroll
      for (int r = 0; r < NR; ++r)
        av[u][r] = *reinterpret_cast<const float4 *>(&L.a[cur][32 * (BX0 + r) + c32][8 * q + 4 * kh]);
#pragma unroll
      for (int c = 0; c < NYB; ++c)
        bv[u][c] = *reinterpret_cast<const float4 *>(&L.b[cur][32 * c + c32][8 * q + 4 * kh]);
      if (!OWN_LAST_ROW && q == QS)
        al[u] = *reinterpret_cast<const float4 *>(&L.a[cur][32 * (NXB - 1) + c32][8 * q + 4 * kh]);
    };
    // coefficients of the next chunk's group (after the last chunk, the last
    // chunk's again: what they generate is never read)
    float4 cq[4], cn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cq[k] = coef(ch + 1, 0, k);
    rd(0, 0);
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int u = q & 1;
      // the next group's reads and coefficients go out before this group's
      // MFMAs; the scheduling barriers keep them there
      if (q + 1 < NG) {
        rd(u ^ 1, q + 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) cn[k] = coef(ch + 1, q + 1, k);
      }
      __builtin_amdgcn_sched_barrier(0);
      float ga[4], gb[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
          const float4 &xa = av[u][(Q0 + i) / NYB - BX0];
          const float4 &yb = bv[u][(Q0 + i) % NYB];
          const float fa = j == 0 ? xa.x : j == 1 ? xa.y : j == 2 ? xa.z : xa.w;
          const float fb = j == 0 ? yb.x : j == 1 ? yb.y : j == 2 ? yb.z : yb.w;
          acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fb, acc[i], 0, 0, 0);
        }
        if ((4 * q + j) / SPW == W) {              // this wave's steps of the shared block
          const float4 &xa = OWN_LAST_ROW ? av[u][NR - 1] : al[u];
          const float4 &yb = bv[u][NYB - 1];
          const float fa = j == 0 ? xa.x : j == 1 ? xa.y : j == 2 ? xa.z : xa.w;
          const float fb = j == 0 ? yb.x : j == 1 ? yb.y : j == 2 ? yb.z : yb.w;
          acc_s = __builtin_amdgcn_mfma_f32_32x32x2f32(fa, fb, acc_s, 0, 0, 0);
        }
        // one term of the next chunk's group q beside the MFMAs
        ga[j] = gen_a(cq[j]);
        gb[j] = gen_b(cq[j]);
      }
      const int k4 = 8 * q + 4 * H;
      *reinterpret_cast<float4 *>(&L.a[nxt][row][k4]) = make_float4(ga[0], ga[1], ga[2], ga[3]);
      *reinterpret_cast<float4 *>(&L.b[nxt][row][k4]) = make_float4(gb[0], gb[1], gb[2], gb[3]);
      __builtin_amdgcn_sched_barrier(0);
      if (q + 1 < NG) {
#pragma unroll
        for (int k = 0; k < 4; ++k) cq[k] = cn[k];
      }
    }
    __syncthreads();
  }
  // FP32 partial map of the slice, padded and transposed as k_reduce_f32 reads it
  float *pf = reinterpret_cast<float *>(part + md.part_off) + it.b * part_slice_size(md);
  const int ldh = 32 * NYB;
  auto store = [&](int blk, const v16f &v) {
    float *o = pf + (int64_t)(32 * (blk / NYB) + 4 * kh) * ldh + 32 * (blk % NYB) + c32;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[(int64_t)((r & 3) + 8 * (r >> 2)) * ldh] = v[r];
  };
#pragma unroll
  for (int i = 0; i < NB; ++i) store(Q0 + i, acc[i]);
  // the shared block: the eight waves' partial sums in wave order (the
  // operand buffers are free after the last chunk's barrier)
  float *red = &L.a[0][0][0];
#pragma unroll
  for (int r = 0; r < 16; ++r) red[(W * 16 + r) * 64 + lane] = acc_s[r];
  __syncthreads();
  if (W == kMapWaves - 1) {
    v16f s = zero;
#pragma unroll
    for (int w = 0; w < kMapWaves; ++w)
#pragma unroll
      for (int r = 0; r < 16; ++r) s[r] += red[(w * 16 + r) * 64 + lane];
    store(NBLK - 1, s);
  }
}

__global__ void __launch_bounds__(kMapThreads, 1) k_num_map(const GeomDev *__restrict__ geoms,
                                                           const ModelDev *__restrict__ models,
                                                           const Item *__restrict__ items, int n_it,
                                                           const float4 *__restrict__ terms,
                                                           const int *__restrict__ st_ws,
                                                           double *__restrict__ part, int *queue) {
  __shared__ __attribute__((aligned(16))) MapLds L;
  __shared__ int next;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int i = blockIdx.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      i = __builtin_amdgcn_readfirstlane(next);
      __syncthreads();
    }
    if (i >= n_it) break;
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    // the map shape is 7 x 7 blocks (checked on the host)
    switch (wave) {
      case 0: num_map_item<0>(it, md, g, terms, st_ws, part, L); break;
      case 1: num_map_item<1>(it, md, g, terms, st_ws, part, L); break;
      case 2: num_map_item<2>(it, md, g, terms, st_ws, part, L); break;
      case 3: num_map_item<3>(it, md, g, terms, st_ws, part, L); break;
      case 4: num_map_item<4>(it, md, g, terms, st_ws, part, L); break;
      case 5: num_map_item<5>(it, md, g, terms, st_ws, part, L); break;
      case 6: num_map_item<6>(it, md, g, terms, st_ws, part, L); break;
      default: num_map_item<7>(it, md, g, terms, st_ws, part, L); break;
    }
    __syncthreads();
    if (!queue) i += gridDim.x;
  }
}

// Sum FP32 split-term partial maps (whole-map numerator) in FP64, in a fixed
// order, into the N map.  Item (m, block of 256 consecutive positions of the
// padded partial layout, x * 32 n_yt + y): lane l holds positions 4l..4l+3
// (one float4 per slice), wave w of 8 takes slices w, w + 8, ... in order
// with 16 loads in flight, and the eight waves' sums are added in wave order.
__global__ void __launch_bounds__(512) k_reduce_f32(const GeomDev *__restrict__ geoms,
                                                    const ModelDev *__restrict__ models,
                                                    const Item *__restrict__ items, int n_it,
                                                    const double *__restrict__ part,
                                                    double *__restrict__ pix) {
  __shared__ double red[8][256];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int ldh = 32 * md.n_yt;
    const int p0 = it.a * 256 + 4 * lane;
    const bool valid = p0 < g.n_ux * ldh;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      const float *pp = reinterpret_cast<const float *>(part + md.part_off) + p0;
      const int64_t stride = part_slice_size(md);
      for (int s0 = wave; s0 < md.n_slices; s0 += 8 * 16) {
        float4 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int sl = s0 + 8 * k;
          v[k] = sl < md.n_slices ? *reinterpret_cast<const float4 *>(pp + sl * stride)
                                  : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          acc[0] += (double)v[k].x;
          acc[1] += (double)v[k].y;
          acc[2] += (double)v[k].z;
          acc[3] += (double)v[k].w;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) red[wave][4 * lane + c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 256) {
      const int q = it.a * 256 + threadIdx.x;
      const int x = q / ldh, y = q % ldh;
      if (x < g.n_ux && y < g.n_uy) {
        double v = red[0][threadIdx.x];
        for (int w = 1; w < 8; ++w) v += red[w][threadIdx.x];
        pix[md.pix_off + (int64_t)y * g.n_ux + x] = v;
      }
    }
    __syncthreads();
  }
}

// Sum the split-term partials in a fixed order into the N map.  Item
// (m, block of 64 pixels in the partial maps' order, y fastest); the four
// waves take every fourth slice and their sums are combined in a fixed order.
__global__ void __launch_bounds__(256) k_reduce(const GeomDev *__restrict__ geoms,
                                                const ModelDev *__restrict__ models,
                                                const Item *__restrict__ items, int n_it,
                                                const double *__restrict__ part,
                                                double *__restrict__ pix) {
  __shared__ double red[3][64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    // u walks the map with y fastest, as the partial maps are laid out
    const int u = it.a * 64 + lane;
    const int x = u / g.n_uy, y = u % g.n_uy;
    double acc = 0.0;
    if (u < g.n_pix) {
      const int64_t off = (int64_t)x * (32 * md.n_yt) + y;
      const int64_t stride = part_slice_size(md);
      // eight slices' loads in flight, added in slice order
      if (md.part_f32) {
        const float *pp = reinterpret_cast<const float *>(part + md.part_off) + off;
        for (int s0 = wave; s0 < md.n_slices; s0 += 32) {
          double v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int s = s0 + 4 * k;
            v[k] = s < md.n_slices ? (double)pp[s * stride] : 0.0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) acc += v[k];
        }
      } else {
        const double *pp = part + md.part_off + off;
        for (int s0 = wave; s0 < md.n_slices; s0 += 32) {
          double v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int s = s0 + 4 * k;
            v[k] = s < md.n_slices ? pp[s * stride] : 0.0;
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) acc += v[k];
        }
      }
    }
    if (wave > 0) red[wave - 1][lane] = acc;
    __syncthreads();
    if (wave == 0 && u < g.n_pix)
      pix[md.pix_off + (int64_t)y * g.n_ux + x] = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Bins: sums of the PSF-weighted maps per bin and their FP64 ratio.
// Item (m, bin, 0), launched with 1024 threads: the 16 waves of the block
// share one bin; item (m, first bin, 1), launched with 256 threads: each wave
// takes one of 4 consecutive bins (geometries whose bins all have few
// weights).  binws per model: [Nb | Ib], n_bins doubles each.
// ---------------------------------------------------------------------------
template <int BS>
__global__ void __launch_bounds__(BS) k_bins(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models,
                                              const Item *__restrict__ items, int n_it,
                                              const double *__restrict__ pix,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ vrms2,
                                              double *__restrict__ binws) {
  __shared__ double sh[2 * (BS / 64)];
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const double *Nm = pix + md.pix_off;
    const double *Im = Nm + g.n_pix;
    const bool want_n = vrms2 != nullptr;
    if (it.c == 1) {   // uniform per block: bins it.a + wave, one per wave
      const int lane = threadIdx.x & 63;
      const int b = it.a + (threadIdx.x >> 6);
      if (b >= g.n_bins) continue;   // uniform per wave; no barrier in this variant
      double an[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
      const int e1 = g.bin_ptr[b + 1];
      int e = g.bin_ptr[b] + lane;
      for (; e + 3 * 64 < e1; e += 4 * 64) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double wv = g.bin_w[e + u * 64];
          const int q = g.bin_pix[e + u * 64];
          if (want_n) an[u] += wv * Nm[q];
          ai[u] += wv * Im[q];
        }
      }
      for (int u = 0; e < e1; e += 64, ++u) {
        const double wv = g.bin_w[e];
        const int q = g.bin_pix[e];
        if (want_n) an[u] += wv * Nm[q];
        ai[u] += wv * Im[q];
      }
      double sn = wave_sum((an[0] + an[1]) + (an[2] + an[3]));
      const double si = wave_sum((ai[0] + ai[1]) + (ai[2] + ai[3]));
      if (!want_n) sn = 0.0;
      if (lane == 0) {
        const bool ok = st_ws[it.m] == 0;
        if (binws) {
          binws[md.bin_off + b] = sn;
          binws[md.bin_off + g.n_bins + b] = si;
        }
        if (want_n) vrms2[md.out_off + b] = ok ? sn / si : __builtin_nan("");
      }
      continue;
    }
    const int b = it.a;
    // four independent accumulators keep four gathers in flight per thread
    double an[4] = {0.0, 0.0, 0.0, 0.0}, ai[4] = {0.0, 0.0, 0.0, 0.0};
    const int e1 = g.bin_ptr[b + 1];
    int e = g.bin_ptr[b] + threadIdx.x;
    for (; e + 3 * BS < e1; e += 4 * BS) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double wv = g.bin_w[e + u * BS];
        const int q = g.bin_pix[e + u * BS];
        if (want_n) an[u] += wv * Nm[q];
        ai[u] += wv * Im[q];
      }
    }
    for (int u = 0; e < e1; e += BS, ++u) {
      const double wv = g.bin_w[e];
      const int q = g.bin_pix[e];
      if (want_n) an[u] += wv * Nm[q];
      ai[u] += wv * Im[q];
    }
    // deterministic two-level sums: wave butterflies, then the wave partials
    // in a fixed order
    const double an_w = wave_sum((an[0] + an[1]) + (an[2] + an[3]));
    const double ai_w = wave_sum((ai[0] + ai[1]) + (ai[2] + ai[3]));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
      sh[wv] = an_w;
      sh[BS / 64 + wv] = ai_w;
    }
    __syncthreads();
    double sn = 0.0, si = 0.0;
    if (threadIdx.x == 0)
      for (int w = 0; w < BS / 64; ++w) {
        sn += sh[w];
        si += sh[BS / 64 + w];
      }
    if (!want_n) sn = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      const bool ok = st_ws[it.m] == 0;
      if (binws) {
        binws[md.bin_off + b] = sn;
        binws[md.bin_off + g.n_bins + b] = si;
      }
      if (want_n) vrms2[md.out_off + b] = ok ? sn / si : __builtin_nan("");
    }
  }
}

// Expand the unique-pixel maps to the padded sub-pixel grid.  Item (m, row).
__global__ void __launch_bounds__(256) k_maps(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models,
                                              const Item *__restrict__ items, int n_it,
                                              const double *__restrict__ pix,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ N_map,
                                              double *__restrict__ I_map) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int row = it.a;
    const int iy = g.uy[row];
    const bool ok = st_ws[it.m] == 0;
    for (int c = threadIdx.x; c < g.nxp; c += 256) {
      const int q = iy * g.n_ux + g.ux[c];
      const int64_t o = md.map_off + (int64_t)row * g.nxp + c;
      N_map[o] = ok ? pix[md.pix_off + q] : __builtin_nan("");
      I_map[o] = pix[md.pix_off + g.n_pix + q];
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the bin ratio and of the PSF/bin sums:
//   lambda_N[p] = sum_b W[b,p] cot_b / Ib_b,
//   lambda_I[p] = -sum_b W[b,p] cot_b V_b / Ib_b.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bins_adjoint(const GeomDev *__restrict__ geoms,
                                                      const ModelDev *__restrict__ models,
                                                      const Item *__restrict__ items, int n_it,
                                                      const double *__restrict__ vrms2,
                                                      const double *__restrict__ cot,
                                                      const double *__restrict__ binws,
                                                      const int *__restrict__ st_ws,
                                                      double *__restrict__ pix) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int q = it.a * 256 + threadIdx.x;
    if (q >= g.n_pix) continue;
    const double *Ib = binws + md.bin_off + g.n_bins;
    double ln = 0.0, li = 0.0;
    if (st_ws[it.m] == 0) {
      for (int e = g.pix_ptr[q]; e < g.pix_ptr[q + 1]; ++e) {
        const int b = g.pix_bin[e];
        const double c = cot[md.out_off + b] / Ib[b];
        ln += g.pix_w[e] * c;
        li -= g.pix_w[e] * c * vrms2[md.out_off + b];
      }
    }
    pix[md.pix_off + 2 * (int64_t)g.n_pix + q] = ln;
    pix[md.pix_off + 3 * (int64_t)g.n_pix + q] = li;
  }
}

// ---------------------------------------------------------------------------
// Per-term adjoint sensitivities, per-pixel VALU form.  Lanes are terms; the
// unique pixels (x^2, y^2, lambda_N) are staged through LDS 256 at a time.
//   S0 = sum_p lambda E F,  S1 = sum_p lambda x^2 E F,
//   Sg = sum_p lambda y^2 E F (C0 + C1 x^2),
// with E F = exp(-c1 x^2 - gamma y^2).  Item (m, 256-term block).
// sens per model: [S0 | S1 | Sg], T doubles each.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sens_pix_item(const Item it, const GeomDev *__restrict__ geoms,
    const ModelDev *__restrict__ models, const float4 *__restrict__ terms, const double *__restrict__ pix, const int *__restrict__ st_ws, double *__restrict__ sens, char *smem) {
  float *sx = reinterpret_cast<float *>(smem), *sy = sx + 256, *sl = sy + 256;

  const ModelDev md = models[it.m];
  const GeomDev g = geoms[md.geom];
  if (st_ws[it.m] != 0) return;   // uniform per block
  const int t = it.a * 256 + threadIdx.x;
  const bool valid = t < g.T;
  const float4 c = valid ? terms[md.term_off + t] : make_float4(0.f, 0.f, 0.f, 0.f);
  const double *lam = pix + md.pix_off + 2 * (int64_t)g.n_pix;
  double a0 = 0.0, a1 = 0.0, ag = 0.0;
  for (int base = 0; base < g.n_pix; base += 256) {
    const int q = base + threadIdx.x;
    __syncthreads();
    if (q < g.n_pix) {
      const double x = g.xs[q % g.n_ux], y = g.ys[q / g.n_ux];
      sx[threadIdx.x] = (float)(x * x);
      sy[threadIdx.x] = (float)(y * y);
      sl[threadIdx.x] = (float)lam[q];
    } else {
      sx[threadIdx.x] = 0.f;
      sy[threadIdx.x] = 0.f;
      sl[threadIdx.x] = 0.f;
    }
    __syncthreads();
    const int cnt = min(256, g.n_pix - base);
    float s0 = 0.f, s1 = 0.f, sg = 0.f;
    for (int e = 0; e < cnt; ++e) {
      const float x2 = sx[e], y2 = sy[e];
      const float le = sl[e] * fast_exp2(fmaf(c.x, x2, c.y * y2));
      s0 += le;
      s1 = fmaf(le, x2, s1);
      sg = fmaf(le * y2, fmaf(c.w, x2, c.z), sg);
    }
    a0 += s0;
    a1 += s1;
    ag += sg;
  }
  if (valid) {
    double *S = sens + md.sens_off;
    S[t] = a0;
    S[g.T + t] = a1;
    S[2 * (int64_t)g.T + t] = ag;
  }
}


// ---------------------------------------------------------------------------
// Per-term adjoint sensitivities, matrix-core form.  With E_t(x) = 2^(cx x^2)
// and F_t(y) = 2^(cy y^2) on the unique-pixel map,
//   G[x, t] = sum_y lambda[x, y] F_t(y),   H[x, t] = sum_y lambda[x, y] y^2 F_t(y)
// are two FP32 contractions over y sharing the lambda operand, and
//   S0_t = sum_x E G,  S1_t = sum_x x^2 E G,  Sg_t = sum_x E (C0 + C1 x^2) H.
// Item (m, 32-row x tile, tile of kSensTerms terms); wave w owns a quarter
// of the tile's terms and takes them as 32-term column blocks one after the
// other (lane l: term l % 32, y pair l / 32).  lambda is staged through LDS
// 256 rows of y at a time (once per item when the map has at most 256
// distinct |y|).  G and H are summed in FP32 over up to 128 y values; each
// such partial goes straight through the x epilogue (each lane's 16 rows in
// FP32) and the partial S0, S1, Sg are added in FP64, so no per-row FP64
// accumulators are live.  Output: per x tile, [S0 | S1 | Sg] (T doubles
// each).
// ---------------------------------------------------------------------------
constexpr int YC = 256;
constexpr int kSensWave = kSensTerms / 4;   // terms per wave of an item

__device__ __forceinline__ void sens_mfma_item(const Item it, const GeomDev *__restrict__ geoms,
                                               const ModelDev *__restrict__ models,
                                               const float4 *__restrict__ terms,
                                               const double *__restrict__ pix,
                                               const int *__restrict__ st_ws,
                                               double *__restrict__ sens, char *smem) {
  // lambda[x][y] staged x-major with the y values of each half-wave kh
  // (y = 2 s + kh) consecutive, so one 16-byte read gives a lane four steps'
  // operands; rows padded by 4 floats
  float (*lam)[YC + 4] = reinterpret_cast<float (*)[YC + 4]>(smem);
  float *ysq = reinterpret_cast<float *>(smem + 32 * (YC + 4) * sizeof(float));
  float *xsq = ysq + YC;                   // x^2 of the tile's rows (0 past the map)
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c32 = lane & 31, kh = lane >> 5;
  const ModelDev md = models[it.m];
  const GeomDev g = geoms[md.geom];
  if (st_ws[it.m] != 0) return;   // uniform per block
  const int x0 = it.a * 32;
  const double *lamN = pix + md.pix_off + 2 * (int64_t)g.n_pix;
  const int n_yb = (g.n_uy + YC - 1) / YC;
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int h = 0; h < kSensWave / 32; ++h) {
    // this block's terms: it.b*kSensTerms + w*kSensWave + h*32 + (0..31)
    const int t = it.b * kSensTerms + wave * kSensWave + h * 32 + c32;
    const bool vt = t < g.T;
    const float4 c = vt ? terms[md.term_off + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    double s0 = 0.0, s1 = 0.0, sg = 0.0;
    for (int ybi = 0; ybi < n_yb; ++ybi) {
      const int yb = ybi * YC;
      const int ny = min(YC, g.n_uy - yb);
      if (h == 0 || n_yb > 1) {         // uniform per block
        __syncthreads();
        // the rows the steps read: ny rounded up to whole blocks of 8 y
        const int rows = min(YC, (ny + 7) & ~7);
        for (int e = threadIdx.x; e < rows * 32; e += 256) {
          const int yy = e >> 5, xx = e & 31;
          float v = 0.f;
          if (yy < ny && x0 + xx < g.n_ux) v = (float)lamN[(int64_t)(yb + yy) * g.n_ux + x0 + xx];
          lam[xx][(yy & 1) * (YC / 2) + (yy >> 1)] = v;
        }
        for (int e = threadIdx.x; e < rows; e += 256) {
          float v = 0.f;
          if (e < ny) { const double y = g.ys[yb + e]; v = (float)(y * y); }
          ysq[(e & 1) * (YC / 2) + (e >> 1)] = v;
        }
        if (threadIdx.x < 32) {
          const int xr = x0 + threadIdx.x;
          float v = 0.f;
          if (xr < g.n_ux) { const double xv = g.xs[xr]; v = (float)(xv * xv); }
          xsq[threadIdx.x] = v;
        }
        __syncthreads();
      }
      for (int y0 = 0; y0 < ny; y0 += 128) {
        // operands lambda[x0 + c32][y0 + 2 s + kh] and y^2 for up to 128 y
        // values, four steps (8 y) per 16-byte read (rows past ny hold zero
        // lambda; y0 + 127 < YC)
        v16f dg = zero, dh = zero;
        const int nb = min(16, (ny - y0 + 7) / 8);   // uniform per block
        const float *lrow = &lam[c32][kh * (YC / 2) + y0 / 2];
        const float *yrow = ysq + kh * (YC / 2) + y0 / 2;
        // blocks alternate between two register buffers: the next block's
        // operands read and its exponentials taken behind the current MFMAs
        // (a read one block past the last stays inside the padded row and is
        // not used)
        float ra[2][4], ry[2][4], bb[2][4], by[2][4];
        auto load = [&](int u, int qb) {
          const float4 a4 = *reinterpret_cast<const float4 *>(lrow + 4 * qb);
          const float4 y4 = *reinterpret_cast<const float4 *>(yrow + 4 * qb);
          ra[u][0] = a4.x; ra[u][1] = a4.y; ra[u][2] = a4.z; ra[u][3] = a4.w;
          ry[u][0] = y4.x; ry[u][1] = y4.y; ry[u][2] = y4.z; ry[u][3] = y4.w;
        };
        auto expo = [&](int u) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            bb[u][j] = fast_exp2(c.y * ry[u][j]);
            by[u][j] = bb[u][j] * ry[u][j];
          }
        };
        auto mfma4 = [&](int u) {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            dg = __builtin_amdgcn_mfma_f32_32x32x2f32(ra[u][j], bb[u][j], dg, 0, 0, 0);
            dh = __builtin_amdgcn_mfma_f32_32x32x2f32(ra[u][j], by[u][j], dh, 0, 0, 0);
          }
        };
        load(0, 0);
        expo(0);
        for (int qb = 0; qb < nb; qb += 2) {
          load(1, qb + 1);
          __builtin_amdgcn_sched_barrier(0);
          mfma4(0);
          expo(1);
          // taken here, not sunk into the branch below
          asm volatile("" ::"v"(bb[1][0]), "v"(bb[1][1]), "v"(bb[1][2]), "v"(bb[1][3]),
                       "v"(by[1][0]), "v"(by[1][1]), "v"(by[1][2]), "v"(by[1][3]));
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
          __builtin_amdgcn_sched_barrier(0);
          if (qb + 1 < nb) {                 // uniform
            load(0, qb + 2);
            __builtin_amdgcn_sched_barrier(0);
            mfma4(1);
            expo(0);
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
            __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
        // rows past the map have zero lambda, so zero sums; each lane's 16
        // rows in FP32, the y blocks and the lanes in FP64
        float f0 = 0.f, f1 = 0.f, fg = 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const float x2 = xsq[mfma_row(r, lane)];
          const float e = fast_exp2(c.x * x2);
          const float ed = e * dg[r];
          f0 += ed;
          f1 = fmaf(x2, ed, f1);
          fg = fmaf(e * fmaf(c.w, x2, c.z), dh[r], fg);
        }
        s0 += (double)f0;
        s1 += (double)f1;
        sg += (double)fg;
      }
    }
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 32, 64);
    sg += __shfl_xor(sg, 32, 64);
    if (kh == 0 && vt) {
      double *S = sens + md.sens_off + (int64_t)it.a * 3 * g.T;
      S[t] = s0;
      S[g.T + t] = s1;
      S[2 * (int64_t)g.T + t] = sg;
    }
  }
}

constexpr int kSensSmem = (32 * (YC + 4) + YC + 32) * (int)sizeof(float);
static_assert(kSensSmem >= 3 * 256 * (int)sizeof(float), "per-pixel sensitivity LDS");

// Adjoint sensitivities over a work list, variant in Item::c (0 per-pixel
// VALU, items (m, 256-term block); 1 MFMA, items (m, x tile, 256-term tile));
// queue-driven or strided as k_num.
__global__ void __launch_bounds__(256) k_sens(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models,
                                              const Item *__restrict__ items, int n_it,
                                              const float4 *__restrict__ terms,
                                              const double *__restrict__ pix,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ sens, int *queue) {
  __shared__ __attribute__((aligned(16))) char smem[kSensSmem];
  __shared__ int next;
  int i = blockIdx.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      i = next;
      __syncthreads();
    }
    if (i >= n_it) break;
    const Item it = items[i];
    if (it.c == 0)
      sens_pix_item(it, geoms, models, terms, pix, st_ws, sens, smem);
    else
      sens_mfma_item(it, geoms, models, terms, pix, st_ws, sens, smem);
    __syncthreads();
    if (!queue) i += gridDim.x;
  }
}

// ---------------------------------------------------------------------------
// Per-term adjoint sensitivities, wide matrix-core form: the contractions of
// sens_mfma_item for a part of XT <= 4 consecutive 32-row x tiles at once, so
// that each generated F_t(y) and y^2 F_t(y) feeds 2 XT MFMAs.  lambda_N of
// the part's rows is staged in LDS for up to 256 y at a time (once per item
// when the map has at most 256 distinct |y|) in the layout the MFMA steps
// read: row x holds, for each half kh of the wave, the values at y = 2s + kh
// for consecutive steps s, so one 16-byte read gives a lane four steps'
// operands (a quarter of the LDS instructions; rows are padded by 4 floats
// against bank conflicts).  Per term group the FP32 matrix-core sums run over
// all y (no FP64 fold: the 2 XT accumulator blocks take 128 registers at
// XT = 4), the next four steps' operands read and their exponentials taken
// behind the current MFMAs.  Item (m, part p | XT << 16 covering x tiles 4p ..
// 4p + XT - 1, first 32-term group, end group); eight waves, two per SIMD,
// so that one wave's exponentials and epilogue run beside the other's
// MFMAs; wave w takes the item's groups w, w + 8, ...; output per part,
// [S0 | S1 | Sg] (T doubles each), as sens_mfma_item's per x tile.
// ---------------------------------------------------------------------------
constexpr int kWideTiles = 4;
constexpr int kWideLd = YC + 4;   // floats per staged x row: 2 halves x YC/2 steps + pad

struct SensWideLds {
  float lam[32 * kWideTiles][kWideLd];
  float ysq[YC];                   // [kh][s] = y^2 at y = 2s + kh
  float xsq[32 * kWideTiles];      // x^2 of the part's rows (0 past the map)
};

template <int XT>
__device__ __forceinline__ void sens_wide_item(const Item it, const ModelDev &md, const GeomDev &g,
                                               const float4 *__restrict__ terms,
                                               const double *__restrict__ pix,
                                               double *__restrict__ sens, SensWideLds &L,
                                               int wave) {
  const int lane = threadIdx.x & 63, c32 = lane & 31, kh = lane >> 5;
  const int part = it.a & 0xffff;
  const int x0 = 32 * kWideTiles * part;
  const double *lamN = pix + md.pix_off + 2 * (int64_t)g.n_pix;
  const int n_uy = __builtin_amdgcn_readfirstlane(g.n_uy);
  const int n_yb = (n_uy + YC - 1) / YC;
  const int g0 = it.b, g1 = it.c;
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  bool staged = false;
  constexpr int NT = 64 * kWideWaves;
  if (threadIdx.x < 32 * XT) {
    const int xr = x0 + threadIdx.x;
    float v = 0.f;
    if (xr < g.n_ux) { const double xv = g.xs[xr]; v = (float)(xv * xv); }
    L.xsq[threadIdx.x] = v;          // read after the first staging barrier
  }
  // the group's term coefficients, loaded one group ahead
  auto coef = [&](int gr) {
    const int t = gr * 32 + c32;
    return (gr < g1 && t < g.T) ? terms[md.term_off + t] : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  float4 cnext = coef(g0 + wave);
  for (int gr = g0 + wave; gr - wave < g1; gr += kWideWaves) {   // same trip count in every wave
    const int t = gr * 32 + c32;
    const bool vt = gr < g1 && t < g.T;
    const float4 c = cnext;
    cnext = coef(gr + kWideWaves);
    v16f dg[XT], dh[XT];
#pragma unroll
    for (int bt = 0; bt < XT; ++bt) dg[bt] = dh[bt] = zero;
    for (int ybi = 0; ybi < n_yb; ++ybi) {
      const int yb = ybi * YC;
      const int ny = min(YC, n_uy - yb);
      if (!staged || n_yb > 1) {        // uniform per block
        __syncthreads();
        for (int e = threadIdx.x; e < YC * 32 * XT; e += NT) {
          const int yy = e / (32 * XT), xx = e % (32 * XT);
          float v = 0.f;
          if (yy < ny && x0 + xx < g.n_ux) v = (float)lamN[(int64_t)(yb + yy) * g.n_ux + x0 + xx];
          L.lam[xx][(yy & 1) * (YC / 2) + (yy >> 1)] = v;
        }
        for (int e = threadIdx.x; e < YC; e += NT) {
          float v = 0.f;
          if (e < ny) { const double y = g.ys[yb + e]; v = (float)(y * y); }
          L.ysq[(e & 1) * (YC / 2) + (e >> 1)] = v;
        }
        __syncthreads();
        staged = true;
      }
      // four y pairs per block of steps (rows past ny hold zero lambda);
      // blocks alternate between two operand buffers, the next block's
      // operands read and its exponentials taken behind the current MFMAs
      const int blocks = (((ny + 1) >> 1) + 3) >> 2;
      const float *yrow = L.ysq + kh * (YC / 2);
      float4 a4[2][XT], y4[2];
      float bx[2][4], bxy[2][4];
      auto load = [&](int buf, int q) {
        q = min(q, YC / 8 - 1);                  // past the last block: a harmless re-read
#pragma unroll
        for (int bt = 0; bt < XT; ++bt)
          a4[buf][bt] = *reinterpret_cast<const float4 *>(&L.lam[32 * bt + c32][kh * (YC / 2) + 4 * q]);
        y4[buf] = *reinterpret_cast<const float4 *>(yrow + 4 * q);
      };
      auto expo = [&](int buf) {
        const float ys[4] = {y4[buf].x, y4[buf].y, y4[buf].z, y4[buf].w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          bx[buf][u] = fast_exp2(c.y * ys[u]);
          bxy[buf][u] = bx[buf][u] * ys[u];
        }
      };
      auto mfma4 = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int bt = 0; bt < XT; ++bt) {
            const float4 &av4 = a4[buf][bt];
            const float av = u == 0 ? av4.x : (u == 1 ? av4.y : (u == 2 ? av4.z : av4.w));
            dg[bt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bx[buf][u], dg[bt], 0, 0, 0);
            dh[bt] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bxy[buf][u], dh[bt], 0, 0, 0);
          }
      };
      load(0, 0);
      expo(0);
      for (int q = 0; q < blocks; q += 2) {
        load(1, q + 1);
        __builtin_amdgcn_sched_barrier(0);
        mfma4(0);
        expo(1);
        // taken here, not sunk into the branch below
        asm volatile("" ::"v"(bx[1][0]), "v"(bx[1][1]), "v"(bx[1][2]), "v"(bx[1][3]),
                     "v"(bxy[1][0]), "v"(bxy[1][1]), "v"(bxy[1][2]), "v"(bxy[1][3]));
        // half the MFMAs go out before the exponentials wait for their reads
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * XT, 0);
        __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4 * XT, 0);
        __builtin_amdgcn_sched_barrier(0);
        if (q + 1 < blocks) {                  // uniform
          load(0, q + 2);
          __builtin_amdgcn_sched_barrier(0);
          mfma4(1);
          expo(0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4 * XT, 0);
          __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, 4 * XT, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // rows past the map have zero lambda, so zero g and h.  Each lane's 16
    // rows of a tile are summed in FP32 (beside the FP32 matrix-core sums over
    // y, a relative error of the same order), the tiles in FP64.
    double s0 = 0.0, s1 = 0.0, sg = 0.0;
#pragma unroll
    for (int bt = 0; bt < XT; ++bt) {
      float f0 = 0.f, f1 = 0.f, fg = 0.f;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float x2 = L.xsq[32 * bt + mfma_row(r, lane)];
        const float e = fast_exp2(c.x * x2);
        const float ed = e * dg[bt][r];
        f0 += ed;
        f1 = fmaf(x2, ed, f1);
        fg = fmaf(e * fmaf(c.w, x2, c.z), dh[bt][r], fg);
      }
      s0 += (double)f0;
      s1 += (double)f1;
      sg += (double)fg;
    }
    s0 += __shfl_xor(s0, 32, 64);
    s1 += __shfl_xor(s1, 32, 64);
    sg += __shfl_xor(sg, 32, 64);
    if (kh == 0 && vt) {
      double *S = sens + md.sens_off + (int64_t)part * 3 * g.T;
      S[t] = s0;
      S[g.T + t] = s1;
      S[2 * (int64_t)g.T + t] = sg;
    }
  }
}

// Wide adjoint sensitivities over a work list (one workgroup of eight waves
// per CU: the staged lambda takes 135 KB of LDS); queue-driven or strided as
// k_sens.
__global__ void __launch_bounds__(64 * kWideWaves, 1) k_sens_wide(const GeomDev *__restrict__ geoms,
                                                      const ModelDev *__restrict__ models,
                                                      const Item *__restrict__ items, int n_it,
                                                      const float4 *__restrict__ terms,
                                                      const double *__restrict__ pix,
                                                      const int *__restrict__ st_ws,
                                                      double *__restrict__ sens, int *queue) {
  __shared__ __attribute__((aligned(16))) SensWideLds L;
  __shared__ int next;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int i = blockIdx.x;
  for (;;) {
    if (queue) {
      if (threadIdx.x == 0) next = atomicAdd(queue, 1);
      __syncthreads();
      i = next;
      __syncthreads();
    }
    if (i >= n_it) break;
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] == 0) {            // uniform per block
      switch (it.a >> 16) {
        case 1: sens_wide_item<1>(it, md, g, terms, pix, sens, L, wave); break;
        case 2: sens_wide_item<2>(it, md, g, terms, pix, sens, L, wave); break;
        case 3: sens_wide_item<3>(it, md, g, terms, pix, sens, L, wave); break;
        default: sens_wide_item<4>(it, md, g, terms, pix, sens, L, wave); break;
      }
    }
    __syncthreads();
    if (!queue) i += gridDim.x;
  }
}

// ---------------------------------------------------------------------------
// FP64 chain from per-term sensitivities to the parameters.  Forward-mode
// dual numbers carry d/d(inclination) through the deprojection and the term
// coefficients.  Items (m, k, jb): wave w of the workgroup takes mass
// Gaussian j = 4 jb + w (BH last) and its lanes the u-nodes.  Chain rows per
// model (doubles, after the sensitivity blocks): [K][J1][3] = (d/di, d/db_k,
// H_kj) for the terms of (k, j), with H_kj = sum_n (S0 c0 + S1 c1) the
// derivative with respect to the amplitude product I0_k M_j.  The
// surface-brightness path of I0_k is k_sb_adj's.
// ---------------------------------------------------------------------------
struct dual {
  double v, d;
};
__device__ inline dual operator+(dual a, dual b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline dual operator-(dual a, dual b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline dual operator*(dual a, dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline dual operator/(dual a, dual b) {
  const double r = a.v / b.v;
  return {r, (a.d - r * b.d) / b.v};
}
__device__ inline dual operator*(double s, dual a) { return {s * a.v, s * a.d}; }
__device__ inline dual operator-(double s, dual a) { return {s - a.v, -a.d}; }
__device__ inline dual operator/(double s, dual a) {
  const double r = s / a.v;
  return {r, -r * a.d / a.v};
}
__device__ inline dual dsqrt(dual a) {
  const double r = sqrt(a.v);
  return {r, 0.5 * a.d / r};
}
__device__ inline dual dconst(double v) { return {v, 0.0}; }

__device__ inline double *chain_rows(double *sens, const ModelDev &md, const GeomDev &g) {
  return sens + md.sens_off + 3 * (int64_t)md.n_sens_parts * g.T;
}

__global__ void __launch_bounds__(256) k_chain(const GeomDev *__restrict__ geoms,
                                               const ModelDev *__restrict__ models,
                                               const Item *__restrict__ items, int n_it,
                                               ParamsDev p, double *__restrict__ sens,
                                               const int *__restrict__ st_ws) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;   // uniform per block; k_grads writes NaN
    const int k = it.a;
    const int J1 = g.J1, J = J1 - 1;
    double *rows = chain_rows(sens, md, g);
    const double qok = g.lum_q[k], sk = g.lum_sigma[k];
    const int j = it.b * 4 + wave;
    if (j >= J1) continue;            // uniform per wave; no block barrier follows
    const double inc = p.inc[it.m];
    const dual s = {sin(inc), cos(inc)};
    const dual c = {cos(inc), -sin(inc)};
    const dual si2 = s * s, ci2 = c * c;
    const double G = grav_const();
    const double sp = g.s_pc;
    const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
    const double b = 1.0 / (1.0 - p.beta[md.lum_off + k]);
    const dual qk = dsqrt(qok * qok - ci2) / s;
    const double alpha = 0.5 / (sk * sk);
    const dual alphaq = dconst(alpha) / (qk * qk);
    const dual nu1 = dconst(qok / (sqrt(2.0 * kPi) * sk)) / qk;   // nu0 / I0
    dual e2;
    double r, Kt, Mj;
    if (j < J) {
      const double qo = g.mass_q[j], sj = g.mass_sigma[j];
      const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
      const dual qj = dsqrt(qo * qo - ci2) / s;
      e2 = 1.0 - qj * qj;
      r = 0.5 / (sj * sj);
      Kt = sqrt(2.0 / kPi) * G / (sp * sj);
      Mj = p.mass_scale[it.m] * 2.0 * kPi * S0 * (sp * sj) * (sp * sj) * qo;
    } else {
      e2 = dconst(0.0);
      r = 0.5 / (g.bh_sigma * g.bh_sigma);
      Kt = sqrt(2.0 / kPi) * G / (sp * g.bh_sigma);
      Mj = p.m_bh[it.m];
    }
    const double amp = I0 * Mj;
    const double *S0a = sens + md.sens_off;
    const int np_ = md.n_sens_parts;
    double acc_i = 0.0, acc_b = 0.0, hj = 0.0;
    for (int n = lane; n < g.n_u; n += 64) {
      const int64_t t = ((int64_t)k * J1 + j) * g.n_u + n;
      // partial sensitivities of the x-row blocks, summed in block order;
      // eight blocks' loads are issued before their adds
      double S0 = 0.0, S1 = 0.0, Sg = 0.0;
      for (int q0 = 0; q0 < np_; q0 += 8) {
        double v0[8], v1[8], v2[8];
#pragma unroll
        for (int qq = 0; qq < 8; ++qq) {
          v0[qq] = v1[qq] = v2[qq] = 0.0;
          if (q0 + qq < np_) {
            const double *blk = S0a + (int64_t)(q0 + qq) * 3 * g.T;
            v0[qq] = blk[t];
            v1[qq] = blk[g.T + t];
            v2[qq] = blk[2 * (int64_t)g.T + t];
          }
        }
#pragma unroll
        for (int qq = 0; qq < 8; ++qq) {
          S0 += v0[qq];
          S1 += v1[qq];
          Sg += v2[qq];
        }
      }
      const double u = g.u[n], wq = g.w[n];
      const double u2 = u * u;
      const dual h = 1.0 - u2 * e2;
      const double c1 = alpha + r * u2;
      const dual A = alphaq + (r * u2) * (dconst(1.0) / h);
      const dual a = c1 * si2 + A * ci2;
      const dual gam = c1 * A / a;
      const dual sh_ = dsqrt(h);
      const dual base = (Kt * r * u2) * nu1;                    // per unit I0 M
      const dual gg = base / (A * h * sh_);
      const dual ww = 2.0 * base / sh_;
      const dual P = (ci2 + b * si2) * gg;
      const dual Q = si2 * (ww - (2.0 * c1 * b) * gg);
      const dual f = wq * dsqrt(kPi / a);
      const dual c0 = f * P, c1u = f * Q;                       // C = I0 M c
      acc_i += amp * (S0 * c0.d + S1 * c1u.d) - Sg * gam.d;
      // dC0/db = f si2 g, dC1/db = -2 f si2 c1 g
      acc_b += amp * f.v * si2.v * gg.v * (S0 - 2.0 * c1 * S1);
      hj += S0 * c0.v + S1 * c1u.v;
    }
    acc_i = wave_sum(acc_i);
    acc_b = wave_sum(acc_b);
    hj = wave_sum(hj);
    if (lane == 0) {
      double *o = rows + ((int64_t)k * J1 + j) * 3;
      o[0] = acc_i;
      o[1] = acc_b;
      o[2] = hj;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of a small-map model (its unique-pixel map fits one 32x32 block):
// the per-term sensitivities and the FP64 chain in one pass, lane = term.
// Each term's coefficients are computed in place as FP64 dual numbers
// carrying d/di (the set-up and term formulas of the forward), rounded to
// FP32 for the sums
//   S0 = sum_p lambda E F,  S1 = sum_p lambda x^2 E F,
//   Sg = sum_p lambda y^2 E F (C0 + C1 x^2),   E F = exp(-c1 x^2 - gamma y^2):
// F(y) and y^2 F(y) for every y in registers, then per x the FP32 sums
// g = sum_y lambda F and h = sum_y lambda y^2 F (lambda broadcast from LDS,
// four y at a time) and the x-sums in FP32, converted to FP64; the y loops
// are unrolled for the map's number of y quads.
// The term's chain values (those of k_chain) go through LDS and every (k, j)
// row is summed over its u-nodes by one wave in a fixed order.  Item (m,
// first tracer k0 | k1 << 16): tracers k0 <= k < k1 (at most
// kSmallAdjTracers); lambda_N, the squared coordinates, every mass
// Gaussian's and every tracer's set-up values are staged in LDS once per
// item, and the item's (k, j) rows, tracer-major, are taken in windows of
// whole rows with at most kAdjTerms terms, so that the passes of 256 terms
// run across tracers.  Writes the chain rows of k_chain (the model has no
// partial sensitivity blocks).
// ---------------------------------------------------------------------------
constexpr int kSmallMap = 32;
constexpr int kAdjTerms = kSmallAdjTerms;

// The three FP32 map sums of one term (lane) over NYQ quads of y (past the
// map y^2 = 0 and lambda = 0, so the padding adds nothing) and nx values of
// x: F(y) and y^2 F(y) in registers, per x g and h over y with lambda read
// four at a time from LDS (the same address in every lane), then E(x).
template <int NYQ>
__device__ __forceinline__ void small_sums(float cx, float cy, float C0, float C1,
                                           const float (*lam)[kSmallMap], const float *xsq,
                                           const float *ysq, int nx, float &s0, float &s1,
                                           float &sg) {
  float F[4 * NYQ], Fy[4 * NYQ];
#pragma unroll
  for (int yy = 0; yy < 4 * NYQ; ++yy) {
    const float y2 = ysq[yy];
    F[yy] = fast_exp2(cy * y2);
    Fy[yy] = F[yy] * y2;
  }
  // an offset the compiler cannot prove loop-invariant, so that the lambda
  // reads are not hoisted out of the caller's term loop into registers
  int zoff;
  asm volatile("s_mov_b32 %0, 0" : "=s"(zoff));
  s0 = 0.f;
  s1 = 0.f;
  sg = 0.f;
#pragma unroll 2
  for (int xx = 0; xx < nx; ++xx) {
    const float4 *lr = reinterpret_cast<const float4 *>(lam[xx]) + zoff;
    float gs = 0.f, hs = 0.f;
#pragma unroll
    for (int yq = 0; yq < NYQ; ++yq) {
      const float4 l = lr[yq];
      gs = fmaf(l.x, F[4 * yq], gs);
      hs = fmaf(l.x, Fy[4 * yq], hs);
      gs = fmaf(l.y, F[4 * yq + 1], gs);
      hs = fmaf(l.y, Fy[4 * yq + 1], hs);
      gs = fmaf(l.z, F[4 * yq + 2], gs);
      hs = fmaf(l.z, Fy[4 * yq + 2], hs);
      gs = fmaf(l.w, F[4 * yq + 3], gs);
      hs = fmaf(l.w, Fy[4 * yq + 3], hs);
    }
    const float x2 = xsq[xx];
    const float E = fast_exp2(cx * x2);
    const float Eg = E * gs;
    s0 += Eg;
    s1 = fmaf(Eg, x2, s1);
    sg = fmaf(E * hs, fmaf(C1, x2, C0), sg);
  }
}

__global__ void __launch_bounds__(256) k_adj_small(const GeomDev *__restrict__ geoms,
                                                   const ModelDev *__restrict__ models,
                                                   const Item *__restrict__ items, int n_it,
                                                   ParamsDev p, const double *__restrict__ pix,
                                                   const int *__restrict__ st_ws,
                                                   double *__restrict__ sens) {
  __shared__ __attribute__((aligned(16))) float lam[kSmallMap][kSmallMap];   // [x][y]
  __shared__ float xsq[kSmallMap], ysq[kSmallMap];
  // per mass Gaussian: e2, de2/di, r, K_j / M_j, M_j
  __shared__ double jv[kSmallAdjMass][5];
  // per tracer: alpha, alphaq and d/di, nu0 / I0 and d/di, cos^2 i + b sin^2 i
  // and d/di, b, I0
  __shared__ double tv[kSmallAdjTracers][9];
  __shared__ double vals[kAdjTerms][3];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;   // uniform per block; k_grads writes NaN
    // block-uniform bounds in scalar registers, so the unrolled loops'
    // guards are scalar branches
    const int k0 = __builtin_amdgcn_readfirstlane(it.a & 0xffff);
    const int k1 = __builtin_amdgcn_readfirstlane(it.a >> 16);
    const int nx = __builtin_amdgcn_readfirstlane(g.n_ux);
    const int ny = __builtin_amdgcn_readfirstlane(g.n_uy);
    const int nu = __builtin_amdgcn_readfirstlane(g.n_u);
    const int J1 = __builtin_amdgcn_readfirstlane(g.J1), J = J1 - 1;
    __syncthreads();                  // the previous item's LDS reads are done
    const double *lamN = pix + md.pix_off + 2 * (int64_t)g.n_pix;
    for (int e = threadIdx.x; e < kSmallMap * kSmallMap; e += 256) {
      const int xx = e / kSmallMap, yy = e % kSmallMap;
      lam[xx][yy] = (yy < ny && xx < nx) ? (float)lamN[yy * nx + xx] : 0.f;
    }
    if (threadIdx.x < kSmallMap) {
      const int q = threadIdx.x;
      xsq[q] = q < nx ? (float)(g.xs[q] * g.xs[q]) : 0.f;
      ysq[q] = q < ny ? (float)(g.ys[q] * g.ys[q]) : 0.f;
    }
    const double inc = p.inc[it.m];
    const dual sn = {sin(inc), cos(inc)};
    const dual cs = {cos(inc), -sin(inc)};
    const dual si2 = sn * sn, ci2 = cs * cs;
    const double G = grav_const(), sp = g.s_pc;
    for (int j = threadIdx.x; j < J1; j += 256) {
      double *v = jv[j];
      if (j < J) {
        const double qo = g.mass_q[j], sj = g.mass_sigma[j];
        const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
        const dual qj = dsqrt(qo * qo - ci2) / sn;
        const dual e2 = 1.0 - qj * qj;
        v[0] = e2.v;
        v[1] = e2.d;
        v[2] = 0.5 / (sj * sj);
        v[3] = sqrt(2.0 / kPi) * G / (sp * sj);
        v[4] = p.mass_scale[it.m] * 2.0 * kPi * S0 * (sp * sj) * (sp * sj) * qo;
      } else {
        v[0] = 0.0;
        v[1] = 0.0;
        v[2] = 0.5 / (g.bh_sigma * g.bh_sigma);
        v[3] = sqrt(2.0 / kPi) * G / (sp * g.bh_sigma);
        v[4] = p.m_bh[it.m];
      }
    }
    if (threadIdx.x < k1 - k0) {
      // tracer k: deprojection (App. A) with its inclination derivative
      const int k = k0 + threadIdx.x;
      const double qok = g.lum_q[k], sk = g.lum_sigma[k];
      const double b = 1.0 / (1.0 - p.beta[md.lum_off + k]);
      const dual qk = dsqrt(qok * qok - ci2) / sn;
      const double alpha = 0.5 / (sk * sk);
      const dual alphaq = dconst(alpha) / (qk * qk);
      const dual nu1 = dconst(qok / (sqrt(2.0 * kPi) * sk)) / qk;   // nu0 / I0
      const dual pf = ci2 + b * si2;
      double *v = tv[threadIdx.x];
      v[0] = alpha;
      v[1] = alphaq.v;
      v[2] = alphaq.d;
      v[3] = nu1.v;
      v[4] = nu1.d;
      v[5] = pf.v;
      v[6] = pf.d;
      v[7] = b;
      v[8] = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
    }
    double *rows = chain_rows(sens, md, g);
    const int n_rows = (k1 - k0) * J1;
    const int per_win = max(1, kAdjTerms / nu);   // whole rows per window
    for (int r0 = 0; r0 < n_rows; r0 += per_win) {
      const int nr = min(per_win, n_rows - r0);
      const int n_terms = nr * nu;
      __syncthreads();                // staging done; earlier readers of vals done
      for (int base = 0; base < n_terms; base += 256) {
        const int tl = base + threadIdx.x;
        if (tl >= n_terms) break;
        const int rr = tl / nu, n = tl - rr * nu;
        const int row = r0 + rr, kk = row / J1, jj = row - kk * J1;
        const double *tk = tv[kk];
        const double *v = jv[jj];
        const double alpha = tk[0], b = tk[7];
        const dual alphaq = {tk[1], tk[2]}, nu1 = {tk[3], tk[4]}, pf = {tk[5], tk[6]};
        const double r = v[2], Mj = v[4];
        const double u = g.u[n], wq = g.w[n], u2 = u * u;
        const dual h = {fma(-v[0], u2, 1.0), -u2 * v[1]};
        const double c1 = alpha + r * u2;
        const double rhv = rcp64(h.v);
        const dual rh = {rhv, -rhv * rhv * h.d};
        const dual A = alphaq + (r * u2) * rh;
        const dual a = c1 * si2 + A * ci2;
        const double rav = rcp64(a.v);
        const dual gam = c1 * A * dual{rav, -rav * rav * a.d};
        const double rshv = rsq64(h.v);
        const dual rsh = {rshv, -0.5 * rshv * rhv * h.d};
        const dual bse = (v[3] * r * u2) * nu1;               // per unit I0 M
        const double rAv = rcp64(A.v);
        const dual gg = bse * dual{rAv, -rAv * rAv * A.d} * rh * rsh;
        const dual ww = 2.0 * bse * rsh;
        const dual P = pf * gg;
        const dual Q = si2 * (ww - (2.0 * c1 * b) * gg);
        const double fv = wq * kSqrtPi * rsq64(a.v);
        const dual f = {fv, -0.5 * fv * rav * a.d};
        const dual c0 = f * P, c1u = f * Q;                   // C = I0 M c
        const double amp = tk[8] * Mj;
        const float cx = (float)(-c1 * kLog2e), cy = (float)(-gam.v * kLog2e);
        const float C0 = (float)(amp * c0.v), C1 = (float)(amp * c1u.v);
        float s0, s1, sg;
        switch ((ny + 3) >> 2) {    // uniform
          case 1: small_sums<1>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 2: small_sums<2>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 3: small_sums<3>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 4: small_sums<4>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 5: small_sums<5>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 6: small_sums<6>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          case 7: small_sums<7>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
          default: small_sums<8>(cx, cy, C0, C1, lam, xsq, ysq, nx, s0, s1, sg); break;
        }
        const double S0 = s0, S1 = s1, Sg = sg;
        vals[tl][0] = amp * (S0 * c0.d + S1 * c1u.d) - Sg * gam.d;
        // dC0/db = f si2 g, dC1/db = -2 f si2 c1 g
        vals[tl][1] = amp * f.v * si2.v * gg.v * (S0 - 2.0 * c1 * S1);
        vals[tl][2] = S0 * c0.v + S1 * c1u.v;
      }
      __syncthreads();
      // (k, j) rows: one wave per row, lanes over the u-nodes in order, then
      // a butterfly
      for (int rr = wave; rr < nr; rr += 4) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int n = lane; n < nu; n += 64) {
          const double *v = vals[rr * nu + n];
          a0 += v[0];
          a1 += v[1];
          a2 += v[2];
        }
        a0 = wave_sum(a0);
        a1 = wave_sum(a1);
        a2 = wave_sum(a2);
        if (lane == 0) {
          double *o = rows + ((int64_t)k0 * J1 + r0 + rr) * 3;
          o[0] = a0;
          o[1] = a1;
          o[2] = a2;
        }
      }
    }
  }
}

// Final per-model gradients from the chain rows.  One 1024-thread block per
// model: each wave reduces one luminous Gaussian's row at a time over the
// mass Gaussians (lanes), then the waves reduce the mass derivatives over
// the luminous Gaussians; partial sums are combined in a fixed order.
__global__ void __launch_bounds__(1024) k_grads(const GeomDev *__restrict__ geoms,
                                               const ModelDev *__restrict__ models, int n,
                                               ParamsDev p, double *__restrict__ sens,
                                               const double *__restrict__ sbp,
                                               const int *__restrict__ st_ws, GradsDev out) {
  constexpr int kW = 16;   // waves per block
  __shared__ double part[kW];
  __shared__ double mpart[kW][64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const int K = g.K, J1 = g.J1, J = J1 - 1;
    const double *rows = chain_rows(sens, md, g);
    const bool ok = st_ws[m] == 0;
    const double nan = __builtin_nan("");
    const double sp = g.s_pc;
    const double ml = p.mass_scale[m];
    auto mass = [&](int j) {
      if (j == J) return p.m_bh[m];
      const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
      return ml * 2.0 * kPi * S0 * (sp * g.mass_sigma[j]) * (sp * g.mass_sigma[j]) * g.mass_q[j];
    };
    // d/di, d/dbeta_k, d/dI0_k
    double di = 0.0;
    for (int k = wave; k < K; k += kW) {
      double a = 0.0, db = 0.0, dI = 0.0;
      for (int j = lane; j < J1; j += 64) {
        const double *o = rows + ((int64_t)k * J1 + j) * 3;
        a += o[0];
        db += o[1];
        dI += mass(j) * o[2];
      }
      // surface-brightness path of I0_k: the tile partials, in tile order
      double sb = 0.0;
      const int n_tiles = sb_tiles(g.n_ux, g.n_uy);
      if (ok)
        for (int tl = lane; tl < n_tiles; tl += 64) sb += sbp[md.sbp_off + (int64_t)k * n_tiles + tl];
      a = wave_sum(a);
      db = wave_sum(db);
      dI = wave_sum(dI);
      sb = wave_sum(sb);
      di += a;
      if (lane == 0) {
        const double b = 1.0 / (1.0 - p.beta[md.lum_off + k]);
        if (out.beta) out.beta[md.lum_off + k] = ok ? db * b * b : nan;   // db/dbeta = b^2
        if (out.lum_I0) out.lum_I0[md.lum_off + k] = ok ? dI + sb : nan;
      }
    }
    // d/dM_j = sum_k I0_k H_kj; then the mass scale, Sigma0_j and the BH
    double dml = 0.0;
    for (int j0 = 0; j0 < J1; j0 += 64) {
      const int j = j0 + lane;
      double dM = 0.0;
      if (j < J1) {
        // loads of eight tracers are issued before their (ordered) adds
        for (int k0 = wave; k0 < K; k0 += 8 * kW) {
          double iv[8], hv[8];
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            const int k = k0 + kW * kk;
            iv[kk] = 0.0;
            hv[kk] = 0.0;
            if (k < K) {
              iv[kk] = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
              hv[kk] = rows[((int64_t)k * J1 + j) * 3 + 2];
            }
          }
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) dM += iv[kk] * hv[kk];
        }
      }
      __syncthreads();
      mpart[wave][lane] = dM;
      __syncthreads();
      if (wave == 0 && j < J1) {
        dM = 0.0;
        for (int w = 0; w < kW; ++w) dM += mpart[w][lane];
        if (j < J) {
          const double qo = g.mass_q[j], sj = g.mass_sigma[j];
          const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
          const double unit = 2.0 * kPi * (sp * sj) * (sp * sj) * qo;   // dM/d(ml S0)
          if (out.mass_S0) out.mass_S0[md.mass_off + j] = ok ? dM * ml * unit : nan;
          dml += dM * S0 * unit;
        } else {
          if (out.m_bh) out.m_bh[m] = ok ? dM : nan;
        }
      }
    }
    if (wave == 0) dml = wave_sum(dml);
    if (lane == 0) part[wave] = di;
    __syncthreads();
    if (threadIdx.x == 0) {
      double dsum = 0.0;
      for (int w = 0; w < kW; ++w) dsum += part[w];
      if (out.inc) out.inc[m] = ok ? dsum : nan;
      if (out.mass_scale) out.mass_scale[m] = ok ? dml : nan;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Goodness of fit, eq. (chi2_dyn): chi^2 = r^T P r with r_b = v_obs,b -
// sqrt(V_b) (eq. (Vrms)) and P the inverse covariance of the measured v_rms.
// One workgroup per model: r in LDS; s = P r by rows, one row per wave at a
// time with the lanes along the row and a fixed-order wave sum; chi^2 = r.s
// summed in a fixed order.  dV (optional) receives cot_m * d chi^2 / dV_b =
// -cot_m s_b / sqrt(V_b).  All FP64; NaN for a model whose status is not OK
// or with any V_b <= 0 (v_rms undefined).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_chi2(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models, int n,
                                              const KinDev *__restrict__ kin,
                                              const double *__restrict__ V,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ chi2,
                                              const double *__restrict__ cot,
                                              double *__restrict__ dV) {
  __shared__ double r[kChi2MaxBins];
  __shared__ double part[4];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double nan = __builtin_nan("");
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const int nb = geoms[md.geom].n_bins;
    const KinDev kd = kin[md.geom];
    const double *Vm = V + md.out_off;
    if (tid == 0) bad = (st_ws && st_ws[m] != 0) ? 1 : 0;
    __syncthreads();
    for (int b = tid; b < nb; b += 256) {
      const double v = Vm[b];
      if (!(v > 0.0)) bad = 1;       // every writer stores the same value
      r[b] = kd.vobs[b] - sqrt(v);
    }
    __syncthreads();
    const bool ok = bad == 0;
    const double scale = cot ? cot[m] : 1.0;
    double acc = 0.0;
    for (int b = wave; b < nb; b += 4) {
      const double *row = kd.prec + (int64_t)b * nb;
      double sb = 0.0;
      for (int c = lane; c < nb; c += 64) sb = fma(row[c], r[c], sb);
      sb = wave_sum(sb);
      acc = fma(r[b], sb, acc);
      if (dV && lane == 0) dV[md.out_off + b] = ok ? -scale * sb / sqrt(Vm[b]) : nan;
    }
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (tid == 0 && chi2) chi2[m] = ok ? ((part[0] + part[1]) + part[2]) + part[3] : nan;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One-dimensional MGE of radial profiles (Sect. 3.2, eq. integral_transfer
// and the Euler approximation after it).  A profile F(R) = sum_c a_c
// (R^2 + c_c^2)^(-p_c) is expanded as F(R) ~ sum_n A_n exp(-R^2/(2 sigma_n^2))
// with A_n = scale_n sum_k eta_k Re F(sigma_n chi_k), chi_k^2 = 2 beta_k, so
// F is needed at R^2 = 2 sigma_n^2 beta_k, where Re(R^2) > 0 and the
// principal logarithm of R^2 + c^2 is analytic.  FP64 throughout.
// ---------------------------------------------------------------------------
struct cplx {
  double re, im;
};
__device__ inline cplx c_log(cplx z) { return {log(hypot(z.re, z.im)), atan2(z.im, z.re)}; }
__device__ inline cplx c_exp(cplx z) {
  double sn, cs;
  sincos(z.im, &sn, &cs);
  const double e = exp(z.re);
  return {e * cs, e * sn};
}
__device__ inline cplx c_mul(cplx a, cplx b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ inline cplx c_div(cplx a, cplx b) {
  const double d = b.re * b.re + b.im * b.im;
  return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// Thread per (profile, Gaussian n); the terms k and components c are summed
// in a fixed order.
__global__ void __launch_bounds__(256) k_mge1d(int n_prof, int n_comp,
                                               const double *__restrict__ comp, MgeConst kc,
                                               double *__restrict__ amp) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n_prof * kc.n_sigma) return;
  const int prof = (int)(id / kc.n_sigma), n = (int)(id % kc.n_sigma);
  const double *cp = comp + (int64_t)prof * n_comp * 3;
  double f = 0.0;
  for (int k = 0; k < kc.n_terms; ++k) {
    const cplx r2 = {2.0 * kc.sigma2[n] * kc.beta_re, 2.0 * kc.sigma2[n] * kc.beta_im[k]};
    double fr = 0.0;   // Re F(R)
    for (int c = 0; c < n_comp; ++c) {
      const double a = cp[3 * c], cc = cp[3 * c + 1], p = cp[3 * c + 2];
      const cplx L = c_log({r2.re + cc * cc, r2.im});
      fr += a * c_exp({-p * L.re, -p * L.im}).re;
    }
    f += kc.eta[k] * fr;
  }
  amp[id] = kc.scale[n] * f;
}

// Thread per (profile, component): its three derivatives summed over the
// Gaussians n (weighted by the cotangent) and the terms k in a fixed order.
__global__ void __launch_bounds__(256) k_mge1d_vjp(int n_prof, int n_comp,
                                                   const double *__restrict__ comp, MgeConst kc,
                                                   const double *__restrict__ cot,
                                                   double *__restrict__ grad) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)n_prof * n_comp) return;
  const int prof = (int)(id / n_comp);
  const double *cp = comp + id * 3;
  const double a = cp[0], cc = cp[1], p = cp[2];
  double ga = 0.0, gc = 0.0, gp = 0.0;
  for (int n = 0; n < kc.n_sigma; ++n) {
    double da = 0.0, dc = 0.0, dp = 0.0;
    for (int k = 0; k < kc.n_terms; ++k) {
      const cplx w = {2.0 * kc.sigma2[n] * kc.beta_re + cc * cc, 2.0 * kc.sigma2[n] * kc.beta_im[k]};
      const cplx L = c_log(w);
      const cplx E = c_exp({-p * L.re, -p * L.im});          // w^-p
      const cplx Ew = c_div(E, w);                            // w^-(p+1)
      const double eta = kc.eta[k];
      da += eta * E.re;
      dc += eta * (-2.0 * p * cc * a) * Ew.re;
      dp += eta * (-a) * c_mul(L, E).re;
    }
    const double s = kc.scale[n] * cot[(int64_t)prof * kc.n_sigma + n];
    ga += s * da;
    gc += s * dc;
    gp += s * dp;
  }
  grad[id * 3] = ga;
  grad[id * 3 + 1] = gc;
  grad[id * 3 + 2] = gp;
}

// ---------------------------------------------------------------------------
// Spherically aligned model (eqs. J1, J2).  For tracer Gaussian k with
// constant beta the Jeans equations integrate along the characteristics
// r^(1-beta) sin(theta) = const:
//   P_k = nu v_r^2 = r^(-2 beta) int_r^inf r'^(2 beta) nu (d_z Phi) / cos(theta') dr',
//   d_theta P_k = r^(1 - 3 beta) cos(theta) I_D,
//   I_D = int_r^inf r'^(3 beta + 1) R' nu [G_theta + G (1/q^2 - 1) / sigma^2] dr',
//   nu v_phi^2 = (1 - beta) P + (1 - beta) sin(theta) r^(1 - 3 beta) I_D - nu R^2 G_phi,
// with G = (d_z Phi) / z, G_theta and G_phi u-integrals over the mass
// Gaussians (each term w K exp(-r_j u^2 (R^2 + z^2 / h)) times a polynomial
// in u).  The moments summed over the tracers, A_r = sum P_k, A_theta =
// sum (1 - beta_k) P_k and A_phi = sum nu v_phi^2_k, are tabulated on a polar
// grid and interpolated along the line of sight.
// ---------------------------------------------------------------------------
constexpr int kSphChunk = 1024;   // (j, u) terms staged in LDS at a time

// FP32 coefficients of the (j, u) terms of G, G_theta and G_phi, once per
// model: (-r_j u^2 log2e, -r_j u^2 / h log2e, gP, gT) and gF, zero-padded to
// a whole number of 64-term groups (a zero term adds exactly nothing).
// Item (m, block of 256 terms); thread = term.
__global__ void __launch_bounds__(256) k_sph_terms(const GeomDev *__restrict__ geoms,
                                                   const ModelDev *__restrict__ models,
                                                   const Item *__restrict__ items, int n_it,
                                                   const double *__restrict__ gauss,
                                                   const int *__restrict__ st_ws,
                                                   float4 *__restrict__ terms) {
  constexpr double kLog2e = 1.4426950408889634;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int nu_n = g.n_u, T = g.J1 * nu_n, Tp = sph_terms_padded(g.J1, nu_n);
    const int t = it.a * 256 + threadIdx.x;
    if (t >= Tp) continue;
    float4 *tc = terms + md.term_off;
    float *tf = (float *)(tc + Tp);
    if (t >= T || st_ws[it.m] != 0) {
      tc[t] = make_float4(0.f, 0.f, 0.f, 0.f);
      tf[t] = 0.f;
      continue;
    }
    const double *mt = gauss + md.gauss_off + 4 * g.K;
    const int j = t / nu_n, n = t % nu_n;
    const double rj = mt[j], e2 = mt[g.J1 + j], Kp = mt[2 * g.J1 + j];
    const double u = g.u[n], u2 = u * u, wK = g.w[n] * Kp;
    const double hh = 1.0 - e2 * u2, h15 = hh * sqrt(hh);
    tc[t] = make_float4((float)(-rj * u2 * kLog2e), (float)(-rj * u2 / hh * kLog2e),
                        (float)(wK * 2.0 * rj * u2 / h15),
                        (float)(wK * e2 * 4.0 * rj * rj * u2 * u2 * u2 / (h15 * hh)));
    tf[t] = (float)(wK * e2 * 2.0 * rj * u2 * u2 / h15);
  }
}

// ---------------------------------------------------------------------------
// Potential grid.  G and G_theta do not depend on the tracer, only on the
// point (R, z), and each (j, u) term factorises as gP 2^(cR R^2) 2^(cZ z^2)
// (resp. gT ...).  On a tensor grid of R and z values the two sums are
// therefore the matrix products A_G B^T and A_T B^T over the terms, with
// A[i, t] = g_t 2^(cR_t R_i^2) and B[l, t] = 2^(cZ_t z_l^2), which run on
// the matrix cores; the moment kernel then interpolates them at the
// characteristic nodes.  The grid is uniform in asinh(R / aR) and
// asinh(z / aZ): a quarter of the narrowest mass Gaussian (aR = min sigma_j
// / 4, aZ = min sigma_j q_j / 4) near the centre, logarithmic far out, up to
// r_max, the farthest node (sqrt(r_hi^2 + 50 max sigma_k^2)), at grid index
// kSphGridN - 3.  4-point Lagrange interpolation in both indices (G is even
// in R and in z, so the point below index 0 is index 1).
// ---------------------------------------------------------------------------
struct SphGrid {
  double aR, aZ, iR, iZ;   // scales and grid points per unit of asinh(R / aR), asinh(z / aZ)
};

__device__ inline SphGrid sph_grid_scales(const GeomDev &g, const double *tab) {
  const int K = g.K, J1 = g.J1;
  const double *mt = tab + 4 * K;         // per mass Gaussian: r_j = 1 / (2 sigma_j^2), e_j^2
  double s2 = 1e300, z2 = 1e300, sk2 = 0.0;
  for (int j = 0; j < J1; ++j) {
    const double sj2 = 0.5 / mt[j];
    s2 = fmin(s2, sj2);
    z2 = fmin(z2, sj2 * (1.0 - mt[J1 + j]));
  }
  for (int k = 0; k < K; ++k) sk2 = fmax(sk2, 0.5 / tab[k]);
  const double rhi = exp(g.sph_lnr0 + (kSphNR - 1) * g.sph_dlnr);
  const double rmax = sqrt(rhi * rhi + 50.0 * sk2);
  SphGrid s;
  s.aR = 0.25 * sqrt(s2);
  s.aZ = 0.25 * sqrt(z2);
  s.iR = (kSphGridN - 3) / asinh(rmax / s.aR);
  s.iZ = (kSphGridN - 3) / asinh(rmax / s.aZ);
  return s;
}

// Lagrange weights of the points -1, 0, 1, 2 at fraction f of [0, 1].
__device__ inline void lagrange4(double f, double w[4]) {
  const double fm = f - 1.0, fm2 = f - 2.0, fp = f + 1.0;
  w[0] = -f * fm * fm2 * (1.0 / 6.0);
  w[1] = fp * fm * fm2 * 0.5;
  w[2] = -fp * f * fm2 * 0.5;
  w[3] = fp * f * fm * (1.0 / 6.0);
}

// Values per grid point: the forward's G, G_theta (2 floats), or the
// adjoint's G, G_theta and their coefficient-weighted sums for the R'^2 and
// z'^2 derivatives (6 values, stored in 8 floats for two 16-byte reads).
template <int NC> struct SphGridVals { static constexpr int S = NC == 2 ? 2 : 8; };

// The NC sums at (R, z) from a model's grid sg ([N][N][S]).
template <int NC>
__device__ inline void sph_grid_at(const float *__restrict__ sg, const SphGrid &s, double R,
                                   double z, double (&v)[NC]) {
  constexpr int N = kSphGridN, S = SphGridVals<NC>::S;
  const double x = asinh(R / s.aR) * s.iR, y = asinh(z / s.aZ) * s.iZ;
  const int i0 = min(max((int)floor(x), 0), N - 3), l0 = min(max((int)floor(y), 0), N - 3);
  double wx[4], wy[4];
  lagrange4(x - i0, wx);
  lagrange4(y - l0, wy);
  int lb[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) lb[b] = abs(l0 - 1 + b);
#pragma unroll
  for (int c = 0; c < NC; ++c) v[c] = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const float *row = sg + (int64_t)abs(i0 - 1 + a) * N * S;
    double rv[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) rv[c] = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const float *pt = row + lb[b] * S;
      float f[NC];
      if constexpr (NC == 2) {
        const float2 q = *reinterpret_cast<const float2 *>(pt);
        f[0] = q.x; f[1] = q.y;
      } else {
        const float4 q0 = *reinterpret_cast<const float4 *>(pt);
        const float4 q1 = *reinterpret_cast<const float4 *>(pt + 4);
        f[0] = q0.x; f[1] = q0.y; f[2] = q0.z; f[3] = q0.w; f[4] = q1.x; f[5] = q1.y;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) rv[c] += wy[b] * (double)f[c];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] += wx[a] * rv[c];
  }
}

// Item (m, 64 x 64 tile, term slice): wave w computes the 32 x 32 block
// (w & 1, w >> 1) of the tile for all NC sums, over the slice's 64-term
// chunks (staged in LDS, shared by the four waves); lane l generates row
// l % 32 of the A operands (one exponential, NC products) and column l % 32
// of B for the term of its half-wave; FP32 matrix-core sums per chunk
// folded into FP64; the slice partial is stored in FP32 ([N][N][S] per
// slice).  The sums, per term (c.x, c.y the exponent coefficients of R'^2,
// z'^2 with log2 e, gP = c.z, gT = c.w): G = gP E, G_theta = gT E, and for
// the adjoint gP c.x E, gP c.y E, gT c.x E, gT c.y E.
template <int NC>
__global__ void __launch_bounds__(256) k_sph_grid(const GeomDev *__restrict__ geoms,
                                                  const ModelDev *__restrict__ models,
                                                  const Item *__restrict__ items, int n_it,
                                                  const double *__restrict__ gauss,
                                                  const float4 *__restrict__ terms,
                                                  const int *__restrict__ st_ws,
                                                  float *__restrict__ sgrid) {
  constexpr int N = kSphGridN, NT = kSphGridN / kSphGridTile, S = SphGridVals<NC>::S;
  __shared__ float4 cs[64];
  const int lane = threadIdx.x & 63, c32 = lane & 31, kh = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;         // uniform per block; the grid is not read
    const SphGrid sc = sph_grid_scales(g, gauss + md.gauss_off);
    const int r0 = kSphGridTile * (it.a / NT) + 32 * (wave & 1);
    const int z0 = kSphGridTile * (it.a % NT) + 32 * (wave >> 1);
    const double Rv = sc.aR * sinh((r0 + c32) / sc.iR), Zv = sc.aZ * sinh((z0 + c32) / sc.iZ);
    const float R2 = (float)(Rv * Rv), Z2 = (float)(Zv * Zv);
    const int chunks = sph_terms_padded(g.J1, g.n_u) / 64;
    const int per = (chunks + md.sgrid_slices - 1) / md.sgrid_slices;
    const int c0 = min(chunks, it.b * per), c1 = min(chunks, c0 + per);
    const float4 *tc = terms + md.term_off;
    double acc[NC][16];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[c][r] = 0.0;
    for (int ch = c0; ch < c1; ++ch) {
      __syncthreads();
      if (threadIdx.x < 64) cs[threadIdx.x] = tc[64 * ch + threadIdx.x];
      __syncthreads();
      v16f f[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) f[c] = zero;
#pragma unroll 4
      for (int s2 = 0; s2 < 32; ++s2) {
        const float4 c = cs[2 * s2 + kh];   // (cR log2e, cZ log2e, gP, gT)
        const float e = fast_exp2(c.x * R2);
        const float b = fast_exp2(c.y * Z2);
        const float eP = c.z * e, eT = c.w * e;
        f[0] = __builtin_amdgcn_mfma_f32_32x32x2f32(eP, b, f[0], 0, 0, 0);
        f[1] = __builtin_amdgcn_mfma_f32_32x32x2f32(eT, b, f[1], 0, 0, 0);
        if constexpr (NC == 6) {
          f[2] = __builtin_amdgcn_mfma_f32_32x32x2f32(eP * c.x, b, f[2], 0, 0, 0);
          f[3] = __builtin_amdgcn_mfma_f32_32x32x2f32(eP * c.y, b, f[3], 0, 0, 0);
          f[4] = __builtin_amdgcn_mfma_f32_32x32x2f32(eT * c.x, b, f[4], 0, 0, 0);
          f[5] = __builtin_amdgcn_mfma_f32_32x32x2f32(eT * c.y, b, f[5], 0, 0, 0);
        }
      }
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[c][r] += (double)f[c][r];
    }
    float *og = sgrid + (NC == 2 ? md.sgrid_off : md.sgrid6_off) + (int64_t)it.b * N * N * S;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      float *o = og + ((int64_t)(r0 + mfma_row(r, lane)) * N + z0 + c32) * S;
      if constexpr (NC == 2) {
        *reinterpret_cast<float2 *>(o) = make_float2((float)acc[0][r], (float)acc[1][r]);
      } else {
        *reinterpret_cast<float4 *>(o) = make_float4((float)acc[0][r], (float)acc[1][r],
                                                     (float)acc[2][r], (float)acc[3][r]);
        *reinterpret_cast<float4 *>(o + 4) =
            make_float4((float)acc[4][r], (float)acc[5][r], 0.f, 0.f);
      }
    }
  }
}

// Item (m, block of 1024 grid floats): the slice partials summed in slice
// order (FP64) into slice 0; len = N^2 S floats per slice, off selects the
// forward's or the adjoint's grid.
__global__ void __launch_bounds__(256) k_sph_grid_reduce(const ModelDev *__restrict__ models,
                                                         const Item *__restrict__ items, int n_it,
                                                         const int *__restrict__ st_ws,
                                                         float *__restrict__ sgrid, int adjoint) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;
    const ModelDev md = models[it.m];
    const int64_t len = (int64_t)kSphGridN * kSphGridN * (adjoint ? 8 : 2);
    float *base = sgrid + (adjoint ? md.sgrid6_off : md.sgrid_off);
    const int64_t e1 = min(len, (int64_t)(it.a + 1) * 1024);
    for (int64_t e = (int64_t)it.a * 1024 + threadIdx.x; e < e1; e += 256) {
      double v = 0.0;
      for (int sl = 0; sl < md.sgrid_slices; ++sl) v += (double)base[sl * len + e];
      base[e] = (float)v;
    }
  }
}

// Item (m, group of four table points): wave w computes point 4 q + w (one
// table point per wave, so no block-wide reductions), taking the tracers two
// per round (each coefficient read from LDS feeds both); lane l is node l of
// the composite Gauss-Legendre rule in tau = ln(r'/r) on [0, ln(r_max / r)],
// r_max^2 = r^2 + 50 sigma_k^2.  Without the grid the per-model term
// coefficients go through LDS in chunks shared by the four waves; each group
// of 64 terms is summed in FP32 (fully unrolled, the coefficient reads are
// wave-wide broadcasts) and folded into FP64; everything else is FP64; all
// sums run in a fixed order.
template <bool kGrid>
__global__ void __launch_bounds__(256) k_sph_moments(const GeomDev *__restrict__ geoms,
                                                     const ModelDev *__restrict__ models,
                                                     const Item *__restrict__ items, int n_it,
                                                     const double *__restrict__ gauss,
                                                     const float4 *__restrict__ terms,
                                                     const int *__restrict__ st_ws,
                                                     const float *__restrict__ sgrid,
                                                     double *__restrict__ table) {
  __shared__ float4 tc[kSphChunk];   // (-c log2e, -d log2e, gP, gT)
  __shared__ float tf[kSphChunk];    // gF
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int cell = 4 * it.a + wave;
    double *out = table + md.sph_off + (int64_t)cell * 3;
    if (st_ws[it.m] != 0) {                 // uniform per block
      if (lane < 3) out[lane] = 0.0;
      continue;
    }
    const int K = g.K, Tp = sph_terms_padded(g.J1, g.n_u);
    const float4 *gtc = terms + md.term_off;
    const float *gtf = (const float *)(gtc + Tp);
    const double *tab = gauss + md.gauss_off;
    const int ir = cell / kSphNT, ith = cell % kSphNT;
    const double lnr = g.sph_lnr0 + ir * g.sph_dlnr, r = exp(lnr);
    const double th = ith * (0.5 * kPi / (kSphNT - 1));
    const double sth = sin(th), cth = cos(th);
    const double Rp0 = r * sth, zp0 = r * cth;
    const float R20 = (float)(Rp0 * Rp0), Z20 = (float)(zp0 * zp0);
    const int seg = lane >> 3, gi = lane & 7;
    // the rule's node and weight of this lane, read from global memory (a
    // lane-dependent index into the by-value descriptor would go to scratch)
    const double glx = geoms[md.geom].gl8_x[gi], glw = geoms[md.geom].gl8_w[gi];
    // G and G_theta at the nodes: from the model's potential grid, or summed
    // over the terms here
    const float *sg = kGrid ? sgrid + md.sgrid_off : nullptr;
    SphGrid sc = {1.0, 1.0, 1.0, 1.0};
    if (kGrid) sc = sph_grid_scales(g, tab);
    double Ar = 0.0, At = 0.0, Ap = 0.0;   // the point's moments (lane 0)
    double accF = 0.0;                      // this lane's share of G_phi
    constexpr int kTr = 2;                  // tracers per round
    const int rounds = (K + kTr - 1) / kTr; // the same in every wave
    for (int q = 0; q < rounds; ++q) {
      double alpha[kTr], alphaq[kTr], beta[kTr], wn[kTr], nuv[kTr], rp[kTr], Rp[kTr], Zp[kTr];
      double rbe[kTr], rpb[kTr];             // r^beta, r'^beta (the powers are their products)
      float R2[kTr], Z2[kTr];
      bool on[kTr];
#pragma unroll
      for (int u = 0; u < kTr; ++u) {
        const int k = kTr * q + u;
        on[u] = k < K;                      // uniform
        alpha[u] = 1.0; alphaq[u] = 1.0; beta[u] = 0.0; wn[u] = 0.0; nuv[u] = 0.0;
        rp[u] = r; rbe[u] = 1.0; rpb[u] = 1.0; Rp[u] = 0.0; Zp[u] = 0.0; R2[u] = 0.f; Z2[u] = 0.f;
        if (on[u]) {
          alpha[u] = tab[k];
          alphaq[u] = tab[K + k];
          beta[u] = 1.0 - 1.0 / tab[3 * K + k];
          const double tmax = 0.5 * log1p(50.0 * (0.5 / alpha[u]) / (r * r));
          const double hs = tmax / kSphSeg;
          const double tau = (seg + 0.5 + 0.5 * glx) * hs;
          rp[u] = exp(lnr + tau);
          // (r'/r)^beta; sin theta' = sin theta (r / r')^(1 - beta)
          const double rbt = exp(beta[u] * tau);
          rbe[u] = exp(beta[u] * lnr);
          rpb[u] = rbe[u] * rbt;
          const double st = fmin(1.0, sth * (r / rp[u]) * rbt);
          const double ct = sqrt(fmax(0.0, 1.0 - st * st));
          Rp[u] = rp[u] * st;
          const double zp = rp[u] * ct;
          Zp[u] = zp;
          R2[u] = (float)(Rp[u] * Rp[u]);
          Z2[u] = (float)(zp * zp);
          wn[u] = 0.5 * glw * hs * rp[u];
          nuv[u] = tab[2 * K + k] * exp(-(alpha[u] * Rp[u] * Rp[u] + alphaq[u] * zp * zp));
        }
      }
      double accG[kTr], accT[kTr];
#pragma unroll
      for (int u = 0; u < kTr; ++u) { accG[u] = 0.0; accT[u] = 0.0; }
      if (kGrid) {
#pragma unroll
        for (int u = 0; u < kTr; ++u)
          if (on[u]) {
            double v[2];
            sph_grid_at<2>(sg, sc, Rp[u], Zp[u], v);
            accG[u] = v[0];
            accT[u] = v[1];
          }
      }
      // the terms: the node sums (without a grid) and, in the first round,
      // G_phi at the table point
      if (!kGrid || q == 0)
      for (int c0 = 0; c0 < Tp; c0 += kSphChunk) {
        const int cn = min(kSphChunk, Tp - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += 256) {
          tc[t] = gtc[c0 + t];
          tf[t] = gtf[c0 + t];
        }
        __syncthreads();
        if (!kGrid) {
          for (int t0 = 0; t0 < cn; t0 += 64) {
            float sg0 = 0.f, sd0 = 0.f, sg1 = 0.f, sd1 = 0.f;
#pragma unroll
            for (int t = 0; t < 64; ++t) {
              const float4 c = tc[t0 + t];
              const float e0 = fast_exp2(fmaf(c.x, R2[0], c.y * Z2[0]));
              const float e1 = fast_exp2(fmaf(c.x, R2[1], c.y * Z2[1]));
              sg0 = fmaf(c.z, e0, sg0);
              sd0 = fmaf(c.w, e0, sd0);
              sg1 = fmaf(c.z, e1, sg1);
              sd1 = fmaf(c.w, e1, sd1);
            }
            accG[0] += (double)sg0;
            accT[0] += (double)sd0;
            accG[1] += (double)sg1;
            accT[1] += (double)sd1;
          }
        }
        if (q == 0) {
          for (int t = lane; t < cn; t += 64) {
            const float4 c = tc[t];
            accF += (double)(tf[t] * fast_exp2(fmaf(c.x, R20, c.y * Z20)));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kTr; ++u) {
        if (!on[u]) continue;
        const double sk2 = 0.5 / alpha[u], qk2 = alpha[u] / alphaq[u];
        // r'^(2 beta + 1) and r'^(3 beta + 1)
        const double p2 = rp[u] * rpb[u] * rpb[u], p3 = p2 * rpb[u];
        double fP = wn[u] * p2 * nuv[u] * accG[u];
        double fD = wn[u] * p3 * Rp[u] * nuv[u] * (accT[u] + accG[u] * (1.0 / qk2 - 1.0) / sk2);
        fP = wave_sum(fP);
        fD = wave_sum(fD);
        // r^(-2 beta) and r^(1 - 3 beta)
        const double rb2 = rbe[u] * rbe[u];
        const double P = fP / rb2;
        Ar += P;
        At += (1.0 - beta[u]) * P;
        Ap += (1.0 - beta[u]) * P + (1.0 - beta[u]) * sth * (r / (rb2 * rbe[u])) * fD;
      }
    }
    // G_phi and the tracer density at the point, lane sums in a fixed order
    const double Gphi = wave_sum(accF);
    double nus = 0.0;
    for (int k = lane; k < K; k += 64)
      nus += tab[2 * K + k] * exp(-(tab[k] * Rp0 * Rp0 + tab[K + k] * zp0 * zp0));
    nus = wave_sum(nus);
    if (lane == 0) {
      out[0] = Ar;
      out[1] = At;
      out[2] = Ap - nus * Rp0 * Rp0 * Gphi;
    }
  }
}

// ---------------------------------------------------------------------------
// Adjoint of the spherically aligned model.  With lambda_N per unique pixel
// (bin adjoint) the chain runs back through the line-of-sight rule (to the
// table and, at fixed table, to i and the node scale a), through the
// characteristic integrals (to beta_k, alphaq_k, nu0_k per table cell and
// tracer, and to the (j, u) term coefficients by term-major sums over all
// (cell, tracer, node) points), through the term coefficients (to e_j^2 and
// K_j), and through the set-up to the parameters.  FP64 except the FP32
// exponentials and their sums over 64 or 256 points, as in the forward.
// ---------------------------------------------------------------------------

// Radial interpolation of the moment table: Catmull-Rom (cubic convolution,
// a = -1/2) in ln r over the radii xi - 1 .. xi + 2 around the cell [xi,
// xi + 1] holding fraction fx; at the ends of the range the missing radius is
// the linear extrapolation of the two nearest, folded into the weights.
// ew: weights of radii xi - 1 + a (0 where out of range); dew: d ew / d fx.
__device__ inline void sph_radial_weights(int xi, double fx, double *ew, double *dew) {
  const double f2 = fx * fx, f3 = f2 * fx;
  ew[0] = 0.5 * (-f3 + 2.0 * f2 - fx);
  ew[1] = 0.5 * (3.0 * f3 - 5.0 * f2 + 2.0);
  ew[2] = 0.5 * (-3.0 * f3 + 4.0 * f2 + fx);
  ew[3] = 0.5 * (f3 - f2);
  dew[0] = 0.5 * (-3.0 * f2 + 4.0 * fx - 1.0);
  dew[1] = 0.5 * (9.0 * f2 - 10.0 * fx);
  dew[2] = 0.5 * (-9.0 * f2 + 8.0 * fx + 1.0);
  dew[3] = 0.5 * (3.0 * f2 - 2.0 * fx);
  if (xi == 0) {                  // radius -1 = 2 r_0 - r_1
    ew[1] += 2.0 * ew[0];
    ew[2] -= ew[0];
    ew[0] = 0.0;
    dew[1] += 2.0 * dew[0];
    dew[2] -= dew[0];
    dew[0] = 0.0;
  }
  if (xi + 2 > kSphNR - 1) {      // radius NR = 2 r_(NR-1) - r_(NR-2)
    ew[2] += 2.0 * ew[3];
    ew[1] -= ew[3];
    ew[3] = 0.0;
    dew[2] += 2.0 * dew[3];
    dew[1] -= dew[3];
    dew[3] = 0.0;
  }
}

// Angular weights, Catmull-Rom in theta over the angles yi - 1 .. yi + 2;
// the moments are even about theta = 0 and theta = pi/2, so a missing angle
// is the mirror image of the one inside, folded into the weights.
__device__ inline void sph_angular_weights(int yi, double fy, double *ew, double *dew) {
  const double f2 = fy * fy, f3 = f2 * fy;
  ew[0] = 0.5 * (-f3 + 2.0 * f2 - fy);
  ew[1] = 0.5 * (3.0 * f3 - 5.0 * f2 + 2.0);
  ew[2] = 0.5 * (-3.0 * f3 + 4.0 * f2 + fy);
  ew[3] = 0.5 * (f3 - f2);
  dew[0] = 0.5 * (-3.0 * f2 + 4.0 * fy - 1.0);
  dew[1] = 0.5 * (9.0 * f2 - 10.0 * fy);
  dew[2] = 0.5 * (-9.0 * f2 + 8.0 * fy + 1.0);
  dew[3] = 0.5 * (3.0 * f2 - 2.0 * fy);
  if (yi == 0) {                  // angle -1 mirrors angle 1 (= yi + 1)
    ew[2] += ew[0];
    ew[0] = 0.0;
    dew[2] += dew[0];
    dew[0] = 0.0;
  }
  if (yi + 2 > kSphNT - 1) {      // angle NT mirrors angle NT - 2 (= yi)
    ew[1] += ew[3];
    ew[3] = 0.0;
    dew[1] += dew[3];
    dew[3] = 0.0;
  }
}

// Node of tracer k's characteristic through table point (r, theta): the same
// FP64 operations as the forward moment kernel.
struct SphNode {
  double rp, st, ct, Rp, zp, wn, en, tau, rbt;   // rbt = (r'/r)^beta
  bool clamped;
};
__device__ inline SphNode sph_node(double r, double lnr, double sth, double alpha, double alphaq,
                                   double beta, int seg, double glx, double glw) {
  SphNode o;
  const double tmax = 0.5 * log1p(50.0 * (0.5 / alpha) / (r * r));
  const double hs = tmax / kSphSeg;
  o.tau = (seg + 0.5 + 0.5 * glx) * hs;
  o.rp = exp(lnr + o.tau);
  o.rbt = exp(beta * o.tau);
  const double sraw = sth * (r / o.rp) * o.rbt;   // sin theta (r / r')^(1 - beta)
  o.clamped = !(sraw < 1.0);
  o.st = fmin(1.0, sraw);
  o.ct = sqrt(fmax(0.0, 1.0 - o.st * o.st));
  o.Rp = o.rp * o.st;
  o.zp = o.rp * o.ct;
  o.wn = 0.5 * glw * hs * o.rp;
  o.en = exp(-(alpha * o.Rp * o.Rp + alphaq * o.zp * o.zp));
  return o;
}

__device__ inline void sph_cell(const GeomDev &g, int cell, double &r, double &sth, double &cth) {
  const int ir = cell / kSphNT, ith = cell % kSphNT;
  r = exp(g.sph_lnr0 + ir * g.sph_dlnr);
  const double th = ith * (0.5 * kPi / (kSphNT - 1));
  sth = sin(th);
  cth = cos(th);
}

__device__ inline SphAdj sph_adj_of(double *sens, const ModelDev &md, const GeomDev &g) {
  return sph_adj_layout(sens + md.sens_off, g.K, g.n_pix, sph_terms_padded(g.J1, g.n_u),
                        md.n_sens_parts);
}

// Start of the line-of-sight adjoint, block per model: clears the table
// cotangent and fixes its fixed-point scale.  Every contribution to the
// cotangent is lambda_N w_z (n.e_f)^2 times interpolation weights, so the
// sum of their magnitudes over all pixels, nodes and cells is at most
// sum_p |lambda_N| x sum_nodes w_z (the node rule integrates a cosh(w) over
// [-W, W]: 2 a sinh W = 24 max sigma_k, taken as 25) x sum |radial weights|
// x sum |angular weights| (each below 2; sum_f (n.e_f)^2 = 1).  The scale is
// the power of two that maps that bound below 2^61 (at most 2^1000, for
// tiny bounds), so the 64-bit integer sums cannot overflow and do not depend
// on the order of the additions.
// A non-finite bound stores NaN, which k_sph_dtab_fix turns into a NaN
// cotangent.
constexpr int kZeroThreads = 1024;
__global__ void __launch_bounds__(kZeroThreads) k_sph_zero(const GeomDev *__restrict__ geoms,
                                                           const ModelDev *__restrict__ models,
                                                           int n, const double *__restrict__ gauss,
                                                           const int *__restrict__ st_ws,
                                                           const double *__restrict__ pix,
                                                           double *__restrict__ sens) {
  constexpr int kWaves = kZeroThreads / 64;
  __shared__ double sh[kWaves];
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const SphAdj adj = sph_adj_of(sens, md, g);
    unsigned long long *d = reinterpret_cast<unsigned long long *>(adj.dtab);
    for (int i = threadIdx.x; i < 3 * kSphCells; i += kZeroThreads) d[i] = 0ull;
    if (st_ws[m] != 0) continue;   // uniform per block
    const double *lam = pix + md.pix_off + 2 * (int64_t)g.n_pix;
    // eight loads in flight per thread; partial sums added in a fixed order,
    // then the lanes by butterflies and the waves in order
    double sp[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q0 = 0; q0 < g.n_pix; q0 += 8 * kZeroThreads) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = q0 + u * kZeroThreads + threadIdx.x;
        if (q < g.n_pix) sp[u] += fabs(lam[q]);
      }
    }
    double s = ((sp[0] + sp[1]) + (sp[2] + sp[3])) + ((sp[4] + sp[5]) + (sp[6] + sp[7]));
    s = wave_sum(s);
    __syncthreads();                 // the previous model's reads of sh
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      s = 0.0;
      for (int w = 0; w < kWaves; ++w) s += sh[w];
      const double *tab = gauss + md.gauss_off;
      double smax = 0.0;
      for (int k = 0; k < g.K; ++k) smax = fmax(smax, sqrt(0.5 / tab[k]));
      const double bound = s * 25.0 * smax * 4.0;
      double scale = __builtin_nan("");
      if (bound == 0.0) scale = 1.0;
      else if (bound < __builtin_inf()) scale = ldexp(1.0, min(1000, 60 - ilogb(bound)));
      adj.dscale[0] = scale;
    }
  }
}

// End of the line-of-sight adjoint, block per model: the fixed-point table
// cotangent back to FP64 in place.
__global__ void __launch_bounds__(256) k_sph_dtab_fix(const GeomDev *__restrict__ geoms,
                                                      const ModelDev *__restrict__ models, int n,
                                                      const int *__restrict__ st_ws,
                                                      double *__restrict__ sens) {
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    if (st_ws[m] != 0) continue;   // uniform per block
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const SphAdj adj = sph_adj_of(sens, md, g);
    const double scale = adj.dscale[0];
    long long *d = reinterpret_cast<long long *>(adj.dtab);
    for (int i = threadIdx.x; i < 3 * kSphCells; i += 256) {
      const long long v = d[i];
      adj.dtab[i] = scale == scale ? (double)v / scale : scale;
    }
  }
}

// Line-of-sight kernels: four lanes per pixel, each taking a quarter of the
// line-of-sight nodes.
constexpr int kLosLanes = 4;                       // lanes per pixel
constexpr int kLosNodes = kSphNodes / kLosLanes;   // nodes per lane

// Line-of-sight adjoint.  Item (m, 64-pixel block), one workgroup each, the
// lanes as in k_sph_num.  The table cotangent receives lambda_N w_z
// (n.e_f)^2 times the interpolation weights, each rounded to a 64-bit
// fixed-point integer at the model's scale (k_sph_zero), accumulated in a
// block-private LDS copy of the table (integer LDS atomics) and added to the
// model's table once per block (integer global atomics, non-zero entries
// only): integer sums, so the result does not depend on the order of the
// additions.  The derivatives of the node's integrand at fixed table with
// respect to i (line of sight and node position) and to the node scale a
// are summed per block in a fixed order (butterflies over each wave, then
// the waves in order).
__global__ void __launch_bounds__(256) k_sph_num_adj(const GeomDev *__restrict__ geoms,
                                                     const ModelDev *__restrict__ models,
                                                     const Item *__restrict__ items, int n_it,
                                                     const double *__restrict__ gauss,
                                                     const int *__restrict__ st_ws,
                                                     const double *__restrict__ table,
                                                     const double *__restrict__ pix,
                                                     double *__restrict__ sens) {
  __shared__ unsigned long long ldt[3 * kSphCells];
  __shared__ double wred[4][2];
  const int pl = threadIdx.x / kLosLanes, h = threadIdx.x % kLosLanes;
  for (int ii = blockIdx.x; ii < n_it; ii += gridDim.x) {
    const Item it = items[ii];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;              // uniform per block
    const SphAdj adj = sph_adj_of(sens, md, g);
    const double scale = adj.dscale[0];
    const bool fixed = scale == scale;           // NaN: non-finite cotangent
    for (int i = threadIdx.x; i < 3 * kSphCells; i += 256) ldt[i] = 0ull;
    __syncthreads();
    const int q = it.a * 64 + pl;
    const bool on = q < g.n_pix;
    const int K = g.K;
    const double *tab = gauss + md.gauss_off;
    const double *mt = tab + 4 * K;
    const double si = sqrt(mt[3 * g.J1]), ci = sqrt(mt[3 * g.J1 + 1]);
    double smin = 1e300, smax = 0.0;
    for (int k = 0; k < K; ++k) {
      const double sk = sqrt(0.5 / tab[k]), qk = sqrt(tab[k] / tab[K + k]);
      smin = fmin(smin, sk * qk);
      smax = fmax(smax, sk);
    }
    const double a = 0.25 * smin, cW = 12.0 * smax, W = asinh(cW / a);
    const double Wa = -(cW / (a * a)) / sqrt(1.0 + (cW / a) * (cW / a));   // dW/da
    const double x = on ? g.xs[q % g.n_ux] : 0.0, y = on ? g.ys[q / g.n_ux] : 0.0;
    const double lamN = on ? pix[md.pix_off + 2 * (int64_t)g.n_pix + q] : 0.0;
    const double *T = table + md.sph_off;
    const double dth = 0.5 * kPi / (kSphNT - 1);
    const double hw = 2.0 * W / kSphSeg;
    const double *glx = geoms[md.geom].gl8_x, *glw = geoms[md.geom].gl8_w;
    double acc_i = 0.0, acc_a = 0.0;
    for (int nd = h * kLosNodes; on && nd < (h + 1) * kLosNodes; ++nd) {
      const int seg = nd >> 3, gi = nd & 7;
      const double om = -1.0 + (seg + 0.5 + 0.5 * glx[gi]) / 4.0;   // w = W om
      const double w = -W + (seg + 0.5 + 0.5 * glx[gi]) * hw;
      // sinh w, cosh w from one exponential (|w| > 0.004 W at every node)
      const double ex = exp(w), iex = 1.0 / ex;
      const double shw = 0.5 * (ex - iex), chw = 0.5 * (ex + iex);
      const double zp = a * shw, wz = 0.5 * glw[gi] * hw * a * chw;
      const double X = x, Y = zp * si - y * ci, Z = y * si + zp * ci;
      const double R = sqrt(X * X + Y * Y), r = sqrt(R * R + Z * Z);
      const double ct = Z / r, st = R / r;
      const double sp = R > 0.0 ? Y / R : 0.0, cp = R > 0.0 ? X / R : 0.0;
      const double xf = (log(r) - g.sph_lnr0) / g.sph_dlnr;
      if (xf > kSphNR - 1) continue;
      const double yf = acos(fmin(1.0, fabs(ct))) / dth;
      const int xi = (int)fmin(fmax(floor(xf), 0.0), (double)(kSphNR - 2));
      const int yi = (int)fmin(fmax(floor(yf), 0.0), (double)(kSphNT - 2));
      const double fx = fmin(fmax(xf - xi, 0.0), 1.0), fy = fmin(fmax(yf - yi, 0.0), 1.0);
      double ew[4], dew[4], tw[4], dtw[4];
      sph_radial_weights(xi, fx, ew, dew);
      sph_angular_weights(yi, fy, tw, dtw);
      const double ner = si * st * sp + ci * ct;
      const double net = si * ct * sp - ci * st;
      const double nep = si * cp;
      const double nf[3] = {ner, net, nep};
      // table cotangent
      double A[3] = {0.0, 0.0, 0.0}, AL[3] = {0.0, 0.0, 0.0}, AT[3] = {0.0, 0.0, 0.0};
      const bool xin = xf >= 0.0;          // below the first radius the table is constant
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (ew[a] == 0.0 && dew[a] == 0.0) continue;   // out of range (folded)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (tw[b] == 0.0 && dtw[b] == 0.0) continue;
          const int64_t i0 = ((int64_t)(xi - 1 + a) * kSphNT + (yi - 1 + b)) * 3;
          const double *c = T + i0;
          unsigned long long *d = ldt + i0;
#pragma unroll
          for (int f = 0; f < 3; ++f) {
            const double cf = lamN * wz * nf[f] * nf[f] * ew[a] * tw[b];
            if (cf != 0.0 && fixed)
              atomicAdd(d + f, (unsigned long long)__double2ll_rn(cf * scale));
            A[f] += ew[a] * tw[b] * c[f];
            if (xin) AL[f] += dew[a] * tw[b] * c[f];
            AT[f] += ew[a] * dtw[b] * c[f];
          }
        }
      }
      // the weight derivatives are per unit of the table's index steps
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        AL[f] /= g.sph_dlnr;
        AT[f] /= dth;
      }
      // derivatives of ln r and theta = atan2(R, |Z|) with respect to Y and Z
      const double r2 = r * r, sz = Z < 0.0 ? -1.0 : 1.0;
      const double lY = Y / r2, lZ = Z / r2;
      const double tY = R > 0.0 ? fabs(Z) * (Y / R) / r2 : 0.0, tZ = -R * sz / r2;
      // line-of-sight components and their derivatives (Y, Z; explicit i)
      double nY[3] = {0.0, 0.0, 0.0}, nZ[3] = {0.0, 0.0, 0.0}, ni[3] = {0.0, 0.0, 0.0};
      nY[0] = (si - ner * Y / r) / r;
      nZ[0] = (ci - ner * Z / r) / r;
      ni[0] = (ci * Y - si * Z) / r;
      if (R > 0.0) {
        const double rR = r * R;
        nY[1] = ((si * Z - 2.0 * ci * Y) - net * (Y / r * R + r * Y / R)) / rR;
        nZ[1] = (si * Y - net * (Z / r) * R) / rR;
        ni[1] = (ci * Z * Y + si * R * R) / rR;
        nY[2] = -si * X * Y / (R * R * R);
        ni[2] = ci * X / R;
      }
      double F = 0.0, FY = 0.0, FZ = 0.0, Fi = 0.0;
  #pragma unroll
      for (int f = 0; f < 3; ++f) {
        const double dAY = AL[f] * lY + AT[f] * tY, dAZ = AL[f] * lZ + AT[f] * tZ;
        F += nf[f] * nf[f] * A[f];
        FY += 2.0 * nf[f] * nY[f] * A[f] + nf[f] * nf[f] * dAY;
        FZ += 2.0 * nf[f] * nZ[f] * A[f] + nf[f] * nf[f] * dAZ;
        Fi += 2.0 * nf[f] * ni[f] * A[f];
      }
      const double Yi = zp * ci + y * si, Zi = y * ci - zp * si;
      acc_i += lamN * wz * (Fi + FY * Yi + FZ * Zi);
      const double dzp = shw + a * chw * om * Wa;
      const double dwz = 0.5 * glw[gi] * (2.0 / kSphSeg) *
                         (Wa * a * chw + W * chw + W * a * shw * om * Wa);
      acc_a += lamN * (dwz * F + wz * (FY * si + FZ * ci) * dzp);
    }
    // fixed-order sums: each wave's 64 lanes by a butterfly, then the waves
    acc_i = wave_sum(acc_i);
    acc_a = wave_sum(acc_a);
    if ((threadIdx.x & 63) == 0) {
      wred[threadIdx.x >> 6][0] = acc_i;
      wred[threadIdx.x >> 6][1] = acc_a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      adj.losp[2 * it.a] = ((wred[0][0] + wred[1][0]) + wred[2][0]) + wred[3][0];
      adj.losp[2 * it.a + 1] = ((wred[0][1] + wred[1][1]) + wred[2][1]) + wred[3][1];
    }
    unsigned long long *dt = reinterpret_cast<unsigned long long *>(adj.dtab);
    for (int i = threadIdx.x; i < 3 * kSphCells; i += 256) {
      const unsigned long long v = ldt[i];
      if (v != 0ull) atomicAdd(dt + i, v);
    }
    __syncthreads();
  }
}

// Forward pass of the adjoint: the moment table (as k_sph_moments) with the
// node sums its adjoint needs.  Item (m, table cell), the forward's layout:
// wave w takes tracers 8 q + w and 8 q + 4 + w, lane = node.  Per node the
// term sums G, G_theta and their derivatives in R'^2 and z'^2; per (cell,
// tracer) the node sums of the characteristic integrals (fP, fD) and of
// their derivatives with respect to beta_k (bP, bD), alphaq_k (qP, qD) and
// nu0_k (eP, eD) go to SphAdj::jac, none of which depends on the table
// cotangent, and the cell's G_phi to SphAdj::gphi; k_sph_rows combines
// them with the cotangent once the line-of-sight adjoint has produced it.
template <bool kGrid>
__global__ void __launch_bounds__(256) k_sph_moments_jac(const GeomDev *__restrict__ geoms,
                                                         const ModelDev *__restrict__ models,
                                                         const Item *__restrict__ items, int n_it,
                                                         const double *__restrict__ gauss,
                                                         const float4 *__restrict__ terms,
                                                         const int *__restrict__ st_ws,
                                                         const float *__restrict__ sgrid6,
                                                         double *__restrict__ table,
                                                         double *__restrict__ sens) {
  __shared__ float4 tc[kSphChunk];
  __shared__ float4 tx[kSphChunk];   // (gP c_x, gP c_y, gT c_x, gT c_y)
  __shared__ float tf[kSphChunk];
  __shared__ double sh[256];
  __shared__ double wred[3][4];
  constexpr double kLn2 = 0.6931471805599453;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    double *out = table + md.sph_off + (int64_t)it.a * 3;
    if (st_ws[it.m] != 0) {                  // uniform per block
      if (threadIdx.x < 3) out[threadIdx.x] = 0.0;
      continue;
    }
    const SphAdj adj = sph_adj_of(sens, md, g);
    // the six node sums: from the model's adjoint grid, or summed over the
    // terms here
    const float *sg = kGrid ? sgrid6 + md.sgrid6_off : nullptr;
    SphGrid sgs = {1.0, 1.0, 1.0, 1.0};
    if (kGrid) sgs = sph_grid_scales(g, gauss + md.gauss_off);
    const int K = g.K, Tp = sph_terms_padded(g.J1, g.n_u);
    const float4 *gtc = terms + md.term_off;
    const float *gtf = (const float *)(gtc + Tp);
    const double *tab = gauss + md.gauss_off;
    const int cell = it.a;
    double r, sth, cth;
    sph_cell(g, cell, r, sth, cth);
    const double lnr = g.sph_lnr0 + (cell / kSphNT) * g.sph_dlnr;   // ln r (r = e^lnr)
    const double Rp0 = r * sth, zp0 = r * cth;
    const float R20 = (float)(Rp0 * Rp0), Z20 = (float)(zp0 * zp0);
    const int seg = lane >> 3, gi = lane & 7;
    const double glx = geoms[md.geom].gl8_x[gi], glw = geoms[md.geom].gl8_w[gi];
    double accF = 0.0;
    double Ar = 0.0, At = 0.0, Ap = 0.0;    // this wave's tracers (lane 0)
    constexpr int kTr = 2;                  // tracers per wave and round
    const int rounds = (K + 4 * kTr - 1) / (4 * kTr);
    for (int q = 0; q < rounds; ++q) {
      int kk[kTr];
      bool on[kTr];
      double alpha[kTr], alphaq[kTr], beta[kTr], nu0[kTr];
      SphNode nd[kTr];
      float R2[kTr], Z2[kTr];
#pragma unroll
      for (int u = 0; u < kTr; ++u) {
        kk[u] = 4 * (kTr * q + u) + wave;
        on[u] = kk[u] < K;                  // uniform per wave
        alpha[u] = 1.0; alphaq[u] = 1.0; beta[u] = 0.0; nu0[u] = 0.0;
        nd[u] = SphNode{};
        R2[u] = 0.f; Z2[u] = 0.f;
        if (on[u]) {
          const int k = kk[u];
          alpha[u] = tab[k];
          alphaq[u] = tab[K + k];
          nu0[u] = tab[2 * K + k];
          beta[u] = 1.0 - 1.0 / tab[3 * K + k];
          nd[u] = sph_node(r, lnr, sth, alpha[u], alphaq[u], beta[u], seg, glx, glw);
          R2[u] = (float)(nd[u].Rp * nd[u].Rp);
          Z2[u] = (float)(nd[u].zp * nd[u].zp);
        }
      }
      double aG[kTr], aT[kTr], aGR[kTr], aGZ[kTr], aTR[kTr], aTZ[kTr];
#pragma unroll
      for (int u = 0; u < kTr; ++u) aG[u] = aT[u] = aGR[u] = aGZ[u] = aTR[u] = aTZ[u] = 0.0;
      if (kGrid) {
#pragma unroll
        for (int u = 0; u < kTr; ++u)
          if (on[u]) {
            double v[6];
            sph_grid_at<6>(sg, sgs, nd[u].Rp, nd[u].zp, v);
            aG[u] = v[0]; aT[u] = v[1]; aGR[u] = v[2]; aGZ[u] = v[3]; aTR[u] = v[4]; aTZ[u] = v[5];
          }
      }
      // the terms: the node sums (without a grid) and, in the first round,
      // G_phi at the table point
      if (!kGrid || q == 0)
      for (int c0 = 0; c0 < Tp; c0 += kSphChunk) {
        const int cn = min(kSphChunk, Tp - c0);
        __syncthreads();
        for (int t = threadIdx.x; t < cn; t += 256) {
          const float4 c = gtc[c0 + t];
          tc[t] = c;
          tx[t] = make_float4(c.z * c.x, c.z * c.y, c.w * c.x, c.w * c.y);
          tf[t] = gtf[c0 + t];
        }
        __syncthreads();
        if (!kGrid && on[0]) {
          for (int t0 = 0; t0 < cn; t0 += 64) {
            float sG0 = 0.f, sT0 = 0.f, sGR0 = 0.f, sGZ0 = 0.f, sTR0 = 0.f, sTZ0 = 0.f;
            float sG1 = 0.f, sT1 = 0.f, sGR1 = 0.f, sGZ1 = 0.f, sTR1 = 0.f, sTZ1 = 0.f;
#pragma unroll 16
            for (int t = 0; t < 64; ++t) {
              const float4 c = tc[t0 + t], d = tx[t0 + t];
              const float e0 = fast_exp2(fmaf(c.x, R2[0], c.y * Z2[0]));
              const float e1 = fast_exp2(fmaf(c.x, R2[1], c.y * Z2[1]));
              sG0 = fmaf(c.z, e0, sG0);
              sT0 = fmaf(c.w, e0, sT0);
              sGR0 = fmaf(d.x, e0, sGR0);
              sGZ0 = fmaf(d.y, e0, sGZ0);
              sTR0 = fmaf(d.z, e0, sTR0);
              sTZ0 = fmaf(d.w, e0, sTZ0);
              sG1 = fmaf(c.z, e1, sG1);
              sT1 = fmaf(c.w, e1, sT1);
              sGR1 = fmaf(d.x, e1, sGR1);
              sGZ1 = fmaf(d.y, e1, sGZ1);
              sTR1 = fmaf(d.z, e1, sTR1);
              sTZ1 = fmaf(d.w, e1, sTZ1);
            }
            aG[0] += (double)sG0;
            aT[0] += (double)sT0;
            aGR[0] += (double)sGR0;
            aGZ[0] += (double)sGZ0;
            aTR[0] += (double)sTR0;
            aTZ[0] += (double)sTZ0;
            aG[1] += (double)sG1;
            aT[1] += (double)sT1;
            aGR[1] += (double)sGR1;
            aGZ[1] += (double)sGZ1;
            aTR[1] += (double)sTR1;
            aTZ[1] += (double)sTZ1;
          }
        }
        if (q == 0) {
          for (int t = threadIdx.x; t < cn; t += 256) {
            const float4 c = tc[t];
            accF += (double)(tf[t] * fast_exp2(fmaf(c.x, R20, c.y * Z20)));
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kTr; ++u) {
        if (!on[u]) continue;               // uniform per wave
        const SphNode &n = nd[u];
        const double be = beta[u];
        const double kap = 2.0 * (alphaq[u] - alpha[u]);
        const double nu = nu0[u] * n.en;
        const double H = aT[u] + kap * aG[u];
        // d/dbeta of the node: s' = s (r/r')^(1-beta) -> ds'/dbeta = s' tau
        const double ds = n.clamped ? 0.0 : n.st * n.tau;
        const double dc = n.ct > 0.0 ? -n.st * ds / n.ct : 0.0;
        const double dR = n.rp * ds, dz = n.rp * dc;
        const double dR2 = 2.0 * n.Rp * dR, dZ2 = 2.0 * n.zp * dz;
        const double dnu = -nu * (alpha[u] * dR2 + alphaq[u] * dZ2);
        // the term coefficients carry log2 e: dE/d(R'^2) = ln 2 c.x E
        const double dG = kLn2 * (aGR[u] * dR2 + aGZ[u] * dZ2);
        const double dH = kLn2 * (aTR[u] * dR2 + aTZ[u] * dZ2) + kap * dG;
        const double lrp = lnr + n.tau;     // ln r'
        // r'^beta = r^beta (r'/r)^beta; r'^(2 beta + 1), r'^(3 beta + 1)
        const double rbe = exp(be * lnr), rpb = rbe * n.rbt;
        const double pP = n.wn * n.rp * rpb * rpb;
        const double pD = pP * rpb;
        double fP = pP * nu * aG[u];
        double fD = pD * n.Rp * nu * H;
        double bP = pP * (2.0 * lrp * nu * aG[u] + dnu * aG[u] + nu * dG);
        double bD = pD * (3.0 * lrp * n.Rp * nu * H + dR * nu * H + n.Rp * dnu * H +
                          n.Rp * nu * dH);
        double qP = pP * aG[u] * (-n.zp * n.zp * nu);
        double qD = pD * n.Rp * (-n.zp * n.zp * nu * H + nu * 2.0 * aG[u]);
        double eP = pP * n.en * aG[u];
        double eD = pD * n.Rp * n.en * H;
        // the eight node sums; lanes 8 f .. 8 f + 7 hold sum f
        const double vs[8] = {fP, fD, bP, bD, qP, qD, eP, eD};
        const double ys = wave_sum8(vs, lane);
        if ((lane & 7) == 0)
          adj.jac[((int64_t)kk[u] * kSphCells + cell) * 8 + (lane >> 3)] = ys;
        fP = ys;                            // in lane 0
        fD = __shfl(ys, 8, 64);
        if (lane == 0) {
          const double rb2 = rbe * rbe;     // r^(-2 beta), r^(1 - 3 beta) below
          const double P = fP / rb2;
          Ar += P;
          At += (1.0 - be) * P;
          Ap += (1.0 - be) * P + (1.0 - be) * sth * (r / (rb2 * rbe)) * fD;
        }
      }
    }
    if (lane == 0) {
      wred[0][wave] = Ar;
      wred[1][wave] = At;
      wred[2][wave] = Ap;
    }
    const double Gphi = block_sum256(accF, sh);   // synchronises the block
    if (threadIdx.x == 0) {
      double nus = 0.0;
      for (int k = 0; k < K; ++k)
        nus += tab[2 * K + k] * exp(-(tab[k] * Rp0 * Rp0 + tab[K + k] * zp0 * zp0));
      out[0] = ((wred[0][0] + wred[0][1]) + wred[0][2]) + wred[0][3];
      out[1] = ((wred[1][0] + wred[1][1]) + wred[1][2]) + wred[1][3];
      out[2] = (((wred[2][0] + wred[2][1]) + wred[2][2]) + wred[2][3]) - nus * Rp0 * Rp0 * Gphi;
      adj.gphi[cell] = Gphi;
    }
    __syncthreads();
  }
}

// Rows of the characteristic integrals' adjoint: per (cell, tracer) the
// derivatives of the cell's L = lambda . (A_r, A_theta, A_phi) with respect
// to beta_k, alphaq_k and nu0_k from the node sums of k_sph_moments_jac and
// the table cotangent lambda; the A_phi term -nu R^2 G_phi adds its
// alphaq_k, nu0_k derivatives.  Item (m, table cell), thread = tracer.
__global__ void __launch_bounds__(64) k_sph_rows(const GeomDev *__restrict__ geoms,
                                                 const ModelDev *__restrict__ models,
                                                 const Item *__restrict__ items, int n_it,
                                                 const double *__restrict__ gauss,
                                                 const int *__restrict__ st_ws,
                                                 double *__restrict__ sens) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;          // uniform per block
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const SphAdj adj = sph_adj_of(sens, md, g);
    const int K = g.K, cell = it.a;
    const double *tab = gauss + md.gauss_off;
    double r, sth, cth;
    sph_cell(g, cell, r, sth, cth);
    const double Rp0 = r * sth, zp0 = r * cth;
    const double lr = adj.dtab[3 * cell], lt = adj.dtab[3 * cell + 1], lp = adj.dtab[3 * cell + 2];
    const double Gphi = adj.gphi[cell];
    const double lnr = log(r);
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const double *jr = adj.jac + ((int64_t)k * kSphCells + cell) * 8;
      const double fP = jr[0], fD = jr[1], bP = jr[2], bD = jr[3];
      const double qP = jr[4], qD = jr[5], eP = jr[6], eD = jr[7];
      const double be = 1.0 - 1.0 / tab[3 * K + k];
      const double rbe = exp(be * lnr);   // r^beta: r^(-2 beta), r^(1 - 3 beta)
      const double rb = 1.0 / (rbe * rbe), rd = r * rb / rbe;
      const double P = rb * fP;
      const double muP = lr + (1.0 - be) * (lt + lp);
      const double muD = lp * (1.0 - be) * sth * rd;
      const double dbeta = muP * rb * bP + muD * bD - (lt + lp) * P - 2.0 * lnr * muP * P -
                           fD * lp * sth * rd * (1.0 + 3.0 * (1.0 - be) * lnr);
      const double e0 = exp(-(tab[k] * Rp0 * Rp0 + tab[K + k] * zp0 * zp0));
      double *row = adj.rows + ((int64_t)k * kSphCells + cell) * 3;
      row[0] = dbeta;
      row[1] = (muP * rb * qP + muD * qD) + lp * Rp0 * Rp0 * Gphi * tab[2 * K + k] * e0 * zp0 * zp0;
      row[2] = (muP * rb * eP + muD * eD) + -lp * Rp0 * Rp0 * Gphi * e0;
    }
  }
}

// Point p = (cell, tracer, node) of a model's characteristic integrals: the
// node (as in the forward, with the powers of r and r' written as
// exponentials of ln r and tau, r' = r e^tau) and the cotangents phi =
// dL/dG and psi = dL/dG_theta there, from the table cotangent in adj.dtab.
// sinth: sin of the table's polar angles; gp: the geometry (its 8-node rule
// is read from global memory: a lane-dependent index into a by-value
// descriptor would go to scratch).
__device__ inline void sph_point_cot(const GeomDev &g, const GeomDev *__restrict__ gp,
                                     const double *tab, const SphAdj &adj, const double *sinth,
                                     int64_t p, double &Rp, double &zp, double &phi,
                                     double &psi) {
  const int K = g.K;
  const int cell = (int)(p / ((int64_t)K * kSphNodes));
  const int k = (int)((p / kSphNodes) % K), node = (int)(p % kSphNodes);
  const int ir = cell / kSphNT, ith = cell % kSphNT;
  const double lnr = g.sph_lnr0 + ir * g.sph_dlnr, r = exp(lnr);
  const double sth = sinth[ith];
  const double lr = adj.dtab[3 * cell], lt = adj.dtab[3 * cell + 1];
  const double lp = adj.dtab[3 * cell + 2];
  const double alpha = tab[k], alphaq = tab[K + k], nu0 = tab[2 * K + k];
  const double beta = 1.0 - 1.0 / tab[3 * K + k];
  const int gi = node & 7;
  const double glx = gp->gl8_x[gi], glw = gp->gl8_w[gi];
  const double hs = 0.5 * log1p(50.0 * (0.5 / alpha) / (r * r)) / kSphSeg;
  const double tau = ((node >> 3) + 0.5 + 0.5 * glx) * hs;
  const double rp = exp(lnr + tau);
  const double rbt = exp(beta * tau);    // (r'/r)^beta
  const double st = fmin(1.0, sth * (r / rp) * rbt);
  const double ct = sqrt(fmax(0.0, 1.0 - st * st));
  Rp = rp * st;
  zp = rp * ct;
  const double wn = 0.5 * glw * hs * rp;
  const double nu = nu0 * exp(-(alpha * Rp * Rp + alphaq * zp * zp));
  const double muP = lr + (1.0 - beta) * (lt + lp);
  // r^beta, r'^beta; r^(1 - 3 beta), r'^(3 beta + 1) and r'^(2 beta + 1)
  // r^(-2 beta) = r' (r'/r)^(2 beta) as their products
  const double rbe = exp(beta * lnr), rpb = rbe * rbt;
  const double muD = lp * (1.0 - beta) * sth * (r / (rbe * rbe * rbe));
  const double dD = muD * wn * (rp * rpb * rpb * rpb) * Rp * nu;
  phi = muP * wn * (rp * rbt * rbt) * nu + dD * 2.0 * (alphaq - alpha);
  psi = dD;
}

// Term-major sensitivities.  Item (m, 256-term tile, point range); thread =
// term.  Each 256-point chunk of the range is regenerated (thread = point):
// node position and the cotangents phi = dL/dG, psi = dL/dG_theta at the
// node; then every term sums phi E, psi E and their R'^2, z'^2 moments over
// the chunk in FP32, folded into FP64.
__global__ void __launch_bounds__(256) k_sph_sens(const GeomDev *__restrict__ geoms,
                                                  const ModelDev *__restrict__ models,
                                                  const Item *__restrict__ items, int n_it,
                                                  const double *__restrict__ gauss,
                                                  const float4 *__restrict__ terms,
                                                  const int *__restrict__ st_ws,
                                                  double *__restrict__ sens) {
  __shared__ float4 pa[256];   // (R'^2, z'^2, phi, psi)
  __shared__ float4 pb[256];   // (phi R'^2, psi R'^2, phi z'^2, psi z'^2)
  __shared__ double sc[2][kSphNT];   // sin, cos of the table's polar angles
  if (threadIdx.x < kSphNT) {
    const double th = threadIdx.x * (0.5 * kPi / (kSphNT - 1));
    sc[0][threadIdx.x] = sin(th);
    sc[1][threadIdx.x] = cos(th);
  }
  __syncthreads();
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;
    const SphAdj adj = sph_adj_of(sens, md, g);
    const int K = g.K, Tp = sph_terms_padded(g.J1, g.n_u);
    const double *tab = gauss + md.gauss_off;
    const int t = it.a * 256 + threadIdx.x;
    const bool tv = t < Tp;
    const float4 c = tv ? terms[md.term_off + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t len = sph_range_len(K, md.n_sens_parts), P = sph_points(K);
    const int64_t p0 = (int64_t)it.b * len, p1 = min(P, p0 + len);
    double SP = 0.0, ST = 0.0, SxP = 0.0, SxT = 0.0, SyP = 0.0, SyT = 0.0;
    for (int64_t c0 = p0; c0 < p1; c0 += 256) {
      // regenerate this chunk's points
      const int64_t p = c0 + threadIdx.x;
      float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
      if (p < p1) {
        double Rp, zp, phi, psi;
        sph_point_cot(g, geoms + md.geom, tab, adj, sc[0], p, Rp, zp, phi, psi);
        const float R2 = (float)(Rp * Rp), Z2 = (float)(zp * zp);
        const float fphi = (float)phi, fpsi = (float)psi;
        va = make_float4(R2, Z2, fphi, fpsi);
        vb = make_float4(fphi * R2, fpsi * R2, fphi * Z2, fpsi * Z2);
      }
      __syncthreads();
      pa[threadIdx.x] = va;
      pb[threadIdx.x] = vb;
      __syncthreads();
      float sP = 0.f, sT = 0.f, sxP = 0.f, sxT = 0.f, syP = 0.f, syT = 0.f;
      if (tv) {
#pragma unroll 16
        for (int j = 0; j < 256; ++j) {   // points past the range are zero
          const float4 A = pa[j], B = pb[j];
          const float e = fast_exp2(fmaf(c.x, A.x, c.y * A.y));
          sP = fmaf(A.z, e, sP);
          sT = fmaf(A.w, e, sT);
          sxP = fmaf(B.x, e, sxP);
          sxT = fmaf(B.y, e, sxT);
          syP = fmaf(B.z, e, syP);
          syT = fmaf(B.w, e, syT);
        }
      }
      SP += (double)sP;
      ST += (double)sT;
      SxP += (double)sxP;
      SxT += (double)sxT;
      SyP += (double)syP;
      SyT += (double)syT;
    }
    if (tv) {
      double *o = adj.sparts + ((int64_t)it.b * Tp + t) * 6;
      o[0] = SP;
      o[1] = ST;
      o[2] = SxP;
      o[3] = SxT;
      o[4] = SyP;
      o[5] = SyT;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Term-major sensitivities through the potential grid.  With the adjoint's
// node sums interpolated from the grid, the term sensitivities are those of
// the grid values: the point cotangents phi, psi are spread onto the grid
// with the interpolation's own weights (its transpose), and per term
//   S_phi = sum_il Phi[i, l] E_t(R_i, z_l),  E_t = 2^(cx R_i^2) 2^(cy z_l^2),
// with the R^2 and z^2 moments, is one more matrix-core contraction over the
// grid.  The spreading adds 64-bit fixed-point integers at a per-model
// power-of-two scale, so the grid cotangent, like the table cotangent, does
// not depend on the order of the additions.
// Workspace per model (8-byte slots from sgcot_off): the fixed-point grid
// [N][N][2] (phi, psi), the FP32 grid [N][N][2], the bound partials
// [items][2] and the two scales.
// ---------------------------------------------------------------------------
__device__ inline long long *sph_gcot_fixed(double *sgcot, const ModelDev &md) {
  return reinterpret_cast<long long *>(sgcot + md.sgcot_off);
}
__device__ inline float *sph_gcot_float(double *sgcot, const ModelDev &md) {
  return reinterpret_cast<float *>(sgcot + md.sgcot_off + 2LL * kSphGridN * kSphGridN);
}
__device__ inline double *sph_gcot_bounds(double *sgcot, const ModelDev &md) {
  return sgcot + md.sgcot_off + 3LL * kSphGridN * kSphGridN;
}

// The int32 part of the grid-cotangent workspace: per (point item, tile)
// list positions, tile offsets, the consistency flag, the point list; then
// one byte per point, its tile.
__device__ inline int *sph_gcot_int(double *sgcot, const ModelDev &md, int K) {
  return reinterpret_cast<int *>(sph_gcot_bounds(sgcot, md) + 2LL * sph_pitems(K) + 2);
}
__device__ inline unsigned char *sph_gcot_ptile(double *sgcot, const ModelDev &md, int K) {
  return reinterpret_cast<unsigned char *>(sph_gcot_int(sgcot, md, K) + sph_gcot_ints(K));
}

// The grid tile (of kSphTileB x kSphTileB stencil base cells) that holds
// the stencil base cell of a point at (R, z): tile row b starts at
// R = aR sinh(kSphTileB b / iR) (bR[b], b = 1 .. kSphTilesAx - 1), and
// likewise in z (bZ).  A point within rounding of a boundary may land in
// the neighbouring tile; the tile pass takes its stencil all the same.
__device__ inline void sph_tile_bounds(const SphGrid &sc, double *bR, double *bZ) {
  for (int b = threadIdx.x; b < kSphTilesAx; b += blockDim.x) {
    bR[b] = sc.aR * sinh(kSphTileB * b / sc.iR);
    bZ[b] = sc.aZ * sinh(kSphTileB * b / sc.iZ);
  }
}
__device__ inline int sph_tile_at(const double *bR, const double *bZ, double R, double z) {
  static_assert(kSphTilesAx == 16, "a four-step search");
  int tx = 0, tz = 0;
#pragma unroll
  for (int step = 8; step >= 1; step >>= 1) {
    if (R >= bR[tx + step]) tx += step;
    if (z >= bZ[tz + step]) tz += step;
  }
  return tx * kSphTilesAx + tz;
}

// Item (m, point item q): clears a share of the fixed-point grid, sums
// |phi|, |psi| over the item's points (fixed-order block sums), and counts
// them per grid tile, recording each point's tile.
__global__ void __launch_bounds__(256) k_sph_pcot_bound(const GeomDev *__restrict__ geoms,
                                                        const ModelDev *__restrict__ models,
                                                        const Item *__restrict__ items, int n_it,
                                                        const double *__restrict__ gauss,
                                                        const int *__restrict__ st_ws,
                                                        double *__restrict__ sens,
                                                        double *__restrict__ sgcot) {
  static_assert(kSphTiles == 256, "one thread per tile");
  __shared__ double sinth[kSphNT];
  __shared__ double sh[256];
  __shared__ double bR[kSphTilesAx], bZ[kSphTilesAx];
  __shared__ int hist[kSphTiles];
  if (threadIdx.x < kSphNT) sinth[threadIdx.x] = sin(threadIdx.x * (0.5 * kPi / (kSphNT - 1)));
  __syncthreads();
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;          // uniform per block
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const SphAdj adj = sph_adj_of(sens, md, g);
    const double *tab = gauss + md.gauss_off;
    const SphGrid sc = sph_grid_scales(g, tab);
    const int np = sph_pitems(g.K);
    const int64_t n2 = 2LL * kSphGridN * kSphGridN, share = (n2 + np - 1) / np;
    long long *fx = sph_gcot_fixed(sgcot, md);
    const int64_t e0 = (int64_t)it.a * share, e1 = min(n2, e0 + share);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) fx[e] = 0;
    int *gi = sph_gcot_int(sgcot, md, g.K);
    unsigned char *ptile = sph_gcot_ptile(sgcot, md, g.K);
    if (it.a == 0 && threadIdx.x == 0) gi[(int64_t)np * kSphTiles + kSphTiles + 1] = 0;   // flag
    hist[threadIdx.x] = 0;
    sph_tile_bounds(sc, bR, bZ);
    __syncthreads();
    const int64_t P = sph_points(g.K), p0 = (int64_t)it.a * kSphPtsItem,
                  p1 = min(P, p0 + kSphPtsItem);
    double sa = 0.0, sb = 0.0;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
      double R, z, phi, psi;
      sph_point_cot(g, geoms + md.geom, tab, adj, sinth, p, R, z, phi, psi);
      sa += fabs(phi);
      sb += fabs(psi);
      const int tile = sph_tile_at(bR, bZ, R, z);
      ptile[p] = (unsigned char)tile;
      atomicAdd(&hist[tile], 1);
    }
    sa = block_sum256(sa, sh);
    sb = block_sum256(sb, sh);
    if (threadIdx.x == 0) {
      double *bnd = sph_gcot_bounds(sgcot, md);
      bnd[2 * it.a] = sa;
      bnd[2 * it.a + 1] = sb;
    }
    __syncthreads();
    gi[(int64_t)it.a * kSphTiles + threadIdx.x] = hist[threadIdx.x];
    __syncthreads();                         // hist, bR, bZ read before the next item
  }
}

// Model m: the per-item tile counts become list positions, items in order
// within a tile and tiles in order, and the tile offsets.  Thread (tile,
// part) takes a quarter of the items; the parts are added in order.
constexpr int kScanParts = 4;
__global__ void __launch_bounds__(kSphTiles * kScanParts) k_sph_pcot_scan(
    const GeomDev *__restrict__ geoms, const ModelDev *__restrict__ models, int n,
    const int *__restrict__ st_ws, double *__restrict__ sgcot) {
  __shared__ int part[kScanParts][kSphTiles];   // per part: its count, then its offset
  __shared__ int tsz[kSphTiles], tot[kSphTiles];
  const int t = threadIdx.x % kSphTiles, r = threadIdx.x / kSphTiles;
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    if (st_ws[m] != 0) continue;             // uniform per block
    const ModelDev md = models[m];
    const int K = geoms[md.geom].K;
    const int np = sph_pitems(K);
    int *pos = sph_gcot_int(sgcot, md, K);
    int *toff = pos + (int64_t)np * kSphTiles;
    const int per = (np + kScanParts - 1) / kScanParts;
    const int q0 = min(np, r * per), q1 = min(np, q0 + per);
    // the part's items: counts to offsets within the part
    int acc = 0;
    for (int q = q0; q < q1; q += 8) {
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = q + u < q1 ? pos[(int64_t)(q + u) * kSphTiles + t] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (q + u < q1) pos[(int64_t)(q + u) * kSphTiles + t] = acc;
        acc += v[u];
      }
    }
    __syncthreads();                         // the previous model's reads of part, tsz, tot
    part[r][t] = acc;
    __syncthreads();
    if (r == 0) {
      int s0 = 0;
      for (int rr = 0; rr < kScanParts; ++rr) {
        const int v = part[rr][t];
        part[rr][t] = s0;
        s0 += v;
      }
      tsz[t] = s0;
      tot[t] = s0;
    }
    __syncthreads();
    // inclusive scan of the tile sizes over the tiles
    for (int off = 1; off < kSphTiles; off <<= 1) {
      const int v = (r == 0 && t >= off) ? tot[t - off] : 0;
      __syncthreads();
      if (r == 0) tot[t] += v;
      __syncthreads();
    }
    const int tile0 = tot[t] - tsz[t];
    if (r == 0) {
      toff[t] = tile0;
      if (t == kSphTiles - 1) toff[kSphTiles] = tot[t];
    }
    const int base = tile0 + part[r][t];
    for (int q = q0; q < q1; q += 8) {
      int v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = q + u < q1 ? pos[(int64_t)(q + u) * kSphTiles + t] : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q + u < q1) pos[(int64_t)(q + u) * kSphTiles + t] = v[u] + base;
    }
  }
}

// Item (m, point item q): the item's point indices into the list, each at
// its recorded tile's range for this item (the order within a range is
// immaterial: the grid sums are exact).  A count that disagrees with the
// counting pass sets the model's flag, and the tile pass then spreads that
// model's points directly.
__global__ void __launch_bounds__(256) k_sph_pcot_fill(const GeomDev *__restrict__ geoms,
                                                       const ModelDev *__restrict__ models,
                                                       const Item *__restrict__ items, int n_it,
                                                       const double *__restrict__ gauss,
                                                       const int *__restrict__ st_ws,
                                                       double *__restrict__ sgcot) {
  __shared__ int cur[kSphTiles], rb[kSphTiles], rl[kSphTiles];   // fill count, range
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;          // uniform per block
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int np = sph_pitems(g.K);
    int *pos = sph_gcot_int(sgcot, md, g.K);
    const unsigned char *ptile = sph_gcot_ptile(sgcot, md, g.K);
    const int *toff = pos + (int64_t)np * kSphTiles;
    int *flag = pos + (int64_t)np * kSphTiles + kSphTiles + 1;
    int *list = flag + 1;
    rb[threadIdx.x] = pos[(int64_t)it.a * kSphTiles + threadIdx.x];
    rl[threadIdx.x] = it.a + 1 < np ? pos[(int64_t)(it.a + 1) * kSphTiles + threadIdx.x]
                                    : toff[threadIdx.x + 1];
    cur[threadIdx.x] = 0;
    __syncthreads();                         // ranges read, cur cleared
    const int64_t P = sph_points(g.K), p0 = (int64_t)it.a * kSphPtsItem,
                  p1 = min(P, p0 + kSphPtsItem);
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
      const int tile = ptile[p];
      const int at = rb[tile] + atomicAdd(&cur[tile], 1);
      if (at < rl[tile]) list[at] = (int)p;
    }
    __syncthreads();
    if (cur[threadIdx.x] != rl[threadIdx.x] - rb[threadIdx.x]) atomicOr(flag, 1);
    __syncthreads();                         // before the next item rewrites cur, rb, rl
  }
}

// The power of two that maps 1.6 x bound (the interpolation weights of a
// point sum to at most 1.25^2 in magnitude) below 2^60; NaN for a
// non-finite bound.
__device__ inline double sph_gcot_scale(double bound) {
  if (bound == 0.0) return 1.0;
  if (!(bound < __builtin_inf())) return __builtin_nan("");
  return ldexp(1.0, min(1000, 60 - ilogb(1.6 * bound)));
}

// The point cotangents of p onto the grid through the interpolation's
// weights, in fixed point: into the LDS block acc (rows r0 .. r0 + kL - 1,
// columns c0 .. c0 + kL - 1) where the stencil lies inside it, else
// straight into the grid.
constexpr int kTileL = kSphTileB + 5;   // a tile's stencils with one cell to spare
constexpr int kTileSub = 4;             // list parts per point item in the tile pass
__device__ inline void sph_spread_point(const GeomDev &g, const GeomDev *__restrict__ gp,
                                        const double *tab, const SphAdj &adj,
                                        const double *sinth, const SphGrid &sc, double sa,
                                        double sb, int64_t p, unsigned long long *fx,
                                        unsigned long long *acc, int r0, int c0) {
  constexpr int N = kSphGridN;
  double R, z, phi, psi;
  sph_point_cot(g, gp, tab, adj, sinth, p, R, z, phi, psi);
  const double x = asinh(R / sc.aR) * sc.iR, y = asinh(z / sc.aZ) * sc.iZ;
  const int i0 = min(max((int)floor(x), 0), N - 3), l0 = min(max((int)floor(y), 0), N - 3);
  double wx[4], wy[4];
  lagrange4(x - i0, wx);
  lagrange4(y - l0, wy);
  const int ra = abs(i0 - 1), ca = abs(l0 - 1);
  const bool in = acc && ra >= r0 && i0 + 2 < r0 + kTileL && ca >= c0 && l0 + 2 < c0 + kTileL &&
                  i0 >= r0 && l0 >= c0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int row = abs(i0 - 1 + a);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int col = abs(l0 - 1 + b);
      const double w = wx[a] * wy[b];
      const long long va = __double2ll_rn(phi * w * sa), vb = __double2ll_rn(psi * w * sb);
      unsigned long long *c = in ? acc + ((row - r0) * kTileL + (col - c0)) * 2
                                 : fx + ((int64_t)row * N + col) * 2;
      if (va) atomicAdd(c, (unsigned long long)va);
      if (vb) atomicAdd(c + 1, (unsigned long long)vb);
    }
  }
}

// Item (m, q) split in kTileSub parts: part s takes entries
// q * kSphPtsItem + s * kSphPtsItem / kTileSub onwards (kSphPtsItem /
// kTileSub of them) of the model's tile-sorted point list.  Per tile met
// there, the entries' stencils are summed in an LDS block (fixed point, so
// in any order) and the block is added to the grid; with the model's flag
// set, the same range of points is spread straight onto the grid instead.
__global__ void __launch_bounds__(256) k_sph_pcot_tiles(const GeomDev *__restrict__ geoms,
                                                        const ModelDev *__restrict__ models,
                                                        const Item *__restrict__ items, int n_it,
                                                        const double *__restrict__ gauss,
                                                        const int *__restrict__ st_ws,
                                                        double *__restrict__ sens,
                                                        double *__restrict__ sgcot) {
  constexpr int N = kSphGridN;
  __shared__ double sinth[kSphNT];
  __shared__ double sh[256];
  __shared__ unsigned long long acc[kTileL * kTileL * 2];
  __shared__ int tr[2];
  if (threadIdx.x < kSphNT) sinth[threadIdx.x] = sin(threadIdx.x * (0.5 * kPi / (kSphNT - 1)));
  __syncthreads();
  constexpr int kSub = kSphPtsItem / kTileSub;
  for (int vi = blockIdx.x; vi < n_it * kTileSub; vi += gridDim.x) {
    const Item it = items[vi / kTileSub];
    const int sub = vi % kTileSub;
    if (st_ws[it.m] != 0) continue;          // uniform per block
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const SphAdj adj = sph_adj_of(sens, md, g);
    const double *tab = gauss + md.gauss_off;
    const int np = sph_pitems(g.K);
    const int64_t P = sph_points(g.K), e0 = (int64_t)it.a * kSphPtsItem + sub * kSub,
                  e1 = min(P, e0 + kSub);
    if (e0 >= P) continue;                   // uniform: the model's last item ends early
    double *bnd = sph_gcot_bounds(sgcot, md);
    double ba = 0.0, bb = 0.0;
    for (int q = threadIdx.x; q < np; q += 256) { ba += bnd[2 * q]; bb += bnd[2 * q + 1]; }
    ba = block_sum256(ba, sh);
    bb = block_sum256(bb, sh);
    const double sa = sph_gcot_scale(ba), sb = sph_gcot_scale(bb);
    if (it.a == 0 && sub == 0 && threadIdx.x == 0) { bnd[2 * np] = sa; bnd[2 * np + 1] = sb; }
    if (!(sa == sa) || !(sb == sb)) continue;   // uniform: a non-finite cotangent
    const SphGrid sc = sph_grid_scales(g, tab);
    unsigned long long *fx = reinterpret_cast<unsigned long long *>(sph_gcot_fixed(sgcot, md));
    const int *pos = sph_gcot_int(sgcot, md, g.K);
    const int *toff = pos + (int64_t)np * kSphTiles;
    const int flag = toff[kSphTiles + 1];
    const int *list = toff + kSphTiles + 2;
    if (flag) {                              // uniform
      for (int64_t p = e0 + threadIdx.x; p < e1; p += 256)
        sph_spread_point(g, geoms + md.geom, tab, adj, sinth, sc, sa, sb, p, fx, nullptr, 0, 0);
      continue;
    }
    // the tiles whose list ranges meet [e0, e1)
    const int t = threadIdx.x;
    if (toff[t] <= e0 && e0 < toff[t + 1]) tr[0] = t;
    if (toff[t] < e1 && e1 <= toff[t + 1]) tr[1] = t;
    __syncthreads();
    const int ta = tr[0], tb = tr[1];
    __syncthreads();                         // tr read before the next item writes it
    for (int tile = ta; tile <= tb; ++tile) {
      const int64_t s0 = max(e0, (int64_t)toff[tile]), s1 = min(e1, (int64_t)toff[tile + 1]);
      if (s0 >= s1) continue;                // uniform
      const int r0 = (tile / kSphTilesAx) * kSphTileB - 2, c0 = (tile % kSphTilesAx) * kSphTileB - 2;
      for (int e = t; e < kTileL * kTileL * 2; e += 256) acc[e] = 0ull;
      __syncthreads();
      for (int64_t e = s0 + t; e < s1; e += 256)
        sph_spread_point(g, geoms + md.geom, tab, adj, sinth, sc, sa, sb, list[e], fx, acc, r0, c0);
      __syncthreads();
      for (int e = t; e < kTileL * kTileL; e += 256) {
        const int row = r0 + e / kTileL, col = c0 + e % kTileL;
        const unsigned long long va = acc[2 * e], vb = acc[2 * e + 1];
        if (row >= 0 && row < N && col >= 0 && col < N) {
          unsigned long long *c = fx + ((int64_t)row * N + col) * 2;
          if (va) atomicAdd(c, va);
          if (vb) atomicAdd(c + 1, vb);
        }
      }
      __syncthreads();                       // the block is read before it is cleared
    }
  }
}

// Item (m, block of 1024 grid points): the fixed-point grid cotangent back
// to FP32 (NaN for a non-finite cotangent).
__global__ void __launch_bounds__(256) k_sph_pcot_fix(const GeomDev *__restrict__ geoms,
                                                      const ModelDev *__restrict__ models,
                                                      const Item *__restrict__ items, int n_it,
                                                      const int *__restrict__ st_ws,
                                                      double *__restrict__ sgcot) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const double *bnd = sph_gcot_bounds(sgcot, md);
    const int np = sph_pitems(g.K);
    const double sa = bnd[2 * np], sb = bnd[2 * np + 1];
    const long long *fx = sph_gcot_fixed(sgcot, md);
    float *fl = sph_gcot_float(sgcot, md);
    for (int e = it.a * 1024 + threadIdx.x; e < (it.a + 1) * 1024; e += 256) {
      fl[2 * e] = (float)(sa == sa ? (double)fx[2 * e] / sa : sa);
      fl[2 * e + 1] = (float)(sb == sb ? (double)fx[2 * e + 1] / sb : sb);
    }
  }
}

// Item (m, block of 32 terms, part ip of kSphIParts): wave w contracts grid
// rows 32 (4 ip + w) .. + 31 with the terms' z factors, D = Phi B and
// Dz = Phi (z^2 B) (and for psi), reading four grid columns per lane and
// 16 bytes at a time; then per term the row sums with 2^(cx R_i^2) and
// R_i^2 2^(cx R_i^2), FP32 per lane, FP64 across lanes and waves (fixed
// order).  Output: the part's [S_phi, S_psi, R^2 S_phi, R^2 S_psi, z^2 S_phi,
// z^2 S_psi] per term, as k_sph_sens's ranges.
__global__ void __launch_bounds__(256) k_sph_sens_grid(const GeomDev *__restrict__ geoms,
                                                       const ModelDev *__restrict__ models,
                                                       const Item *__restrict__ items, int n_it,
                                                       const double *__restrict__ gauss,
                                                       const float4 *__restrict__ terms,
                                                       const int *__restrict__ st_ws,
                                                       double *__restrict__ sens,
                                                       double *__restrict__ sgcot) {
  constexpr int N = kSphGridN;
  __shared__ __attribute__((aligned(16))) float zsq[N];
  __shared__ float rsq[N];
  __shared__ double red[4][6][32];
  const int lane = threadIdx.x & 63, c32 = lane & 31, kh = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const v16f zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    if (st_ws[it.m] != 0) continue;          // uniform per block
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const SphGrid sc = sph_grid_scales(g, gauss + md.gauss_off);
    __syncthreads();                         // the previous item's reads of zsq, rsq, red
    for (int l = threadIdx.x; l < N; l += 256) {
      const double zv = sc.aZ * sinh(l / sc.iZ), rv = sc.aR * sinh(l / sc.iR);
      zsq[l] = (float)(zv * zv);
      rsq[l] = (float)(rv * rv);
    }
    __syncthreads();
    const int Tp = sph_terms_padded(g.J1, g.n_u);
    const int t = 32 * it.a + c32;           // < Tp (Tp is a multiple of 64)
    const float4 c = terms[md.term_off + t];
    const float *fl = sph_gcot_float(sgcot, md);
    const int row = 32 * (kSphIParts * it.b + wave) + c32;
    const float *fr = fl + (int64_t)row * N * 2;
    v16f dP = zero, dPz = zero, dT = zero, dTz = zero;
    for (int q = 0; q < N / 8; ++q) {
      const int l0 = 8 * q + 4 * kh;
      const float4 pa = *reinterpret_cast<const float4 *>(fr + 2 * l0);
      const float4 pb = *reinterpret_cast<const float4 *>(fr + 2 * l0 + 4);
      const float4 zz = *reinterpret_cast<const float4 *>(&zsq[l0]);
      const float ap[4] = {pa.x, pa.z, pb.x, pb.z}, at[4] = {pa.y, pa.w, pb.y, pb.w};
      const float z4[4] = {zz.x, zz.y, zz.z, zz.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float b = fast_exp2(c.y * z4[j]), bz = b * z4[j];
        dP = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[j], b, dP, 0, 0, 0);
        dPz = __builtin_amdgcn_mfma_f32_32x32x2f32(ap[j], bz, dPz, 0, 0, 0);
        dT = __builtin_amdgcn_mfma_f32_32x32x2f32(at[j], b, dT, 0, 0, 0);
        dTz = __builtin_amdgcn_mfma_f32_32x32x2f32(at[j], bz, dTz, 0, 0, 0);
      }
    }
    // rows of this lane: 32 (4 ip + w) + mfma_row(r, lane); column = term t
    float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int rbase = 32 * (kSphIParts * it.b + wave);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float r2 = rsq[rbase + mfma_row(r, lane)];
      const float e = fast_exp2(c.x * r2);
      s[0] = fmaf(e, dP[r], s[0]);
      s[1] = fmaf(e, dT[r], s[1]);
      s[2] = fmaf(e * r2, dP[r], s[2]);
      s[3] = fmaf(e * r2, dT[r], s[3]);
      s[4] = fmaf(e, dPz[r], s[4]);
      s[5] = fmaf(e, dTz[r], s[5]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = (double)s[k];
      v += __shfl_xor(v, 32, 64);
      if (kh == 0) red[wave][k][c32] = v;
    }
    __syncthreads();
    if (wave == 0 && kh == 0) {
      const SphAdj adj = sph_adj_of(sens, md, g);
      double *o = adj.sparts + ((int64_t)it.b * Tp + t) * 6;
#pragma unroll
      for (int k = 0; k < 6; ++k) o[k] = ((red[0][k][c32] + red[1][k][c32]) + red[2][k][c32]) + red[3][k][c32];
    }
  }
}

// Term sensitivities of the table points' G_phi term (chi = -lambda_phi nu
// R0^2 per cell).  Item (m, 256-term tile) split in kSphCellParts parts of
// 256 cells; thread = term.  Each part's FP32 sums go to their own slot.
__global__ void __launch_bounds__(256) k_sph_sens_cells(const GeomDev *__restrict__ geoms,
                                                        const ModelDev *__restrict__ models,
                                                        const Item *__restrict__ items, int n_it,
                                                        const double *__restrict__ gauss,
                                                        const float4 *__restrict__ terms,
                                                        const int *__restrict__ st_ws,
                                                        double *__restrict__ sens) {
  __shared__ float4 pc[256];   // (R0^2, z0^2, chi, 0)
  for (int vi = blockIdx.x; vi < n_it * kSphCellParts; vi += gridDim.x) {
    const Item it = items[vi / kSphCellParts];
    const int part = vi % kSphCellParts;
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;
    const SphAdj adj = sph_adj_of(sens, md, g);
    const int K = g.K, Tp = sph_terms_padded(g.J1, g.n_u);
    const double *tab = gauss + md.gauss_off;
    const int t = it.a * 256 + threadIdx.x;
    const bool tv = t < Tp;
    const float4 c = tv ? terms[md.term_off + t] : make_float4(0.f, 0.f, 0.f, 0.f);
    double SF = 0.0, SxF = 0.0, SyF = 0.0;
    {
      const int cell = part * 256 + threadIdx.x;
      double r, sth, cth;
      sph_cell(g, cell, r, sth, cth);
      const double R0 = r * sth, z0 = r * cth;
      double nus = 0.0;
      for (int k = 0; k < K; ++k) nus += tab[2 * K + k] * exp(-(tab[k] * R0 * R0 + tab[K + k] * z0 * z0));
      const double chi = -adj.dtab[3 * cell + 2] * nus * R0 * R0;
      __syncthreads();
      pc[threadIdx.x] = make_float4((float)(R0 * R0), (float)(z0 * z0), (float)chi, 0.f);
      __syncthreads();
      float sF = 0.f, sx = 0.f, sy = 0.f;
      if (tv) {
        for (int j = 0; j < 256; ++j) {
          const float4 A = pc[j];
          const float e = A.z * fast_exp2(fmaf(c.x, A.x, c.y * A.y));
          sF += e;
          sx = fmaf(A.x, e, sx);
          sy = fmaf(A.y, e, sy);
        }
      }
      SF += (double)sF;
      SxF += (double)sx;
      SyF += (double)sy;
    }
    if (tv) {
      double *o = adj.cparts + ((int64_t)part * Tp + t) * 3;
      o[0] = SF;
      o[1] = SxF;
      o[2] = SyF;
    }
    __syncthreads();
  }
}

// Per-term chain (FP64): the sensitivities summed over the point ranges in a
// fixed order, then through the coefficients' dependence on e_j^2 and K_j.
// Item (m, 256-term tile); thread = term.
__global__ void __launch_bounds__(256) k_sph_chain(const GeomDev *__restrict__ geoms,
                                                   const ModelDev *__restrict__ models,
                                                   const Item *__restrict__ items, int n_it,
                                                   const double *__restrict__ gauss,
                                                   const int *__restrict__ st_ws,
                                                   double *__restrict__ sens) {
  constexpr double kLn2 = 0.6931471805599453, kLog2e = 1.4426950408889634;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;
    const SphAdj adj = sph_adj_of(sens, md, g);
    const int Tp = sph_terms_padded(g.J1, g.n_u), T = g.J1 * g.n_u;
    const int t = it.a * 256 + threadIdx.x;
    if (t >= T) continue;
    double S[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int rg = 0; rg < md.n_sens_parts; ++rg) {
      const double *o = adj.sparts + ((int64_t)rg * Tp + t) * 6;
#pragma unroll
      for (int c = 0; c < 6; ++c) S[c] += o[c];
    }
    // the cell parts in order
    double cp[3] = {0.0, 0.0, 0.0};
    for (int pt = 0; pt < kSphCellParts; ++pt) {
      const double *o = adj.cparts + ((int64_t)pt * Tp + t) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) cp[c] += o[c];
    }
    const double *mt = gauss + md.gauss_off + 4 * g.K;
    const int j = t / g.n_u, n = t % g.n_u;
    const double rj = mt[j], e2 = mt[g.J1 + j], Kp = mt[2 * g.J1 + j];
    const double u = g.u[n], u2 = u * u, w = g.w[n];
    const double h = 1.0 - e2 * u2, h15 = h * sqrt(h);
    // coefficients per unit K_j
    const double P1 = w * 2.0 * rj * u2 / h15;
    const double T1 = w * e2 * 4.0 * rj * rj * u2 * u2 * u2 / (h15 * h);
    const double F1 = w * e2 * 2.0 * rj * u2 * u2 / h15;
    const double cy = -rj * u2 / h * kLog2e;
    const double dcy = kLn2 * Kp * (P1 * S[4] + T1 * S[5] + F1 * cp[2]);   // dL/dc_y
    const double dP1 = P1 * 1.5 * u2 / h;
    const double dT1 = w * 4.0 * rj * rj * u2 * u2 * u2 * (1.0 / (h15 * h) + e2 * 2.5 * u2 / (h15 * h * h));
    const double dF1 = w * 2.0 * rj * u2 * u2 * (1.0 / h15 + e2 * 1.5 * u2 / (h15 * h));
    double *o = adj.tchain + (int64_t)t * 2;
    o[0] = Kp * (S[0] * dP1 + S[1] * dT1 + cp[0] * dF1) + dcy * cy * u2 / h;   // d/de2
    o[1] = S[0] * P1 + S[1] * T1 + cp[0] * F1;                                // d/dKp
  }
}

// Per-model gradients.  Block per model: sums over cells (rows), u-nodes
// (per-term chain) and pixel blocks (line-of-sight partials) in a fixed
// order, then the set-up's derivatives (App. A) to the parameters.
__global__ void __launch_bounds__(512) k_sph_grads(const GeomDev *__restrict__ geoms,
                                                   const ModelDev *__restrict__ models, int n,
                                                   ParamsDev p, const double *__restrict__ gauss,
                                                   const int *__restrict__ st_ws,
                                                   double *__restrict__ sens,
                                                   const double *__restrict__ sbp, GradsDev out) {
  constexpr int kW = 8;    // waves per block
  __shared__ double sh[4][kW];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const bool ok = st_ws[m] == 0;
    const double nan = __builtin_nan("");
    const int K = g.K, J1 = g.J1, J = J1 - 1;
    const SphAdj adj = sph_adj_of(sens, md, g);
    const double *tab = gauss + md.gauss_off;
    const double *mt = tab + 4 * K;
    const double inc = p.inc[m];
    const double si = sin(inc), ci = cos(inc);
    // dq/di of a deprojected Gaussian of observed axis ratio qo
    auto dqdi = [&](double qo, double q) { return ci * (1.0 - qo * qo) / (q * si * si * si); };
    double di = 0.0;
    // tracers: rows summed over cells (lanes split the cells, four cells'
    // loads in flight, wave sum)
    for (int k = wave; k < K; k += kW) {
      double b = 0.0, aq = 0.0, nv = 0.0;
      if (ok)
        for (int c0 = lane; c0 < kSphCells; c0 += 4 * 64) {
          double vb[4], vq[4], vn[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            vb[u] = vq[u] = vn[u] = 0.0;
            if (c0 + 64 * u < kSphCells) {
              const double *row = adj.rows + ((int64_t)k * kSphCells + c0 + 64 * u) * 3;
              vb[u] = row[0];
              vq[u] = row[1];
              vn[u] = row[2];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            b += vb[u];
            aq += vq[u];
            nv += vn[u];
          }
        }
      double sb = 0.0;
      const int n_tiles = sb_tiles(g.n_ux, g.n_uy);
      if (ok)
        for (int tl = lane; tl < n_tiles; tl += 64) sb += sbp[md.sbp_off + (int64_t)k * n_tiles + tl];
      b = wave_sum(b);
      aq = wave_sum(aq);
      nv = wave_sum(nv);
      sb = wave_sum(sb);
      if (lane == 0) {
        const double qo = g.lum_q[k], sk = g.lum_sigma[k];
        const double alpha = tab[k], q = sqrt(alpha / tab[K + k]);
        const double dq = dqdi(qo, q);
        // alphaq = alpha / q^2, nu0 = qo I0 / (sqrt(2 pi) sigma q)
        di += aq * (-2.0 * alpha / (q * q * q)) * dq + nv * (-tab[2 * K + k] / q) * dq;
        if (out.beta) out.beta[md.lum_off + k] = ok ? b : nan;
        if (out.lum_I0)
          out.lum_I0[md.lum_off + k] =
              ok ? nv * qo / (sqrt(2.0 * kPi) * sk * q) + sb : nan;
      }
    }
    // mass Gaussians and the BH: per-term chain summed over u-nodes
    const double sp = g.s_pc, Gc = grav_const();
    const double ml = p.mass_scale[m];
    double dml = 0.0;
    for (int j = wave; j < J1; j += kW) {
      double de2 = 0.0, dK = 0.0;
      if (ok)
        for (int nn = lane; nn < g.n_u; nn += 64) {
          const double *o = adj.tchain + ((int64_t)j * g.n_u + nn) * 2;
          de2 += o[0];
          dK += o[1];
        }
      de2 = wave_sum(de2);
      dK = wave_sum(dK);
      if (lane != 0) continue;
      if (j < J) {
        const double qo = g.mass_q[j], sj = g.mass_sigma[j];
        const double q = sqrt(fmax(1.0 - mt[J1 + j], 0.0));
        di += de2 * (-2.0 * q) * dqdi(qo, q);
        const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
        // K_j = sqrt(2/pi) G M_j / (s sigma_j), M_j = ml 2 pi S0_j (s sigma'_j)^2 q'_j
        const double unit = sqrt(2.0 / kPi) * Gc * 2.0 * kPi * (sp * sj) * (sp * sj) * qo / (sp * sj);
        if (out.mass_S0) out.mass_S0[md.mass_off + j] = ok ? dK * ml * unit : nan;
        dml += dK * S0 * unit;
      } else if (out.m_bh) {
        out.m_bh[m] = ok ? dK * sqrt(2.0 / kPi) * Gc / (sp * g.bh_sigma) : nan;
      }
    }
    // line-of-sight partials: i at fixed node scale, and the node scale
    // a = min_k sigma_k q_k / 4 through its minimising tracer's q_k(i)
    double li = 0.0, la = 0.0;
    const int npb = (g.n_pix + 63) / 64;
    if (ok)
      for (int b = threadIdx.x; b < npb; b += 64 * kW) {
        li += adj.losp[2 * b];
        la += adj.losp[2 * b + 1];
      }
    // fixed-order block sums: wave butterflies, then the wave partials
    di = wave_sum(di);
    dml = wave_sum(dml);
    li = wave_sum(li);
    la = wave_sum(la);
    if (lane == 0) {
      sh[0][wave] = di;
      sh[1][wave] = dml;
      sh[2][wave] = li;
      sh[3][wave] = la;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double dis = 0.0, dmls = 0.0, lis = 0.0, las = 0.0;
      for (int w = 0; w < kW; ++w) {
        dis += sh[0][w];
        dmls += sh[1][w];
        lis += sh[2][w];
        las += sh[3][w];
      }
      double smin = 1e300, dadi = 0.0;
      for (int k = 0; k < K; ++k) {
        const double sk = sqrt(0.5 / tab[k]), q = sqrt(tab[k] / tab[K + k]);
        if (sk * q < smin) {
          smin = sk * q;
          dadi = 0.25 * sk * dqdi(g.lum_q[k], q);
        }
      }
      if (out.inc) out.inc[m] = ok ? dis + lis + las * dadi : nan;
      if (out.mass_scale) out.mass_scale[m] = ok ? dmls : nan;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Radial anisotropy profile sampled per tracer Gaussian (Sect. 6):
// beta_k = beta_0 + (beta_inf - beta_0) / (1 + (r_a / sigma_k)^alpha).
// Block per model, thread per Gaussian; an invalid profile (r_a or alpha not
// positive and finite) gives NaN, which the forward's set-up reports.
// ---------------------------------------------------------------------------
__device__ inline bool logistic_ok(const double *pf) {
  return pf[2] > 0.0 && pf[3] > 0.0 && isfinite(pf[2]) && isfinite(pf[3]) && isfinite(pf[0]) &&
         isfinite(pf[1]);
}

__global__ void __launch_bounds__(256) k_beta_logistic(const GeomDev *__restrict__ geoms,
                                                       const ModelDev *__restrict__ models, int n,
                                                       const double *__restrict__ prof,
                                                       double *__restrict__ beta) {
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const double *pf = prof + 4 * (int64_t)m;
    const bool ok = logistic_ok(pf);
    for (int k = threadIdx.x; k < g.K; k += blockDim.x) {
      const double x = pow(pf[2] / g.lum_sigma[k], pf[3]);
      beta[md.lum_off + k] = ok ? pf[0] + (pf[1] - pf[0]) / (1.0 + x) : __builtin_nan("");
    }
  }
}

// grad[m][0..3] = sum_k cot_k d beta_k / d (beta_0, beta_inf, r_a, alpha); the
// sum over k runs in a fixed order (thread strides, then the block sum).
__global__ void __launch_bounds__(256) k_beta_logistic_vjp(const GeomDev *__restrict__ geoms,
                                                           const ModelDev *__restrict__ models,
                                                           int n, const double *__restrict__ prof,
                                                           const double *__restrict__ cot,
                                                           double *__restrict__ grad) {
  __shared__ double sh[256];
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const double *pf = prof + 4 * (int64_t)m;
    const bool ok = logistic_ok(pf);
    const double d = pf[1] - pf[0];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < g.K; k += blockDim.x) {
      const double lr = log(pf[2] / g.lum_sigma[k]);
      const double x = exp(pf[3] * lr), f = 1.0 / (1.0 + x);
      const double c = cot[md.lum_off + k];
      const double dfx = -f * f * x;                  // x df/dx
      a[0] += c * (1.0 - f);
      a[1] += c * f;
      a[2] += c * d * dfx * pf[3] / pf[2];
      a[3] += c * d * dfx * lr;
    }
    for (int i = 0; i < 4; ++i) {
      const double s = block_sum256(a[i], sh);
      if (threadIdx.x == 0) grad[4 * (int64_t)m + i] = ok ? s : __builtin_nan("");
      __syncthreads();
    }
  }
}

// Line-of-sight integral of the projected moment table into the unique-pixel
// N map.  Item (m, 64-pixel block), one workgroup each: four lanes per pixel
// (thread = 4 pixel + h), lane h taking nodes 16 h .. 16 h + 15, and the
// four partial sums added in a fixed order.  Nodes z' = a sinh(w), w on
// [-W, W] by the composite rule, a = min_k sigma_k q_k / 4,
// a sinh(W) = 12 max_k sigma_k; the table is interpolated bicubically
// (sph_radial_weights, sph_angular_weights), the first radius standing for
// smaller ones and zero beyond the last.  FP64.
__global__ void __launch_bounds__(256) k_sph_num(const GeomDev *__restrict__ geoms,
                                                 const ModelDev *__restrict__ models,
                                                 const Item *__restrict__ items, int n_it,
                                                 const double *__restrict__ gauss,
                                                 const int *__restrict__ st_ws,
                                                 const double *__restrict__ table,
                                                 double *__restrict__ pix) {
  const int pl = threadIdx.x / kLosLanes, h = threadIdx.x % kLosLanes;
  for (int ii = blockIdx.x; ii < n_it; ii += gridDim.x) {
    const Item it = items[ii];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int q = it.a * 64 + pl;
    const bool on = q < g.n_pix;
    double *Nout = pix + md.pix_off + q;
    if (st_ws[it.m] != 0) {                  // uniform per block
      if (on && h == 0) *Nout = 0.0;
      continue;
    }
    const int K = g.K;
    const double *tab = gauss + md.gauss_off;
    const double *mt = tab + 4 * K;
    const double si = sqrt(mt[3 * g.J1]), ci = sqrt(mt[3 * g.J1 + 1]);
    double smin = 1e300, smax = 0.0;
    for (int k = 0; k < K; ++k) {
      const double sk = sqrt(0.5 / tab[k]), qk = sqrt(tab[k] / tab[K + k]);
      smin = fmin(smin, sk * qk);
      smax = fmax(smax, sk);
    }
    const double a = 0.25 * smin, W = asinh(12.0 * smax / a);
    const double x = on ? g.xs[q % g.n_ux] : 0.0, y = on ? g.ys[q / g.n_ux] : 0.0;
    const double *T = table + md.sph_off;
    const double dth = 0.5 * kPi / (kSphNT - 1);
    const double hw = 2.0 * W / kSphSeg;
    const double *glx = geoms[md.geom].gl8_x, *glw = geoms[md.geom].gl8_w;
    double acc = 0.0;
    for (int nd = h * kLosNodes; on && nd < (h + 1) * kLosNodes; ++nd) {
      const int seg = nd >> 3, gi = nd & 7;
      const double w = -W + (seg + 0.5 + 0.5 * glx[gi]) * hw;
      // sinh w, cosh w from one exponential (|w| > 0.004 W at every node)
      const double ex = exp(w), iex = 1.0 / ex;
      const double zp = a * (0.5 * (ex - iex)), wz = 0.5 * glw[gi] * hw * a * (0.5 * (ex + iex));
      const double X = x, Y = zp * si - y * ci, Z = y * si + zp * ci;
      const double R = sqrt(X * X + Y * Y), r = sqrt(R * R + Z * Z);
      const double ct = Z / r, st = R / r;
      const double sp = R > 0.0 ? Y / R : 0.0, cp = R > 0.0 ? X / R : 0.0;
      const double xf = (log(r) - g.sph_lnr0) / g.sph_dlnr;
      if (xf > kSphNR - 1) continue;
      const double yf = acos(fmin(1.0, fabs(ct))) / dth;
      const int xi = (int)fmin(fmax(floor(xf), 0.0), (double)(kSphNR - 2));
      const int yi = (int)fmin(fmax(floor(yf), 0.0), (double)(kSphNT - 2));
      const double fx = fmin(fmax(xf - xi, 0.0), 1.0), fy = fmin(fmax(yf - yi, 0.0), 1.0);
      double ew[4], dew[4], tw[4], dtw[4];
      sph_radial_weights(xi, fx, ew, dew);
      sph_angular_weights(yi, fy, tw, dtw);
      double A[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (ew[a] == 0.0) continue;           // out of range (folded) or a zero weight
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if (tw[b] == 0.0) continue;
          const double *c = T + ((int64_t)(xi - 1 + a) * kSphNT + (yi - 1 + b)) * 3;
          const double wab = ew[a] * tw[b];
#pragma unroll
          for (int f = 0; f < 3; ++f) A[f] += wab * c[f];
        }
      }
      const double ner = si * st * sp + ci * ct;
      const double net = si * ct * sp - ci * st;
      const double nep = si * cp;
      acc += wz * (ner * ner * A[0] + net * net * A[1] + nep * nep * A[2]);
    }
    // (h0 + h1) + (h2 + h3) in every lane of the pixel
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (on && h == 0) *Nout = acc;
  }
}

inline int grid_of(int n_it) { return n_it < 1 ? 1 : n_it; }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
void launch_setup(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, double *gauss,
                  int *st_ws, int32_t *st_out, int *queues, hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(grid_of(n)), dim3(64), 0, st, g, m, n, p, gauss, st_ws, st_out,
                     queues);
}
void launch_prologue(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                     double *gauss, int *st_ws, int32_t *st_out, int *queues, float4 *terms,
                     double *pix, bool fused, hipStream_t st) {
  if (fused)
    hipLaunchKernelGGL(k_prologue<true>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p,
                       gauss, st_ws, st_out, queues, terms, pix);
  else
    hipLaunchKernelGGL(k_prologue<false>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p,
                       gauss, st_ws, st_out, queues, terms, pix);
}
void launch_sb(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
               double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_sb, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p, pix);
}
void launch_num(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                const float4 *terms, const double *gauss, const int *st_ws, double *part,
                int *queue, int grid, bool mfma, hipStream_t st) {
  if (mfma)
    hipLaunchKernelGGL(k_num_mfma, dim3(grid_of(grid)), dim3(256), 0, st, g, m, it, n_it, terms,
                       gauss, st_ws, part, queue);
  else
    hipLaunchKernelGGL(k_num_pix, dim3(grid_of(grid)), dim3(256), 0, st, g, m, it, n_it, terms,
                       st_ws, part, queue);
}
void launch_num_map(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                    const float4 *terms, const int *st_ws, double *part, int *queue, int grid,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_num_map, dim3(grid_of(grid)), dim3(kMapThreads), 0, st, g, m, it, n_it,
                     terms, st_ws, part, queue);
}
void launch_reduce_f32(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                       const double *part, double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_f32, dim3(grid_of(n_it)), dim3(512), 0, st, g, m, it, n_it, part,
                     pix);
}
void launch_reduce(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                   const double *part, double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, part, pix);
}
void launch_bins(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, int n_wave,
                 const double *pix, const int *st_ws, double *vrms2, double *binws,
                 hipStream_t st) {
  if (n_wave > 0)
    hipLaunchKernelGGL(k_bins<256>, dim3(n_wave), dim3(256), 0, st, g, m, it, n_wave, pix,
                       st_ws, vrms2, binws);
  if (n_it > n_wave)
    hipLaunchKernelGGL(k_bins<1024>, dim3(n_it - n_wave), dim3(1024), 0, st, g, m, it + n_wave,
                       n_it - n_wave, pix, st_ws, vrms2, binws);
}
void launch_maps(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                 const double *pix, const int *st_ws, double *N_map, double *I_map,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_maps, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, pix, st_ws,
                     N_map, I_map);
}
void launch_bins_adjoint(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                         const double *vrms2, const double *cot, const double *binws,
                         const int *st_ws, double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_bins_adjoint, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, vrms2,
                     cot, binws, st_ws, pix);
}
void launch_sens(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                 const float4 *terms, const double *pix, const int *st_ws, double *sens,
                 int *queue, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_sens, dim3(grid_of(grid)), dim3(256), 0, st, g, m, it, n_it, terms, pix,
                     st_ws, sens, queue);
}
void launch_sens_wide(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                      const float4 *terms, const double *pix, const int *st_ws, double *sens,
                      int *queue, int grid, hipStream_t st) {
  hipLaunchKernelGGL(k_sens_wide, dim3(grid_of(grid)), dim3(64 * kWideWaves), 0, st, g, m, it,
                     n_it, terms, pix, st_ws, sens, queue);
}
int occupancy_num(bool mfma) {
  int nb = 0;
  const hipError_t e = mfma ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_num_mfma, 256, 0)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_num_pix, 256, 0);
  if (e != hipSuccess) nb = 1;
  return nb < 1 ? 1 : nb;
}
int occupancy_sens() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sens, 256, 0) != hipSuccess) nb = 1;
  return nb < 1 ? 1 : nb;
}
void launch_adj_small(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                      const double *pix, const int *st_ws, double *sens, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_small, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p, pix,
                     st_ws, sens);
}
void launch_chain(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                  double *sens, const int *st_ws, hipStream_t st) {
  hipLaunchKernelGGL(k_chain, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p, sens, st_ws);
}
void launch_grads(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, double *sens,
                  const double *sbp, const int *st_ws, GradsDev out, hipStream_t st) {
  hipLaunchKernelGGL(k_grads, dim3(grid_of(n)), dim3(1024), 0, st, g, m, n, p, sens, sbp, st_ws,
                     out);
}
void launch_sb_adjoint(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                       const int *st_ws, const double *pix, double *sbp, hipStream_t st) {
  hipLaunchKernelGGL(k_sb_adj, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, st_ws, pix,
                     sbp);
}
void launch_sph_terms(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                      const double *gauss, const int *st_ws, float4 *terms, hipStream_t st) {
  hipLaunchKernelGGL(k_sph_terms, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, gauss,
                     st_ws, terms);
}
void launch_sph_moments(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                        const double *gauss, const float4 *terms, const int *st_ws,
                        const float *sgrid, double *table, hipStream_t st) {
  if (sgrid)
    hipLaunchKernelGGL(k_sph_moments<true>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it,
                       gauss, terms, st_ws, sgrid, table);
  else
    hipLaunchKernelGGL(k_sph_moments<false>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it,
                       n_it, gauss, terms, st_ws, sgrid, table);
}
void launch_sph_grid(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                     const double *gauss, const float4 *terms, const int *st_ws, float *sgrid,
                     bool adjoint, hipStream_t st) {
  if (adjoint)
    hipLaunchKernelGGL(k_sph_grid<6>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, gauss,
                       terms, st_ws, sgrid);
  else
    hipLaunchKernelGGL(k_sph_grid<2>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, gauss,
                       terms, st_ws, sgrid);
}
void launch_sph_grid_reduce(const ModelDev *m, const Item *it, int n_it, const int *st_ws,
                            float *sgrid, bool adjoint, hipStream_t st) {
  hipLaunchKernelGGL(k_sph_grid_reduce, dim3(grid_of(n_it)), dim3(256), 0, st, m, it, n_it, st_ws,
                     sgrid, adjoint ? 1 : 0);
}
void launch_sph_moments_jac(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                            const double *gauss, const float4 *terms, const int *st_ws,
                            const float *sgrid6, double *table, double *sens, hipStream_t st) {
  if (sgrid6)
    hipLaunchKernelGGL(k_sph_moments_jac<true>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it,
                       n_it, gauss, terms, st_ws, sgrid6, table, sens);
  else
    hipLaunchKernelGGL(k_sph_moments_jac<false>, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it,
                       n_it, gauss, terms, st_ws, sgrid6, table, sens);
}
void launch_sph_num(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                    const double *gauss, const int *st_ws, const double *table, double *pix,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_sph_num, dim3(grid_of(n_it)), dim3(64 * kLosLanes), 0, st, g, m, it, n_it,
                     gauss, st_ws, table, pix);
}
void launch_sph_adjoint(const GeomDev *g, const ModelDev *m, int n, const Item *it_los,
                        int n_los, const Item *it_cell, int n_cell, const Item *it_sens,
                        int n_sens, const Item *it_tile, int n_tile, const Item *it_pcot,
                        int n_pcot, const Item *it_pfix, int n_pfix, const Item *it_sgs,
                        int n_sgs, ParamsDev p, const double *gauss, const float4 *terms,
                        const int *st_ws, const double *table, const double *pix,
                        const double *sbp, double *sens, double *sgcot, GradsDev out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_sph_zero, dim3(grid_of(n)), dim3(kZeroThreads), 0, st, g, m, n, gauss,
                     st_ws, pix, sens);
  hipLaunchKernelGGL(k_sph_num_adj, dim3(grid_of(n_los)), dim3(256), 0, st, g, m, it_los, n_los,
                     gauss, st_ws, table, pix, sens);
  hipLaunchKernelGGL(k_sph_dtab_fix, dim3(grid_of(n)), dim3(256), 0, st, g, m, n, st_ws, sens);
  hipLaunchKernelGGL(k_sph_rows, dim3(grid_of(n_cell)), dim3(64), 0, st, g, m, it_cell, n_cell,
                     gauss, st_ws, sens);
  if (sgcot) {
    hipLaunchKernelGGL(k_sph_pcot_bound, dim3(grid_of(n_pcot)), dim3(256), 0, st, g, m, it_pcot,
                       n_pcot, gauss, st_ws, sens, sgcot);
    hipLaunchKernelGGL(k_sph_pcot_scan, dim3(grid_of(n)), dim3(kSphTiles * kScanParts), 0, st, g,
                       m, n, st_ws, sgcot);
    hipLaunchKernelGGL(k_sph_pcot_fill, dim3(grid_of(n_pcot)), dim3(256), 0, st, g, m, it_pcot,
                       n_pcot, gauss, st_ws, sgcot);
    hipLaunchKernelGGL(k_sph_pcot_tiles, dim3(grid_of(n_pcot * kTileSub)), dim3(256), 0, st, g, m,
                       it_pcot, n_pcot, gauss, st_ws, sens, sgcot);
    hipLaunchKernelGGL(k_sph_pcot_fix, dim3(grid_of(n_pfix)), dim3(256), 0, st, g, m, it_pfix,
                       n_pfix, st_ws, sgcot);
    hipLaunchKernelGGL(k_sph_sens_grid, dim3(grid_of(n_sgs)), dim3(256), 0, st, g, m, it_sgs,
                       n_sgs, gauss, terms, st_ws, sens, sgcot);
  } else {
    hipLaunchKernelGGL(k_sph_sens, dim3(grid_of(n_sens)), dim3(256), 0, st, g, m, it_sens, n_sens,
                       gauss, terms, st_ws, sens);
  }
  hipLaunchKernelGGL(k_sph_sens_cells, dim3(grid_of(n_tile * kSphCellParts)), dim3(256), 0, st, g,
                     m, it_tile, n_tile, gauss, terms, st_ws, sens);
  hipLaunchKernelGGL(k_sph_chain, dim3(grid_of(n_tile)), dim3(256), 0, st, g, m, it_tile, n_tile,
                     gauss, st_ws, sens);
  hipLaunchKernelGGL(k_sph_grads, dim3(grid_of(n)), dim3(512), 0, st, g, m, n, p, gauss, st_ws,
                     sens, sbp, out);
}
void launch_beta_logistic(const GeomDev *g, const ModelDev *m, int n, const double *prof,
                          double *beta, hipStream_t st) {
  hipLaunchKernelGGL(k_beta_logistic, dim3(grid_of(n)), dim3(256), 0, st, g, m, n, prof, beta);
}
void launch_beta_logistic_vjp(const GeomDev *g, const ModelDev *m, int n, const double *prof,
                              const double *cot, double *grad, hipStream_t st) {
  hipLaunchKernelGGL(k_beta_logistic_vjp, dim3(grid_of(n)), dim3(256), 0, st, g, m, n, prof, cot,
                     grad);
}
void launch_mge1d(int n_prof, int n_comp, const double *comp, const MgeConst &k, double *amp,
                  hipStream_t st) {
  const int64_t n = (int64_t)n_prof * k.n_sigma;
  hipLaunchKernelGGL(k_mge1d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_prof, n_comp,
                     comp, k, amp);
}
void launch_mge1d_vjp(int n_prof, int n_comp, const double *comp, const MgeConst &k,
                      const double *cot, double *grad, hipStream_t st) {
  const int64_t n = (int64_t)n_prof * n_comp;
  hipLaunchKernelGGL(k_mge1d_vjp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n_prof,
                     n_comp, comp, k, cot, grad);
}
void launch_chi2(const GeomDev *g, const ModelDev *m, int n, const KinDev *kin, const double *V,
                 const int *st_ws, double *chi2, const double *cot, double *dV, hipStream_t st) {
  hipLaunchKernelGGL(k_chi2, dim3(grid_of(std::min(n, 65536))), dim3(256), 0, st, g, m, n, kin, V,
                     st_ws, chi2, cot, dV);
}

}  // namespace jam
