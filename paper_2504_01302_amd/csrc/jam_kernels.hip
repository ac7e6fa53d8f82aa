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
#include <cmath>

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

// ---------------------------------------------------------------------------
// Set-up: App. A deprojection and per-Gaussian derived quantities (FP64),
// per-model validity.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_setup(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models, int n,
                                              ParamsDev p, double *__restrict__ gauss,
                                              int *__restrict__ st_ws, int32_t *__restrict__ st_out) {
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
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
}

// ---------------------------------------------------------------------------
// Term table: FP64 coefficients of every (k, j, n) term, stored as FP32
// (-c1 log2e, -gamma log2e, C0, C1).  Term t = (k * J1 + j) * n_u + n.
// ---------------------------------------------------------------------------
__device__ inline void term_fp64(const double *tab, int K, int J1, int k, int j, double u,
                                 double wq, double &c1, double &gam, double &C0, double &C1) {
  const double alpha = tab[k], alphaq = tab[K + k], nu0 = tab[2 * K + k], b = tab[3 * K + k];
  const double *mt = tab + 4 * K;
  const double r = mt[j], e2 = mt[J1 + j], Kp = mt[2 * J1 + j];
  const double si2 = mt[3 * J1], ci2 = mt[3 * J1 + 1];
  const double u2 = u * u;
  const double h = 1.0 - e2 * u2;
  c1 = alpha + r * u2;
  const double A = alphaq + r * u2 / h;
  const double a = c1 * si2 + A * ci2;
  gam = c1 * A / a;
  const double base = nu0 * Kp * r * u2;
  const double sh = sqrt(h);
  const double gg = base / (A * h * sh);
  const double ww = 2.0 * base / sh;
  const double P = (ci2 + b * si2) * gg;
  const double Q = si2 * (ww - 2.0 * c1 * b * gg);
  const double f = wq * sqrt(kPi / a);
  C0 = f * P;
  C1 = f * Q;
}

__global__ void __launch_bounds__(256) k_terms(const GeomDev *__restrict__ geoms,
                                               const ModelDev *__restrict__ models,
                                               const Item *__restrict__ items, int n_it,
                                               const double *__restrict__ gauss,
                                               const int *__restrict__ st_ws,
                                               float4 *__restrict__ terms) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int t = it.a * 256 + threadIdx.x;
    if (t >= g.T) continue;
    float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
    if (st_ws[it.m] == 0) {
      const int n = t % g.n_u;
      const int kj = t / g.n_u;
      const int j = kj % g.J1, k = kj / g.J1;
      double c1, gam, C0, C1;
      term_fp64(gauss + md.gauss_off, g.K, g.J1, k, j, g.u[n], g.w[n], c1, gam, C0, C1);
      out = make_float4((float)(-c1 * kLog2e), (float)(-gam * kLog2e), (float)C0, (float)C1);
    }
    terms[md.term_off + t] = out;
  }
}

// ---------------------------------------------------------------------------
// Surface brightness, eq. (sb_mge_2D), FP64, on the unique-pixel map.
// pix region per model: [N | I | lambda_N | lambda_I], n_pix doubles each.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_sb(const GeomDev *__restrict__ geoms,
                                            const ModelDev *__restrict__ models,
                                            const Item *__restrict__ items, int n_it, ParamsDev p,
                                            double *__restrict__ pix) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int q = it.a * 256 + threadIdx.x;
    if (q >= g.n_pix) continue;
    const double x = g.xs[q % g.n_ux], y = g.ys[q / g.n_ux];
    double acc = 0.0;
    for (int k = 0; k < g.K; ++k) {
      const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
      const double qo = g.lum_q[k], sig = g.lum_sigma[k];
      acc += I0 * exp(-(x * x + y * y / (qo * qo)) / (2.0 * sig * sig));
    }
    pix[md.pix_off + g.n_pix + q] = acc;
  }
}

// ---------------------------------------------------------------------------
// Per-pixel VALU quadrature.  Item (m, 64-pixel block, slice); the slice is a
// range of (k, j) pairs, split over the 4 waves; lanes are unique pixels and
// the term coefficients are wave-uniform (scalar loads).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_num_pix(const GeomDev *__restrict__ geoms,
                                                 const ModelDev *__restrict__ models,
                                                 const Item *__restrict__ items, int n_it,
                                                 const float4 *__restrict__ terms,
                                                 const int *__restrict__ st_ws,
                                                 double *__restrict__ part) {
  __shared__ double red[256];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int q = it.a * 64 + lane;
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
    double acc = 0.0;
    if (st_ws[it.m] == 0) {
      const float4 *tb = terms + md.term_off;
      const int nu = g.n_u;
      for (int pr = p0 + wave; pr < p1; pr += 4) {
        const float4 *tp = tb + (int64_t)pr * nu;
        float s = 0.f;
        for (int n = 0; n < nu; ++n) {
          const float4 c = tp[n];
          const float e = fast_exp2(fmaf(c.x, x2, c.y * y2));
          s = fmaf(e, fmaf(c.w, x2, c.z), s);
        }
        acc += (double)s;
      }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && valid) {
      const double v = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
      part[md.part_off + (int64_t)it.b * g.n_pix + q] = v;
    }
    __syncthreads();
  }
}

// Sum the split-term partials in a fixed order into the N map.
__global__ void __launch_bounds__(256) k_reduce(const GeomDev *__restrict__ geoms,
                                                const ModelDev *__restrict__ models,
                                                const Item *__restrict__ items, int n_it,
                                                const double *__restrict__ part,
                                                double *__restrict__ pix) {
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int q = it.a * 256 + threadIdx.x;
    if (q >= g.n_pix) continue;
    double acc = 0.0;
    for (int s = 0; s < md.n_slices; ++s) acc += part[md.part_off + (int64_t)s * g.n_pix + q];
    pix[md.pix_off + q] = acc;
  }
}

// ---------------------------------------------------------------------------
// Bins: sums of the PSF-weighted maps per bin and their FP64 ratio.
// Item (m, bin).  binws per model: [Nb | Ib], n_bins doubles each.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bins(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models,
                                              const Item *__restrict__ items, int n_it,
                                              const double *__restrict__ pix,
                                              const int *__restrict__ st_ws,
                                              double *__restrict__ vrms2,
                                              double *__restrict__ binws) {
  __shared__ double sh[256];
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int b = it.a;
    const double *Nm = pix + md.pix_off;
    const double *Im = Nm + g.n_pix;
    const bool want_n = vrms2 != nullptr;
    double an = 0.0, ai = 0.0;
    for (int e = g.bin_ptr[b] + threadIdx.x; e < g.bin_ptr[b + 1]; e += 256) {
      const double wv = g.bin_w[e];
      const int q = g.bin_pix[e];
      if (want_n) an += wv * Nm[q];
      ai += wv * Im[q];
    }
    const double sn = want_n ? block_sum256(an, sh) : 0.0;
    const double si = block_sum256(ai, sh);
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
__global__ void __launch_bounds__(256) k_sens_pix(const GeomDev *__restrict__ geoms,
                                                  const ModelDev *__restrict__ models,
                                                  const Item *__restrict__ items, int n_it,
                                                  const float4 *__restrict__ terms,
                                                  const double *__restrict__ pix,
                                                  const int *__restrict__ st_ws,
                                                  double *__restrict__ sens) {
  __shared__ float sx[256], sy[256], sl[256];
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    if (st_ws[it.m] != 0) continue;   // uniform per block
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
}

// ---------------------------------------------------------------------------
// FP64 chain from per-term sensitivities to the parameters.  Forward-mode
// dual numbers carry d/d(inclination) through the deprojection and the term
// coefficients.  Item (m, k): all terms of luminous Gaussian k.
// chain per model: [K][3 + J1] doubles: d/di, d/dbeta_k, d/dI0_k (N and I
// paths), then d/dM_j (j < J1, BH last) partial sums over k.
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
__device__ inline dual operator+(double s, dual a) { return {s + a.v, a.d}; }
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

__global__ void __launch_bounds__(256) k_chain(const GeomDev *__restrict__ geoms,
                                               const ModelDev *__restrict__ models,
                                               const Item *__restrict__ items, int n_it,
                                               ParamsDev p, const double *__restrict__ pix,
                                               const double *__restrict__ sens,
                                               const int *__restrict__ st_ws,
                                               double *__restrict__ chain) {
  // chain rows live in the sens region after the three sensitivity arrays:
  // per model [K][3 + J1] doubles at sens_off + 3 T.
  __shared__ double sh[256];
  __shared__ double shj[4][2];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n_it; i += gridDim.x) {
    const Item it = items[i];
    const ModelDev md = models[it.m];
    const GeomDev g = geoms[md.geom];
    const int k = it.a;
    const int J1 = g.J1, J = J1 - 1;
    double *row = chain + md.sens_off + 3 * (int64_t)g.T + (int64_t)k * (3 + J1);
    if (st_ws[it.m] != 0) {
      for (int c = threadIdx.x; c < 3 + J1; c += 256) row[c] = __builtin_nan("");
      continue;
    }
    const double inc = p.inc[it.m];
    const dual s = {sin(inc), cos(inc)};
    const dual c = {cos(inc), -sin(inc)};
    const dual si2 = s * s, ci2 = c * c;
    const double G = grav_const();
    const double sp = g.s_pc;
    // luminous Gaussian k
    const double qok = g.lum_q[k], sk = g.lum_sigma[k];
    const double I0 = p.lum_I0 ? p.lum_I0[md.lum_off + k] : g.lum_I0[k];
    const double beta = p.beta[md.lum_off + k];
    const double b = 1.0 / (1.0 - beta);
    const dual qk = dsqrt(qok * qok - ci2) / s;
    const double alpha = 0.5 / (sk * sk);
    const dual alphaq = dconst(alpha) / (qk * qk);
    const dual nu1 = dconst(qok / (sqrt(2.0 * kPi) * sk)) / qk;   // nu0 / I0
    const double *S0a = sens + md.sens_off;
    const double *S1a = S0a + g.T;
    const double *Sga = S1a + g.T;
    double acc_i = 0.0, acc_b = 0.0, acc_I = 0.0;
    for (int j0 = 0; j0 < J1; j0 += 4) {
      const int j = j0 + wave;
      double hj = 0.0;
      double Mj = 0.0;
      if (j < J1) {
        dual e2;
        double r, Kt;
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
        for (int n = lane; n < g.n_u; n += 64) {
          const int64_t t = ((int64_t)k * J1 + j) * g.n_u + n;
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
          const double S0 = S0a[t], S1 = S1a[t], Sg = Sga[t];
          const double amp = I0 * Mj;
          acc_i += amp * (S0 * c0.d + S1 * c1u.d) - Sg * gam.d;
          // dC0/db = f si2 g, dC1/db = -2 f si2 c1 g
          acc_b += amp * f.v * si2.v * gg.v * (S0 - 2.0 * c1 * S1);
          hj += S0 * c0.v + S1 * c1u.v;
        }
      }
      hj = wave_sum(hj);
      if (lane == 0) {
        shj[wave][0] = hj;
        shj[wave][1] = Mj;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int w4 = 0; w4 < 4; ++w4) {
          const int jj = j0 + w4;
          if (jj < J1) {
            row[3 + jj] = I0 * shj[w4][0];     // d/dM_j
            acc_I += shj[w4][1] * shj[w4][0];  // d/dI0_k, N path
          }
        }
      }
      __syncthreads();
    }
    // I path: d/dI0_k += sum_p lambda_I[p] exp(-(x^2 + y^2/q'^2)/(2 sigma'^2))
    const double *lamI = pix + md.pix_off + 3 * (int64_t)g.n_pix;
    double acc_l = 0.0;
    for (int q = threadIdx.x; q < g.n_pix; q += 256) {
      const double x = g.xs[q % g.n_ux], y = g.ys[q / g.n_ux];
      acc_l += lamI[q] * exp(-(x * x + y * y / (qok * qok)) / (2.0 * sk * sk));
    }
    const double ti = block_sum256(acc_i, sh);
    const double tb = block_sum256(acc_b, sh);
    const double tl = block_sum256(acc_l, sh);
    if (threadIdx.x == 0) {
      row[0] = ti;
      row[1] = tb * b * b;           // db/dbeta = b^2
      row[2] = acc_I + tl;
    }
    __syncthreads();
  }
}

// Final per-model gradients from the per-k chain rows.  One block per model.
__global__ void __launch_bounds__(64) k_grads(const GeomDev *__restrict__ geoms,
                                              const ModelDev *__restrict__ models, int n,
                                              ParamsDev p, const double *__restrict__ sens,
                                              const int *__restrict__ st_ws, GradsDev out) {
  for (int m = blockIdx.x; m < n; m += gridDim.x) {
    const ModelDev md = models[m];
    const GeomDev g = geoms[md.geom];
    const int K = g.K, J1 = g.J1, J = J1 - 1;
    const double *cm = sens + md.sens_off + 3 * (int64_t)g.T;
    const bool ok = st_ws[m] == 0;
    const double nan = __builtin_nan("");
    const double sp = g.s_pc;
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
      const double *row = cm + (int64_t)k * (3 + J1);
      if (out.beta) out.beta[md.lum_off + k] = ok ? row[1] : nan;
      if (out.lum_I0) out.lum_I0[md.lum_off + k] = ok ? row[2] : nan;
    }
    double dml = 0.0;
    for (int j = threadIdx.x; j < J1; j += blockDim.x) {
      double dM = 0.0;
      for (int k = 0; k < K; ++k) dM += cm[(int64_t)k * (3 + J1) + 3 + j];
      if (j < J) {
        const double qo = g.mass_q[j], sj = g.mass_sigma[j];
        const double S0 = p.mass_S0 ? p.mass_S0[md.mass_off + j] : g.mass_S0[j];
        const double unit = 2.0 * kPi * (sp * sj) * (sp * sj) * qo;   // dM/d(ml S0)
        if (out.mass_S0) out.mass_S0[md.mass_off + j] = ok ? dM * p.mass_scale[m] * unit : nan;
        dml += dM * S0 * unit;
      } else {
        if (out.m_bh) out.m_bh[m] = ok ? dM : nan;
      }
    }
    dml = wave_sum(dml);
    if (threadIdx.x == 0) {
      double di = 0.0;
      for (int k = 0; k < K; ++k) di += cm[(int64_t)k * (3 + J1)];
      if (out.inc) out.inc[m] = ok ? di : nan;
      if (out.mass_scale) out.mass_scale[m] = ok ? dml : nan;
    }
  }
}

inline int grid_of(int n_it) { return n_it < 1 ? 1 : n_it; }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
void launch_setup(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, double *gauss,
                  int *st_ws, int32_t *st_out, hipStream_t st) {
  hipLaunchKernelGGL(k_setup, dim3(grid_of(n)), dim3(64), 0, st, g, m, n, p, gauss, st_ws, st_out);
}
void launch_terms(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                  const double *gauss, const int *st_ws, float4 *terms, hipStream_t st) {
  hipLaunchKernelGGL(k_terms, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, gauss, st_ws,
                     terms);
}
void launch_sb(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
               double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_sb, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p, pix);
}
void launch_num_pix(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                    const float4 *terms, const int *st_ws, double *part, hipStream_t st) {
  hipLaunchKernelGGL(k_num_pix, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, terms,
                     st_ws, part);
}
void launch_reduce(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                   const double *part, double *pix, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, part, pix);
}
void launch_bins(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                 const double *pix, const int *st_ws, double *vrms2, double *binws,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_bins, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, pix, st_ws,
                     vrms2, binws);
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
void launch_sens_pix(const GeomDev *g, const ModelDev *m, const Item *it, int n_it,
                     const float4 *terms, const double *pix, const int *st_ws, double *sens,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_sens_pix, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, terms,
                     pix, st_ws, sens);
}
void launch_chain(const GeomDev *g, const ModelDev *m, const Item *it, int n_it, ParamsDev p,
                  const double *pix, double *sens, const int *st_ws, hipStream_t st) {
  hipLaunchKernelGGL(k_chain, dim3(grid_of(n_it)), dim3(256), 0, st, g, m, it, n_it, p, pix, sens,
                     st_ws, sens);
}
void launch_grads(const GeomDev *g, const ModelDev *m, int n, ParamsDev p, const double *sens,
                  const int *st_ws, GradsDev out, hipStream_t st) {
  hipLaunchKernelGGL(k_grads, dim3(grid_of(n)), dim3(64), 0, st, g, m, n, p, sens, st_ws, out);
}

}  // namespace jam
