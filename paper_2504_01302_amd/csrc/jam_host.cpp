// Host runtime of the JAM-cyl library: the C ABI of include/jam.h.
//
// Responsibilities: validate inputs, build the device description of every
// geometry once (distinct |x'|/|y'| values of the padded sub-pixel grid, the
// PSF-and-bin weight matrix in both orientations, Gauss-Legendre nodes),
// build per-composition work lists ("plans") once, size the caller's
// workspace, and sequence the kernels on the caller's stream.
#include "jam.h"
#include "jam_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <list>
#include <queue>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_err;

jam_status fail(jam_status s, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) return fail(JAM_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr int kMaxNu = 1024;
constexpr double kPi = 3.14159265358979323846;

// n-node Gauss-Legendre rule on [0, 1]: Newton iteration on P_n from the
// asymptotic initial guess, in long double; nodes ascending.
void gauss_legendre01(int n, double *x, double *w) {
  for (int i = 0; i < n; ++i) {
    long double z = std::cos(kPi * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0L; }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      const long double dz = p1 / dp;
      z -= dz;
      if (std::fabs((double)dz) < 1e-19) break;
    }
    // recompute the derivative at the converged node
    long double p0 = 1.0L, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const long double p2 = ((2.0L * k - 1.0L) * z * p1 - (k - 1.0L) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = (n == 1) ? 1.0L : n * (z * p1 - p0) / (z * z - 1.0L);
    const long double wi = 2.0L / ((1.0L - z * z) * dp * dp);
    // z runs from +1 downwards; store ascending on [0, 1]
    x[i] = (double)(0.5L * (1.0L - z));
    w[i] = (double)(0.5L * wi);
  }
}

// Everything the library keeps about one geometry on the host.
struct GeomHost {
  int K = 0, J = 0, J1 = 0, n_u = 0, T = 0;
  int nx = 0, ny = 0, ss = 1, psf_n = 1, h = 0, n_bins = 0;
  int nxp = 0, nyp = 0, n_ux = 0, n_uy = 0, n_pix = 0;
  double bh_sigma = 0, dist = 0, pixsize = 0, xc = 0, yc = 0, s_pc = 0;
  std::vector<double> lum_sigma, lum_q, lum_I0, mass_sigma, mass_q, mass_S0;
  std::vector<double> u, w, xs, ys;
  std::vector<int> ux, uy;
  std::vector<int> bin_ptr, bin_pix, pix_ptr, pix_bin;
  std::vector<double> bin_w, pix_w;
  int max_bin_nnz = 0;   // largest number of weights of one bin
  // spherically aligned model: polar table radii and the 8-node rule
  double sph_lnr0 = 0, sph_dlnr = 0, sph_sig_max = 0;
  double gl8_x[8] = {}, gl8_w[8] = {};
};

jam_status validate(const jam_geometry &g, int gi) {
  auto bad = [&](const char *what) {
    return fail(JAM_E_INVALID_ARG, "geometry %d: %s", gi, what);
  };
  if (g.n_lum < 1) return bad("n_lum must be >= 1");
  if (g.n_mass < 0) return bad("n_mass must be >= 0");
  if (!g.lum_sigma || !g.lum_q || !g.lum_I0) return bad("luminous MGE arrays are NULL");
  if (g.n_mass > 0 && (!g.mass_sigma || !g.mass_q || !g.mass_S0))
    return bad("mass MGE arrays are NULL");
  for (int k = 0; k < g.n_lum; ++k) {
    if (!(g.lum_sigma[k] > 0) || !std::isfinite(g.lum_sigma[k])) return bad("lum_sigma must be > 0");
    if (!(g.lum_q[k] > 0 && g.lum_q[k] <= 1)) return bad("lum_q must be in (0, 1]");
    if (!(g.lum_I0[k] >= 0) || !std::isfinite(g.lum_I0[k])) return bad("lum_I0 must be >= 0");
  }
  for (int j = 0; j < g.n_mass; ++j) {
    if (!(g.mass_sigma[j] > 0) || !std::isfinite(g.mass_sigma[j])) return bad("mass_sigma must be > 0");
    if (!(g.mass_q[j] > 0 && g.mass_q[j] <= 1)) return bad("mass_q must be in (0, 1]");
    if (!(g.mass_S0[j] >= 0) || !std::isfinite(g.mass_S0[j])) return bad("mass_S0 must be >= 0");
  }
  if (!(g.bh_sigma > 0) || !std::isfinite(g.bh_sigma)) return bad("bh_sigma must be > 0");
  if (!(g.distance_mpc > 0) || !std::isfinite(g.distance_mpc)) return bad("distance_mpc must be > 0");
  if (g.nx < 1 || g.ny < 1) return bad("nx, ny must be >= 1");
  if (!(g.pixsize > 0) || !std::isfinite(g.pixsize)) return bad("pixsize must be > 0");
  if (!std::isfinite(g.xc) || !std::isfinite(g.yc)) return bad("xc, yc must be finite");
  if (g.supersample < 1 || g.supersample > 16) return bad("supersample must be in [1, 16]");
  if (g.psf_n < 1 || g.psf_n % 2 == 0) return bad("psf_n must be odd and >= 1");
  if (!g.psf) return bad("psf is NULL");
  for (int i = 0; i < g.psf_n * g.psf_n; ++i)
    if (!std::isfinite(g.psf[i])) return bad("psf must be finite");
  if (g.n_bins < 1) return bad("n_bins must be >= 1");
  if (!g.bin_index) return bad("bin_index is NULL");
  if (g.n_u < 1 || g.n_u > kMaxNu) return bad("n_u must be in [1, 1024]");
  const int64_t nsub_x = (int64_t)g.nx * g.supersample + g.psf_n - 1;
  const int64_t nsub_y = (int64_t)g.ny * g.supersample + g.psf_n - 1;
  if (nsub_x > 16384 || nsub_y > 16384) return bad("padded sub-pixel grid larger than 16384");
  // term counts and the weight matrix's nonzeros are indexed with 32-bit
  // integers on the device
  const int64_t T = (int64_t)g.n_lum * (g.n_mass + 1) * g.n_u;
  const int64_t T_sph = ((int64_t)(g.n_mass + 1) * g.n_u + 63) / 64 * 64;
  if (T > INT32_MAX || T_sph > INT32_MAX)
    return fail(JAM_E_UNSUPPORTED, "geometry %d: %lld terms exceed the supported 2^31 - 1", gi,
                (long long)std::max(T, T_sph));
  const int64_t nnz_max = (int64_t)g.nx * g.supersample * g.ny * g.supersample * g.psf_n * g.psf_n;
  if (nnz_max > INT32_MAX)
    return fail(JAM_E_UNSUPPORTED, "geometry %d: field sub-pixels x PSF taps exceed 2^31 - 1", gi);
  std::vector<int> cnt(g.n_bins, 0);
  for (int64_t i = 0; i < (int64_t)g.nx * g.ny; ++i) {
    const int b = g.bin_index[i];
    if (b < -1 || b >= g.n_bins) return bad("bin_index out of range");
    if (b >= 0) cnt[b]++;
  }
  for (int b = 0; b < g.n_bins; ++b)
    if (cnt[b] == 0) return fail(JAM_E_INVALID_ARG, "geometry %d: bin %d is empty", gi, b);
  return JAM_OK;
}

// Distinct |v| of a list, ascending, with the index map.
void distinct_abs(const std::vector<double> &v, std::vector<double> &vals, std::vector<int> &map) {
  vals.clear();
  for (double x : v) vals.push_back(std::fabs(x));
  std::sort(vals.begin(), vals.end());
  vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
  map.resize(v.size());
  for (size_t i = 0; i < v.size(); ++i)
    map[i] = (int)(std::lower_bound(vals.begin(), vals.end(), std::fabs(v[i])) - vals.begin());
}

void build_geometry(const jam_geometry &g, GeomHost &o) {
  o.K = g.n_lum;
  o.J = g.n_mass;
  o.J1 = g.n_mass + 1;
  o.n_u = g.n_u;
  o.T = o.K * o.J1 * o.n_u;
  o.nx = g.nx;
  o.ny = g.ny;
  o.ss = g.supersample;
  o.psf_n = g.psf_n;
  o.h = (g.psf_n - 1) / 2;
  o.n_bins = g.n_bins;
  o.bh_sigma = g.bh_sigma;
  o.dist = g.distance_mpc;
  o.pixsize = g.pixsize;
  o.xc = g.xc;
  o.yc = g.yc;
  o.s_pc = g.distance_mpc * 1.0e6 * kPi / 648000.0;
  o.lum_sigma.assign(g.lum_sigma, g.lum_sigma + o.K);
  o.lum_q.assign(g.lum_q, g.lum_q + o.K);
  o.lum_I0.assign(g.lum_I0, g.lum_I0 + o.K);
  if (o.J) {
    o.mass_sigma.assign(g.mass_sigma, g.mass_sigma + o.J);
    o.mass_q.assign(g.mass_q, g.mass_q + o.J);
    o.mass_S0.assign(g.mass_S0, g.mass_S0 + o.J);
  }
  o.u.resize(o.n_u);
  o.w.resize(o.n_u);
  gauss_legendre01(o.n_u, o.u.data(), o.w.data());

  // padded sub-pixel centres (galaxy at the origin)
  const int ssx = o.nx * o.ss, ssy = o.ny * o.ss;
  o.nxp = ssx + 2 * o.h;
  o.nyp = ssy + 2 * o.h;
  const double pitch = o.pixsize / o.ss;
  std::vector<double> xp(o.nxp), yp(o.nyp);
  for (int c = 0; c < o.nxp; ++c) xp[c] = o.xc + ((double)(c - o.h) - (ssx - 1) / 2.0) * pitch;
  for (int r = 0; r < o.nyp; ++r) yp[r] = o.yc + ((double)(r - o.h) - (ssy - 1) / 2.0) * pitch;
  distinct_abs(xp, o.xs, o.ux);
  distinct_abs(yp, o.ys, o.uy);
  o.n_ux = (int)o.xs.size();
  o.n_uy = (int)o.ys.size();
  o.n_pix = o.n_ux * o.n_uy;

  // W[b, p]: the convolved map at field sub-pixel f is
  //   C(f) = sum_o psf[o + h] M(f - o),
  // so bin b's sum of C weights padded sub-pixel (f + h - o) by psf[o + h].
  // Built one bin at a time in a dense scratch row (memory O(n_pix + nnz));
  // each weight accumulates its field sub-pixels in raster order.
  std::vector<std::vector<int>> fields(o.n_bins);
  for (int fy = 0; fy < ssy; ++fy)
    for (int fx = 0; fx < ssx; ++fx) {
      const int b = g.bin_index[(fy / o.ss) * o.nx + fx / o.ss];
      if (b >= 0) fields[b].push_back(fy * ssx + fx);
    }
  const int n = o.psf_n;
  std::vector<double> row(o.n_pix, 0.0);
  std::vector<char> hit(o.n_pix, 0);
  std::vector<int> touched;
  o.bin_ptr.assign(o.n_bins + 1, 0);
  std::vector<int> pcount(o.n_pix, 0);
  o.max_bin_nnz = 0;
  for (int b = 0; b < o.n_bins; ++b) {
    touched.clear();
    for (int f : fields[b]) {
      const int fy = f / ssx, fx = f % ssx;
      for (int oy = -o.h; oy <= o.h; ++oy) {
        const int iy = o.uy[fy + o.h - oy] * o.n_ux;
        const double *kr = g.psf + (oy + o.h) * n;
        for (int ox = -o.h; ox <= o.h; ++ox) {
          const int q = iy + o.ux[fx + o.h - ox];
          if (!hit[q]) {
            hit[q] = 1;
            touched.push_back(q);
          }
          row[q] += kr[ox + o.h];
        }
      }
    }
    std::sort(touched.begin(), touched.end());
    for (int q : touched) {
      if (row[q] != 0.0) {
        o.bin_pix.push_back(q);
        o.bin_w.push_back(row[q]);
        pcount[q]++;
      }
      row[q] = 0.0;
      hit[q] = 0;
    }
    o.bin_ptr[b + 1] = (int)o.bin_pix.size();
    o.max_bin_nnz = std::max(o.max_bin_nnz, o.bin_ptr[b + 1] - o.bin_ptr[b]);
    std::vector<int>().swap(fields[b]);
  }
  o.pix_ptr.assign(o.n_pix + 1, 0);
  for (int p = 0; p < o.n_pix; ++p) o.pix_ptr[p + 1] = o.pix_ptr[p] + pcount[p];
  o.pix_bin.resize(o.bin_pix.size());
  o.pix_w.resize(o.bin_pix.size());
  std::vector<int> fill(o.pix_ptr.begin(), o.pix_ptr.end() - 1);
  for (int b = 0; b < o.n_bins; ++b)
    for (int e = o.bin_ptr[b]; e < o.bin_ptr[b + 1]; ++e) {
      const int p = o.bin_pix[e];
      o.pix_bin[fill[p]] = b;
      o.pix_w[fill[p]] = o.bin_w[e];
      fill[p]++;
    }
}

// Polar table of the spherically aligned model: radii log-spaced from half
// the smallest distance of a padded sub-pixel centre from the centre to
// 12 max sigma'_k / min q'_k; and the 8-node Gauss-Legendre rule on [-1, 1].
void build_spherical(GeomHost &o) {
  double rmin = 0.0;
  for (double x : o.xs)
    for (double y : o.ys) {
      const double r = std::sqrt(x * x + y * y);
      if (r > 0.0 && (rmin == 0.0 || r < rmin)) rmin = r;
    }
  const double r_lo = rmin > 0.0 ? 0.5 * rmin : 1e-3;
  double smax = 0.0, qmin = 1.0;
  for (int k = 0; k < o.K; ++k) {
    smax = std::max(smax, o.lum_sigma[k]);
    qmin = std::min(qmin, o.lum_q[k]);
  }
  const double r_hi = 12.0 * smax / qmin;
  o.sph_lnr0 = std::log(r_lo);
  o.sph_dlnr = (std::log(r_hi) - std::log(r_lo)) / (jam::kSphNR - 1);
  o.sph_sig_max = smax;
  double u[8], w[8];
  gauss_legendre01(8, u, w);
  for (int i = 0; i < 8; ++i) {
    o.gl8_x[i] = 2.0 * u[i] - 1.0;
    o.gl8_w[i] = 2.0 * w[i];
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// How a plan schedules its numerator (what the autotuner varies).
struct Tune {
  int rule = 1;     // 0 per-pixel VALU everywhere; 1 matrix cores, one wave per tile of
                    // 32x32 blocks
  int tau = 0;      // a map axis with at least tau distinct values pairs its 32-blocks
                    // into 64-wide tiles
  int gran = 0;     // slice length: units of 64 terms per MFMA item, or (k, j) pairs per
                    // per-pixel item; 0 = derived from the batch
  int launch = 0;   // 0 one workgroup per item; 1 persistent grid pulling items from a
                    // device queue
  int map = 0;      // derived from the batch, not tuned: 1 when rule 1 runs every model
                    // with the whole-map matrix-core kernel (all maps of 7 x 7 blocks)
};

// Every pointer a captured graph was recorded with (parameters, outputs,
// cotangents, gradients, workspace) in a fixed order, and the workspace
// size; a graph is replayed only when all of them match exactly.
struct GraphKey {
  static constexpr int kMax = 16;
  const void *p[kMax] = {};
  int n = 0;
  size_t ws_bytes = 0;
  GraphKey() = default;
  GraphKey(std::initializer_list<const void *> ptrs, size_t ws) : ws_bytes(ws) {
    for (const void *q : ptrs) p[n++] = q;
  }
  bool operator==(const GraphKey &o) const {
    if (n != o.n || ws_bytes != o.ws_bytes) return false;
    for (int i = 0; i < n; ++i)
      if (p[i] != o.p[i]) return false;
    return true;
  }
};

// A prepared batch composition.
struct Plan {
  std::vector<int32_t> key;
  int n = 0;
  Tune tune;
  void *arena = nullptr;
  jam::ModelDev *d_models = nullptr;
  jam::Item *d_terms = nullptr, *d_pix = nullptr, *d_num = nullptr, *d_bins = nullptr,
            *d_maps = nullptr, *d_chain = nullptr, *d_sens = nullptr, *d_sb = nullptr,
            *d_red = nullptr, *d_sph = nullptr, *d_pro = nullptr, *d_adj = nullptr,
            *d_redf = nullptr, *d_sensw = nullptr, *d_sgrid = nullptr, *d_sgred = nullptr,
            *d_sgred6 = nullptr, *d_pcot = nullptr, *d_pfix = nullptr, *d_sgs = nullptr,
            *d_sphm = nullptr;
  int n_terms = 0, n_pix = 0, n_num = 0, n_bins = 0, n_maps = 0, n_chain = 0, n_sens = 0,
      n_sb = 0, n_red = 0, n_sph = 0, n_pro = 0, n_adj = 0, n_redf = 0, n_sensw = 0,
      n_sgrid = 0, n_sgred = 0, n_sgred6 = 0, n_pcot = 0, n_pfix = 0, n_sgs = 0, n_sphm = 0;
  int n_bins_wave = 0;   // leading bin items summed one bin per wave
  bool spherical = false;
  bool fused_prologue = true;
  int grid_num = 1, grid_sens = 1;
  int64_t total_bins = 0, total_lum = 0, total_mass = 0, total_map = 0;
  // workspace regions (bytes)
  size_t off_status = 0, off_queue = 0, off_gauss = 0, off_terms = 0, off_pix = 0, off_part = 0,
         off_bins = 0, off_vfwd = 0, off_sph = 0, off_sgrid = 0, off_sgrid6 = 0, off_sgcot = 0,
         off_sens = 0,
         off_vtmp = 0,
         off_cot = 0,
         off_sbp = 0,
         ws_fwd = 0, ws_vjp = 0;
  // captured evaluations (forward, adjoint, forward + chi^2, adjoint of chi^2)
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  GraphKey gkey[4];
  ~Plan() {
    for (auto &g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    if (arena) (void)hipFree(arena);
  }
};

}  // namespace

// Event pairs bracketing launches of one kernel, for jam_timing.
struct KernelTimer {
  static constexpr int kCap = 4096;
  std::vector<hipEvent_t> start, stop;
  int used = 0;
  bool on = false;
  void destroy() {
    for (auto e : start) (void)hipEventDestroy(e);
    for (auto e : stop) (void)hipEventDestroy(e);
    start.clear();
    stop.clear();
  }
  bool begin(hipStream_t st, bool capturing) {
    if (!on || capturing || used >= (int)start.size()) return false;
    return hipEventRecord(start[used], st) == hipSuccess;
  }
  void end(hipStream_t st) { (void)hipEventRecord(stop[used++], st); }
};

// ---------------------------------------------------------------------------
// Fixed scratch memory of jam_eval_batch_noalloc.  Each GPU the library runs
// on holds its own copy of this array until the process ends.  In host code
// its name is only a host-side stand-in: the device address is taken once
// per device with hipGetSymbolAddress (at jam_create, with that device
// current) and that address, never the name, is what host code passes on.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev`, which must be current.
jam_status scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(JAM_E_UNSUPPORTED, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return JAM_OK;
}
}  // namespace

struct jam_ctx {
  int device = 0;
  int n_cu = 256;
  int occ_num_pix = 1, occ_num_mfma = 1, occ_sens = 1;
  jam_options opt{0, 0, nullptr, 0, 0, 0};
  std::string tune_path;
  std::vector<std::pair<std::string, Tune>> tuned;   // autotuner cache
  std::vector<GeomHost> gh;
  void *arena = nullptr;
  jam::GeomDev *d_geoms = nullptr;
  std::list<std::unique_ptr<Plan>> plans;   // most recent first
  KernelTimer t_num, t_sens;
  hipStream_t cap_stream = nullptr;         // graph capture only
  void *scratch = nullptr;                  // device address of the fixed scratch array
  // observed kinematics per geometry (chi^2): one device buffer each holding
  // [vrms_obs | inverse covariance], and the device table of pointers
  std::vector<void *> kin_buf;
  std::vector<jam::KinDev> kin_host;
  jam::KinDev *d_kin = nullptr;
  ~jam_ctx() {
    plans.clear();
    t_num.destroy();
    t_sens.destroy();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void *b : kin_buf)
      if (b) (void)hipFree(b);
    if (d_kin) (void)hipFree(d_kin);
    if (arena) (void)hipFree(arena);
  }
};

namespace {

constexpr size_t kMaxPlans = 8;
// Batches of at most this many models run the cylindrical prologue as one
// launch (each term block recomputes its (k, j) pairs' set-up, which costs
// latency per block but saves two launches).
constexpr int kFusedPrologueModels = 32;
// Unique-pixel maps with at most this many distinct |x'| and |y'| (one 32x32
// matrix-core block) take the small-map form: terms computed in place by the
// numerator, sensitivities and chain fused in the adjoint (for at most
// jam::kSmallAdjMass mass Gaussians, the BH included).
constexpr int kSmallMap = 32;
// Whole-map numerator: longest slice, in units of 64 terms, summed in FP32.
constexpr int kMapMaxUnits = 32;
// Does a geometry's map suit the whole-map matrix-core numerator?
bool map_fits(int n_ux, int n_uy) {
  const int bx = (n_ux + 31) / 32, by = (n_uy + 31) / 32;
  return bx == jam::kMapBlocks && by == jam::kMapBlocks;
}
// Geometries whose bins have at most this many weights each sum every bin
// with one wave (4 bins per workgroup) instead of a whole workgroup.
constexpr int kBinWaveNnz = 2048;

// Numerator variant and term-range split of one model under a schedule.
// `gran` is the slice length in units: (k, j) pairs for the per-pixel
// variant, 64 terms for the matrix-core variant.  The matrix-core variant
// covers the unique-pixel map with wave tiles of BX x BY blocks of 32x32:
// along an axis with at least tau distinct values the blocks pair up into
// 64-wide tiles (an odd last block stays 32 wide).
struct WaveTile {
  int bx, by, BX, BY;   // origin in 32-blocks, extent in blocks (1 or 2)
};

struct NumChoice {
  int kind;      // 0 per-pixel VALU, 2 matrix-core wave tiles
  bool gen = false;   // matrix core on a map of one 32x32 block, terms computed in place
  bool map = false;   // matrix core, one workgroup per whole map and slice
  int n_slices;
  int units;     // slice units of the whole term range
  std::vector<WaveTile> tiles;   // matrix core
  int pix_blocks = 0;            // per-pixel: 64-pixel blocks
  int n_tiles() const { return kind == 0 ? pix_blocks : (int)tiles.size(); }
  double tile_units(int i) const { return kind == 0 ? 1.0 : tiles[i].BX * tiles[i].BY; }
};

std::vector<std::pair<int, int>> axis_tiles(int n, int tau) {
  const int nb = (n + 31) / 32;
  std::vector<std::pair<int, int>> out;   // (first block, blocks)
  for (int b = 0; b < nb;) {
    const int w = (n >= tau && b + 1 < nb) ? 2 : 1;
    out.push_back({b, w});
    b += w;
  }
  return out;
}

NumChoice choose_numerator(const GeomHost &g, const Tune &t, int gran) {
  NumChoice c;
  if (t.rule == 0) {
    const int pairs = g.K * g.J1;
    const int per = std::max(1, gran);
    c.kind = 0;
    c.n_slices = std::max(1, (pairs + per - 1) / per);
    c.units = pairs;
    c.pix_blocks = (g.n_pix + 255) / 256;
    return c;
  }
  const int chunks = (g.T + 63) / 64;
  c.kind = 2;
  if (t.map) {
    // FP32 accumulation over a slice: at most kMapMaxUnits x 64 terms
    const int per = std::max(1, std::min(kMapMaxUnits, gran));
    c.map = true;
    c.n_slices = std::max(1, (chunks + per - 1) / per);
    c.units = chunks;
    c.tiles.push_back({0, 0, (g.n_ux + 31) / 32, (g.n_uy + 31) / 32});
    return c;
  }
  const int per = std::max(4, gran);
  c.gen = g.n_ux <= kSmallMap && g.n_uy <= kSmallMap && g.J1 <= jam::kSmallAdjMass;
  c.n_slices = std::max(1, (chunks + per - 1) / per);
  c.units = chunks;
  for (const auto &ty : axis_tiles(g.n_uy, t.tau))
    for (const auto &tx : axis_tiles(g.n_ux, t.tau))
      c.tiles.push_back({tx.first, ty.first, tx.second, ty.second});
  return c;
}

// Relative cost of one numerator item, for largest-first ordering and the
// schedule model: the kernels' chunk loop plus a fixed per-item cost (the
// partial-tile store and its reduction).  `tile` indexes c's tiles.
double num_item_cost(const GeomHost &g, const NumChoice &c, int slice, int tile) {
  if (c.kind == 0) {
    const int pairs = g.K * g.J1;
    const int per = (pairs + c.n_slices - 1) / c.n_slices;
    const int cnt = std::max(0, std::min(pairs, (slice + 1) * per) - slice * per);
    return cnt * (double)g.n_u * 256.0 * 5.0 / 32768.0 + 1.0;
  }
  const int chunks = (g.T + 63) / 64;
  const int per = (chunks + c.n_slices - 1) / c.n_slices;
  const int cnt = std::max(0, std::min(chunks, (slice + 1) * per) - slice * per);
  // per chunk of a wave (a quarter of the item's chunks): 32 MFMAs per block
  // and operand generation per row / column block; per item: the start
  // (dependent descriptor and coordinate loads, first chunk), the four-wave
  // sum and the tile store
  const WaveTile &w = c.tiles[tile];
  if (c.map) {
    // every wave runs every chunk for its quarter of the blocks; the
    // workgroup generates the operands of all rows and columns once
    const int nblk = w.BX * w.BY;
    return cnt * (1.5 * ((nblk + 3) / 4) + 0.75) + 8.0;
  }
  // terms computed in place: their FP64 set-up per chunk
  const double gen = c.gen ? 0.5 : 0.0;
  return ((cnt + 3) / 4) * (1.5 * w.BX * w.BY + 0.75 * (w.BX + w.BY) + gen) + 8.0;
}

// Completion time of the numerator launch as modelled: every resident
// workgroup pulls the next item, largest first, from the queue, i.e. list
// scheduling in cost order on `slots` identical workers.
double list_schedule_makespan(std::vector<double> &cost, int slots) {
  std::sort(cost.begin(), cost.end(), std::greater<double>());
  if (cost.empty()) return 0.0;
  if ((int)cost.size() <= slots) return cost[0];
  std::priority_queue<double, std::vector<double>, std::greater<double>> q;
  for (int i = 0; i < slots; ++i) q.push(0.0);
  double mk = 0.0;
  for (double c : cost) {
    const double t = q.top() + c;
    q.pop();
    mk = std::max(mk, t);
    q.push(t);
  }
  return mk;
}

// Workers of the schedule model.  A compute unit processes the workgroups
// resident on it at its full rate however many there are (co-resident
// workgroups share its SIMDs), so the model's workers are the compute units
// and its jobs the workgroup items.
int num_slots(const jam_ctx *ctx, const Tune &) { return std::max(1, ctx->n_cu); }

// Default slice length: the one whose item list the workers finish first
// under the list-scheduling model.  Candidates are geometric around a few
// jobs per worker, plus the exact splits of the largest model, so a uniform
// item list can fill whole rounds of workers.
int default_gran(const jam_ctx *ctx, int n, const int32_t *geom_idx, const Tune &t) {
  const int slots = num_slots(ctx, t);
  double work = 0.0, big_work = -1.0;
  int big_units = 1, big_tiles = 1;
  for (int m = 0; m < n; ++m) {
    const GeomHost &g = ctx->gh[geom_idx[m]];
    const NumChoice c = choose_numerator(g, t, 1 << 29);
    const double w = (double)c.n_tiles() * c.units;
    work += w;
    if (w > big_work) {
      big_work = w;
      big_units = c.units;
      big_tiles = c.n_tiles();
    }
  }
  // jobs a worker holds at once
  const double per_slot = t.rule == 0 ? ctx->occ_num_pix : (t.map ? 1 : ctx->occ_num_mfma);
  const double g0 = std::max(1.0, std::ceil(work / (slots * per_slot)));
  std::vector<int> cands;
  for (int k = -8; k <= 16; ++k)
    cands.push_back((int)std::min(1.0e9, std::max(1.0, std::round(g0 * std::pow(2.0, k / 8.0)))));
  if (big_work >= 0.25 * work) {
    const int s_max = std::min(4096, (int)(4 * per_slot) * slots / std::max(1, big_tiles) + 1);
    for (int sl = 1; sl <= s_max; ++sl) cands.push_back((big_units + sl - 1) / sl);
  }
  // whole-map slices are capped (FP32 accumulation): every length up to the cap
  if (t.map)
    for (int gr = 1; gr <= kMapMaxUnits; ++gr) cands.push_back(gr);
  std::sort(cands.begin(), cands.end());
  cands.erase(std::unique(cands.begin(), cands.end()), cands.end());
  double best = 1e300;
  int best_g = (int)g0;
  std::vector<double> cost;
  for (int gr : cands) {
    cost.clear();
    for (int m = 0; m < n; ++m) {
      const GeomHost &g = ctx->gh[geom_idx[m]];
      const NumChoice c = choose_numerator(g, t, gr);
      for (int sl = 0; sl < c.n_slices; ++sl)
        for (int tl = 0; tl < c.n_tiles(); ++tl) cost.push_back(num_item_cost(g, c, sl, tl));
    }
    if (cost.size() > (size_t)(64 * per_slot) * slots + (size_t)4 * n) continue;   // too fine
    const double mk = list_schedule_makespan(cost, slots);
    if (mk < best * (1.0 - 1e-9) || (mk <= best * (1.0 + 1e-9) && gr > best_g)) {
      best = mk;
      best_g = gr;
    }
  }
  return std::min(1 << 29, std::max(1, best_g));
}

void sort_by_cost(std::vector<jam::Item> &items, std::vector<double> &cost) {
  std::vector<size_t> idx(items.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return cost[a] > cost[b]; });
  std::vector<jam::Item> out(items.size());
  for (size_t i = 0; i < idx.size(); ++i) out[i] = items[idx[i]];
  items.swap(out);
}

// The wide adjoint form (k_sens_wide) is used on maps of at least two x
// tiles with at least this many distinct |y|: each 32-term group then runs
// over enough y steps to amortise its accumulator set-up and epilogue
// (measured: faster than the one-tile form at 215, slower at <= 128).
constexpr int kWideMinY = 160;

struct WidePart { int m, pt, xt, groups; };

// Cut the wide parts into items.  A part of xt tiles takes items of
// per(c, xt) 32-term groups, c for four tiles and proportionally more for
// fewer, a multiple of the workgroup's waves; c is chosen by the modelled
// completion time on n_cu compute units (one workgroup each, items taken
// largest first), an item costing its critical wave's (group x tile) count
// plus one for staging lambda.  Items are emitted largest first.
void wide_items(const std::vector<WidePart> &parts, int n_cu, std::vector<jam::Item> &out) {
  out.clear();
  if (parts.empty()) return;
  constexpr int kWW = jam::kWideWaves;
  int64_t tot = 0;
  for (const WidePart &w : parts) tot += (int64_t)w.xt * w.groups;
  const int64_t share = std::max<int64_t>(1, (tot / 4 + n_cu - 1) / std::max(1, n_cu));
  auto per_of = [](int64_t c, int xt) {
    constexpr int64_t w = jam::kWideWaves;
    return (int)std::max<int64_t>(w, (c * 4 / xt + w - 1) / w * w);
  };
  auto cost_of = [](int ng, int xt) {
    constexpr int w = jam::kWideWaves;
    return (double)((ng + w - 1) / w) * xt + 1.0;
  };
  const int64_t step = std::max<int64_t>(kWW, share / 64 / kWW * kWW);
  int64_t best = kWW;
  double best_t = -1.0;
  std::vector<double> cost;
  for (int64_t c = std::max<int64_t>(kWW, share / 4 / kWW * kWW); c <= 2 * share + kWW; c += step) {
    cost.clear();
    for (const WidePart &w : parts) {
      const int per = per_of(c, w.xt);
      for (int g0 = 0; g0 < w.groups; g0 += per) cost.push_back(cost_of(std::min(per, w.groups - g0), w.xt));
    }
    const double t = list_schedule_makespan(cost, n_cu);
    if (best_t < 0.0 || t < best_t) { best = c; best_t = t; }
  }
  cost.clear();
  for (const WidePart &w : parts) {
    const int per = per_of(best, w.xt);
    for (int g0 = 0; g0 < w.groups; g0 += per) {
      const int g1 = std::min(w.groups, g0 + per);
      out.push_back({w.m, w.pt | (w.xt << 16), g0, g1});
      cost.push_back(cost_of(g1 - g0, w.xt));
    }
  }
  sort_by_cost(out, cost);
}

jam_status build_plan(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, const Tune &tune_in,
                      std::unique_ptr<Plan> &out) {
  auto p = std::make_unique<Plan>();
  p->key.assign(geom_idx, geom_idx + n);
  p->n = n;
  p->tune = tune_in;
  p->tune.map = 0;
  if (p->tune.rule == 1 && ctx->opt.alignment != 1) {
    bool all = true;
    for (int m = 0; m < n && all; ++m)
      all = map_fits(ctx->gh[geom_idx[m]].n_ux, ctx->gh[geom_idx[m]].n_uy);
    p->tune.map = all ? 1 : 0;
  }
  if (p->tune.gran <= 0) p->tune.gran = default_gran(ctx, n, geom_idx, p->tune);
  const Tune &tune = p->tune;
  std::vector<jam::ModelDev> md(n);
  std::vector<jam::Item> it_terms, it_pix, it_num, it_bins, it_maps, it_chain, it_sens, it_sb,
      it_red, it_sph, it_pro, it_adj, it_redf, it_sensw, it_sgrid, it_sgred, it_sgred6, it_pcot,
      it_pfix, it_sgs, it_sphm;
  std::vector<double> c_num, c_sens, c_sensw;
  // wide-sensitivity parts (model, part, x tiles, 32-term groups); their
  // items are cut after the model loop (wide_items)
  std::vector<WidePart> wide_parts;
  int64_t gauss = 0, terms = 0, pixd = 0, part = 0, bins = 0, sens = 0, sph = 0, sbp = 0,
          sgrid = 0, sgrid6 = 0, sgcot = 0;
  const bool spherical = ctx->opt.alignment == 1;
  // spherical forward: the potential grid (form 1: sums at every node)
  const bool use_sgrid = spherical && ctx->opt.form != 1;
  for (int m = 0; m < n; ++m) {
    const int gi = geom_idx[m];
    const GeomHost &g = ctx->gh[gi];
    jam::ModelDev &d = md[m];
    std::memset(&d, 0, sizeof d);
    d.geom = gi;
    d.lum_off = (int)p->total_lum;
    d.mass_off = (int)p->total_mass;
    d.out_off = (int)p->total_bins;
    const NumChoice nc = choose_numerator(g, tune, tune.gran);
    d.n_slices = nc.n_slices;
    const bool small = !spherical && nc.gen;
    d.form = nc.kind == 0 ? 1 : (small ? 3 : (nc.map ? 4 : 2));
    d.part_f32 = nc.map ? 1 : 0;
    // adjoint sensitivity blocks: one (per-pixel), none (small map), one per
    // x tile (one tile), one per part of up to four x tiles (wide)
    // (the wide form pays off where each term group runs over many y steps:
    // its per-group epilogue and accumulator set-up are fixed costs)
    const int n_xt = (g.n_ux + 31) / 32;
    const bool wide = !spherical && !small && d.form != 1 && n_xt >= 2 && g.n_uy >= kWideMinY;
    d.n_sens_parts = d.form == 1 ? 1 : (small ? 0 : (wide ? (n_xt + 3) / 4 : n_xt));
    d.n_xt = (g.n_ux + 31) / 32;
    d.n_yt = (g.n_uy + 31) / 32;
    d.gauss_off = gauss;
    d.term_off = terms;
    d.pix_off = pixd;
    d.part_off = part;
    d.map_off = p->total_map;
    d.sens_off = sens;
    d.bin_off = bins;
    d.sph_off = sph;
    d.sbp_off = sbp;
    sbp += (int64_t)g.K * jam::sb_tiles(g.n_ux, g.n_uy);
    if (spherical) {
      sph += (int64_t)jam::kSphNR * jam::kSphNT * 3;
      for (int q = 0; q < jam::kSphNR * jam::kSphNT; ++q) it_sph.push_back({m, q, 0, 0});
      // forward moments: four table points per item (a wave each)
      for (int q = 0; q < jam::kSphNR * jam::kSphNT / 4; ++q) it_sphm.push_back({m, q, 0, 0});
    }
    if (use_sgrid) {
      // forward grid: 2 floats per point; the adjoint's: 8
      const int64_t nn2 = 2 * (int64_t)jam::kSphGridN * jam::kSphGridN;
      const int64_t nn8 = 4 * nn2;
      // term slices of at least ten 64-term chunks, at most eight (a
      // property of the model alone, so that its grid, and everything
      // computed from it, is the same in any batch)
      const int sl = std::max(1, std::min(8, jam::sph_terms_padded(g.J1, g.n_u) / 640));
      d.sgrid_slices = sl;
      d.sgrid_off = sgrid;
      d.sgrid6_off = sgrid6;
      sgrid += sl * nn2;
      sgrid6 += sl * nn8;
      for (int tile = 0; tile < jam::kSphGridTiles; ++tile)
        for (int q = 0; q < sl; ++q) it_sgrid.push_back({m, tile, q, 0});
      if (sl > 1) {
        for (int64_t bq = 0; bq < (nn2 + 1023) / 1024; ++bq) it_sgred.push_back({m, (int)bq, 0, 0});
        for (int64_t bq = 0; bq < (nn8 + 1023) / 1024; ++bq) it_sgred6.push_back({m, (int)bq, 0, 0});
      }
    }
    gauss += jam::gauss_size(g.K, g.J1);
    const int tsph = jam::sph_terms_padded(g.J1, g.n_u);
    // spherical: float4 terms, then floats; small maps compute their terms in
    // place; cylindrical tables are zero-padded to a multiple of 32 terms
    terms += spherical ? tsph + tsph / 4 : (small ? 0 : jam::padded_terms(g.T));
    pixd += 4 * (int64_t)g.n_pix;
    // padded to whole blocks; FP32 partials (whole-map numerator) take half
    const int64_t part_elems = (int64_t)d.n_slices * (32 * d.n_xt) * (32 * d.n_yt);
    part += nc.map ? (part_elems + 1) / 2 : part_elems;
    bins += 2 * (int64_t)g.n_bins;
    if (spherical) {
      // term sensitivities: point ranges, or (with the potential grid) parts
      // of the grid rows
      d.n_sens_parts = use_sgrid ? jam::kSphIParts : jam::sph_ranges(g.K);
      sens += jam::sph_adj_size(g.K, g.n_pix, tsph, d.n_sens_parts);
    } else {
      sens += 3 * (int64_t)d.n_sens_parts * g.T + (int64_t)g.K * 3 * g.J1;
    }
    p->total_lum += g.K;
    p->total_mass += g.J;
    p->total_bins += g.n_bins;
    p->total_map += (int64_t)g.nxp * g.nyp;
    if (!small)
      for (int tb = 0; tb < ((spherical ? tsph : g.T) + 255) / 256; ++tb)
        it_terms.push_back({m, tb, 0, 0});
    if (spherical && use_sgrid) {
      d.sgcot_off = sgcot;
      sgcot += jam::sph_gcot_size(g.K);
      for (int q = 0; q < jam::sph_pitems(g.K); ++q) it_pcot.push_back({m, q, 0, 0});
      for (int b = 0; b < jam::kSphGridN * jam::kSphGridN / 1024; ++b) it_pfix.push_back({m, b, 0, 0});
      for (int tb = 0; tb < tsph / 32; ++tb)
        for (int ip = 0; ip < jam::kSphIParts; ++ip) it_sgs.push_back({m, tb, ip, 0});
    } else if (spherical) {
      for (int tt = 0; tt < (tsph + 255) / 256; ++tt)
        for (int r = 0; r < d.n_sens_parts; ++r) {
          it_sens.push_back({m, tt, r, 0});
          c_sens.push_back((double)jam::sph_range_len(g.K, d.n_sens_parts));
        }
    } else if (small) {
      // fused sensitivities + chain: items of whole tracers, about 8192
      // terms each
      const int per = std::max(1, std::min(jam::kSmallAdjTracers, 8192 / (g.J1 * g.n_u)));
      for (int k = 0; k < g.K; k += per)
        it_adj.push_back({m, k | (std::min(g.K, k + per) << 16), 0, 0});
    } else if (d.form == 1) {
      for (int tb = 0; tb < (g.T + 255) / 256; ++tb) {
        it_sens.push_back({m, tb, 0, 0});
        c_sens.push_back((double)g.n_pix);
      }
    } else if (wide) {
      // parts of up to four x tiles
      for (int pt = 0; pt < d.n_sens_parts; ++pt)
        wide_parts.push_back({m, pt, std::min(4, n_xt - 4 * pt), (g.T + 31) / 32});
    } else {
      for (int xt = 0; xt < d.n_sens_parts; ++xt)
        for (int tt = 0; tt < (g.T + jam::kSensTerms - 1) / jam::kSensTerms; ++tt) {
          it_sens.push_back({m, xt, tt, 1});
          c_sens.push_back(8.0 * 32.0 * g.n_uy);
        }
    }
    for (int pb = 0; pb < (g.n_pix + 255) / 256; ++pb) it_pix.push_back({m, pb, 0, 0});
    if (nc.map)   // FP32 partials, reduced over the padded layout
      for (int pb = 0; pb < (g.n_ux * 32 * d.n_yt + 255) / 256; ++pb) it_redf.push_back({m, pb, 0, 0});
    else
      for (int pb = 0; pb < (g.n_pix + 63) / 64; ++pb) it_red.push_back({m, pb, 0, 0});
    for (int rb = 0; rb < (g.n_uy + 7) / 8; ++rb)
      for (int cb = 0; cb < (g.n_ux + 63) / 64; ++cb) it_sb.push_back({m, rb, cb, 0});
    for (int s = 0; s < d.n_slices; ++s)
      for (int tl = 0; tl < nc.n_tiles(); ++tl) {
        if (nc.kind == 0) {
          it_num.push_back({m, tl, s, 0});
        } else {
          const WaveTile &w = nc.tiles[tl];
          it_num.push_back({m, w.bx | (w.by << 16), s,
                            nc.map ? 7 : (small ? 6 : 2 + (w.BX - 1) + 2 * (w.BY - 1))});
        }
        c_num.push_back(num_item_cost(g, nc, s, tl));
      }
    if (g.max_bin_nnz <= kBinWaveNnz)
      for (int b = 0; b < g.n_bins; b += 4) it_bins.push_back({m, b, 0, 1});
    else
      for (int b = 0; b < g.n_bins; ++b) it_bins.push_back({m, b, 0, 0});
    for (int r = 0; r < g.nyp; ++r) it_maps.push_back({m, r, 0, 0});
    if (!spherical && !small)
      for (int k = 0; k < g.K; ++k)
        for (int jb = 0; jb < (g.J1 + 3) / 4; ++jb) it_chain.push_back({m, k, jb, 0});
  }
  if (p->total_bins > INT32_MAX || p->total_lum > INT32_MAX || p->total_mass > INT32_MAX)
    return fail(JAM_E_UNSUPPORTED, "batch too large");
  // prologue of the cylindrical model: a few models run set-up, terms and
  // surface brightness in one launch (terms from the parameters); many run
  // the set-up first and then terms from its table beside the tiles
  p->fused_prologue = n <= kFusedPrologueModels;
  if (p->fused_prologue)
    for (int m = 0; m < n; ++m) it_pro.push_back({m, 0, 0, 0});
  for (const jam::Item &t : it_terms) it_pro.push_back({t.m, t.a, 0, p->fused_prologue ? 1 : 3});
  for (const jam::Item &t : it_sb) it_pro.push_back({t.m, t.a, t.b, 2});
  // bin items: the one-bin-per-wave ones first (a launch of 256-thread
  // blocks), then the one-bin-per-block ones (1024-thread blocks)
  std::stable_partition(it_bins.begin(), it_bins.end(), [](const jam::Item &t) { return t.c == 1; });
  p->n_bins_wave = (int)std::count_if(it_bins.begin(), it_bins.end(),
                                      [](const jam::Item &t) { return t.c == 1; });
  sort_by_cost(it_num, c_num);
  sort_by_cost(it_sens, c_sens);
  wide_items(wide_parts, ctx->n_cu, it_sensw);

  constexpr int kLists = 21;
  std::vector<jam::Item> *lists[kLists] = {&it_terms, &it_pix, &it_num, &it_bins,
                                           &it_maps,  &it_chain, &it_sens, &it_sb,
                                           &it_red,   &it_sph, &it_pro, &it_adj, &it_redf,
                                           &it_sensw, &it_sgrid, &it_sgred, &it_sgred6,
                                           &it_pcot,  &it_pfix,  &it_sgs,  &it_sphm};
  for (auto *l : lists)
    if (l->size() > (size_t)INT32_MAX) return fail(JAM_E_UNSUPPORTED, "batch too large");
  // one device arena: models then the item lists
  size_t off = 0;
  const size_t o_models = off;
  off = align256(off + sizeof(jam::ModelDev) * n);
  size_t o_it[kLists];
  for (int i = 0; i < kLists; ++i) {
    o_it[i] = off;
    off = align256(off + sizeof(jam::Item) * std::max<size_t>(1, lists[i]->size()));
  }
  std::vector<char> stage(off, 0);
  std::memcpy(stage.data() + o_models, md.data(), sizeof(jam::ModelDev) * n);
  for (int i = 0; i < kLists; ++i)
    if (!lists[i]->empty())
      std::memcpy(stage.data() + o_it[i], lists[i]->data(), sizeof(jam::Item) * lists[i]->size());
  HIP_TRY(hipMalloc(&p->arena, off));
  HIP_TRY(hipMemcpy(p->arena, stage.data(), off, hipMemcpyHostToDevice));
  char *base = (char *)p->arena;
  p->d_models = (jam::ModelDev *)(base + o_models);
  jam::Item **dl[kLists] = {&p->d_terms, &p->d_pix,  &p->d_num, &p->d_bins,
                            &p->d_maps,  &p->d_chain, &p->d_sens, &p->d_sb,
                            &p->d_red,   &p->d_sph,   &p->d_pro,  &p->d_adj, &p->d_redf,
                            &p->d_sensw, &p->d_sgrid, &p->d_sgred, &p->d_sgred6,
                            &p->d_pcot,  &p->d_pfix,  &p->d_sgs,  &p->d_sphm};
  int *cnt[kLists] = {&p->n_terms, &p->n_pix,  &p->n_num, &p->n_bins,
                      &p->n_maps,  &p->n_chain, &p->n_sens, &p->n_sb,
                      &p->n_red,   &p->n_sph,   &p->n_pro,  &p->n_adj, &p->n_redf,
                      &p->n_sensw, &p->n_sgrid, &p->n_sgred, &p->n_sgred6,
                      &p->n_pcot,  &p->n_pfix,  &p->n_sgs,  &p->n_sphm};
  for (int i = 0; i < kLists; ++i) {
    *dl[i] = (jam::Item *)(base + o_it[i]);
    *cnt[i] = (int)lists[i]->size();
  }
  const int num_wg = p->n_num;   // one workgroup per numerator item
  if (tune.launch == 1) {
    const int occ = tune.rule == 0 ? ctx->occ_num_pix : (tune.map ? 1 : ctx->occ_num_mfma);
    p->grid_num = std::max(1, std::min(num_wg, ctx->n_cu * occ));
    p->grid_sens = std::max(1, std::min(p->n_sens, ctx->n_cu * ctx->occ_sens));
  } else {
    p->grid_num = std::max(1, num_wg);
    p->grid_sens = std::max(1, p->n_sens);
  }
  // workspace layout
  size_t w = 0;
  p->off_status = w; w = align256(w + sizeof(int) * n);
  p->off_queue = w;  w = align256(w + sizeof(int) * 2);
  p->off_gauss = w;  w = align256(w + sizeof(double) * gauss);
  p->off_terms = w;  w = align256(w + sizeof(float4) * terms);
  p->off_pix = w;    w = align256(w + sizeof(double) * pixd);
  p->off_part = w;   w = align256(w + sizeof(double) * part);
  p->off_bins = w;   w = align256(w + sizeof(double) * bins);
  p->off_vfwd = w;   w = align256(w + sizeof(double) * p->total_bins);
  p->off_sph = w;    w = align256(w + sizeof(double) * sph);
  p->off_sgrid = w;  w = align256(w + sizeof(float) * sgrid);
  p->ws_fwd = w;
  p->spherical = spherical;
  p->off_sens = w;   w = align256(w + sizeof(double) * sens);
  p->off_vtmp = w;   w = align256(w + sizeof(double) * p->total_bins);
  p->off_cot = w;    w = align256(w + sizeof(double) * p->total_bins);
  p->off_sbp = w;    w = align256(w + sizeof(double) * sbp);
  p->off_sgrid6 = w; w = align256(w + sizeof(float) * sgrid6);
  p->off_sgcot = w;  w = align256(w + sizeof(double) * sgcot);
  p->ws_vjp = w;
  out = std::move(p);
  return JAM_OK;
}

jam::ParamsDev params_of(const jam_batch *b) {
  return jam::ParamsDev{b->inc, b->mass_scale, b->m_bh, b->beta, b->lum_I0, b->mass_S0};
}

// Set-up, term table and SB map; optionally the numerator map.  Leaves N and
// I in the workspace pix region.
void launch_forward_maps(jam_ctx *ctx, Plan *p, const jam::ParamsDev &pd, int32_t *status,
                         char *ws, hipStream_t st, bool need_numerator, bool capturing) {
  int *st_ws = (int *)(ws + p->off_status);
  int *queue = (int *)(ws + p->off_queue);
  double *gauss = (double *)(ws + p->off_gauss);
  float4 *terms = (float4 *)(ws + p->off_terms);
  double *pix = (double *)(ws + p->off_pix);
  double *part = (double *)(ws + p->off_part);
  if (p->spherical) {
    jam::launch_setup(ctx->d_geoms, p->d_models, p->n, pd, gauss, st_ws, status, queue, st);
    jam::launch_sph_terms(ctx->d_geoms, p->d_models, p->d_terms, p->n_terms, gauss, st_ws, terms,
                          st);
    jam::launch_sb(ctx->d_geoms, p->d_models, p->d_sb, p->n_sb, pd, pix, st);
  } else {
    if (!p->fused_prologue)
      jam::launch_setup(ctx->d_geoms, p->d_models, p->n, pd, gauss, st_ws, status, queue, st);
    jam::launch_prologue(ctx->d_geoms, p->d_models, p->d_pro, p->n_pro, pd, gauss, st_ws, status,
                         queue, terms, pix, p->fused_prologue, st);
  }
  if (p->spherical) {
    if (!need_numerator) return;
    double *tabs = (double *)(ws + p->off_sph);
    float *sgrid = p->n_sgrid ? (float *)(ws + p->off_sgrid) : nullptr;
    const bool timed = ctx->t_num.begin(st, capturing);
    if (sgrid) {
      jam::launch_sph_grid(ctx->d_geoms, p->d_models, p->d_sgrid, p->n_sgrid, gauss, terms, st_ws,
                           sgrid, false, st);
      if (p->n_sgred)
        jam::launch_sph_grid_reduce(p->d_models, p->d_sgred, p->n_sgred, st_ws, sgrid, false, st);
    }
    jam::launch_sph_moments(ctx->d_geoms, p->d_models, p->d_sphm, p->n_sphm, gauss, terms, st_ws,
                            sgrid, tabs, st);
    if (timed) ctx->t_num.end(st);
    jam::launch_sph_num(ctx->d_geoms, p->d_models, p->d_red, p->n_red, gauss, st_ws, tabs, pix, st);
    return;
  }
  if (need_numerator) {
    const bool timed = ctx->t_num.begin(st, capturing);
    if (p->tune.map)
      jam::launch_num_map(ctx->d_geoms, p->d_models, p->d_num, p->n_num, terms, st_ws, part,
                          p->tune.launch == 1 ? queue : nullptr, p->grid_num, st);
    else
      jam::launch_num(ctx->d_geoms, p->d_models, p->d_num, p->n_num, terms, gauss, st_ws, part,
                      p->tune.launch == 1 ? queue : nullptr, p->grid_num, p->tune.rule == 1, st);
    if (timed) ctx->t_num.end(st);
    if (p->n_red) jam::launch_reduce(ctx->d_geoms, p->d_models, p->d_red, p->n_red, part, pix, st);
    if (p->n_redf)
      jam::launch_reduce_f32(ctx->d_geoms, p->d_models, p->d_redf, p->n_redf, part, pix, st);
  }
}

void launch_eval(jam_ctx *ctx, Plan *p, const jam_batch *b, double *vrms2, int32_t *status,
                 char *w, hipStream_t st, bool capturing) {
  launch_forward_maps(ctx, p, params_of(b), status, w, st, true, capturing);
  jam::launch_bins(ctx->d_geoms, p->d_models, p->d_bins, p->n_bins, p->n_bins_wave, (const double *)(w + p->off_pix),
                   (const int *)(w + p->off_status), vrms2, (double *)(w + p->off_bins), st);
}

// Adjoint of sum_b cot_b V_b; with chi2_cot != NULL the cotangent is instead
// chi2_cot[m] * d chi^2_m / dV_b, formed in the workspace from V (given or
// recomputed).
void launch_vjp(jam_ctx *ctx, Plan *p, const jam_batch *b, const double *vrms2, const double *cot,
                const jam_grads *grads, char *w, hipStream_t st, bool capturing,
                const double *chi2_cot = nullptr) {
  const int *st_ws = (const int *)(w + p->off_status);
  int *queue = (int *)(w + p->off_queue);
  double *pix = (double *)(w + p->off_pix);
  double *binws = (double *)(w + p->off_bins);
  double *sens = (double *)(w + p->off_sens);
  const jam::ParamsDev pd = params_of(b);
  const bool recompute = (vrms2 == nullptr);
  if (p->spherical) {
    // the spherical adjoint needs the moment table: one pass computes it with
    // the node sums of the characteristic integrals' adjoint.  When V is
    // recomputed it comes from the forward's own path (with the potential
    // grid, the forward's table and numerator map first, then the adjoint's
    // table over it), so that it equals the forward's V bit for bit
    const bool fwd_v = recompute && p->n_sgrid > 0;
    launch_forward_maps(ctx, p, pd, nullptr, w, st, fwd_v, capturing);
    const double *gauss = (const double *)(w + p->off_gauss);
    double *tabs = (double *)(w + p->off_sph);
    const float4 *terms = (const float4 *)(w + p->off_terms);
    float *sgrid6 = p->n_sgrid ? (float *)(w + p->off_sgrid6) : nullptr;
    if (sgrid6) {
      jam::launch_sph_grid(ctx->d_geoms, p->d_models, p->d_sgrid, p->n_sgrid, gauss, terms, st_ws,
                           sgrid6, true, st);
      if (p->n_sgred6)
        jam::launch_sph_grid_reduce(p->d_models, p->d_sgred6, p->n_sgred6, st_ws, sgrid6, true,
                                    st);
    }
    jam::launch_sph_moments_jac(ctx->d_geoms, p->d_models, p->d_sph, p->n_sph, gauss, terms,
                                st_ws, sgrid6, tabs, (double *)(w + p->off_sens), st);
    if (recompute && !fwd_v)
      jam::launch_sph_num(ctx->d_geoms, p->d_models, p->d_red, p->n_red, gauss, st_ws, tabs, pix,
                          st);
  } else {
    launch_forward_maps(ctx, p, pd, nullptr, w, st, recompute, capturing);
  }
  // V per bin: the caller's forward output, or recomputed into workspace.
  const double *V = vrms2;
  if (recompute) {
    double *vtmp = (double *)(w + p->off_vtmp);
    jam::launch_bins(ctx->d_geoms, p->d_models, p->d_bins, p->n_bins, p->n_bins_wave, pix, st_ws, vtmp, binws, st);
    V = vtmp;
  } else {
    jam::launch_bins(ctx->d_geoms, p->d_models, p->d_bins, p->n_bins, p->n_bins_wave, pix, st_ws, nullptr, binws, st);
  }
  if (chi2_cot) {
    double *c = (double *)(w + p->off_cot);
    jam::launch_chi2(ctx->d_geoms, p->d_models, p->n, ctx->d_kin, V, st_ws, nullptr, chi2_cot, c,
                     st);
    cot = c;
  }
  jam::launch_bins_adjoint(ctx->d_geoms, p->d_models, p->d_pix, p->n_pix, V, cot, binws, st_ws, pix, st);
  double *sbp = (double *)(w + p->off_sbp);
  jam::launch_sb_adjoint(ctx->d_geoms, p->d_models, p->d_sb, p->n_sb, st_ws, pix, sbp, st);
  const jam::GradsDev gd{grads->inc, grads->mass_scale, grads->m_bh, grads->beta, grads->lum_I0,
                         grads->mass_S0};
  if (p->spherical) {
    const bool ts = ctx->t_sens.begin(st, capturing);
    jam::launch_sph_adjoint(ctx->d_geoms, p->d_models, p->n, p->d_red, p->n_red, p->d_sph,
                            p->n_sph, p->d_sens, p->n_sens, p->d_terms, p->n_terms, p->d_pcot,
                            p->n_pcot, p->d_pfix, p->n_pfix, p->d_sgs, p->n_sgs, pd,
                            (const double *)(w + p->off_gauss),
                            (const float4 *)(w + p->off_terms), st_ws,
                            (const double *)(w + p->off_sph), pix, sbp, sens,
                            p->n_sgs ? (double *)(w + p->off_sgcot) : nullptr, gd, st);
    if (ts) ctx->t_sens.end(st);
    return;
  }
  const bool timed = ctx->t_sens.begin(st, capturing);
  if (p->n_sens)
    jam::launch_sens(ctx->d_geoms, p->d_models, p->d_sens, p->n_sens,
                     (const float4 *)(w + p->off_terms), pix, st_ws, sens,
                     p->tune.launch == 1 ? queue + 1 : nullptr, p->grid_sens, st);
  if (p->n_sensw)
    jam::launch_sens_wide(ctx->d_geoms, p->d_models, p->d_sensw, p->n_sensw,
                          (const float4 *)(w + p->off_terms), pix, st_ws, sens, nullptr,
                          p->n_sensw, st);
  if (p->n_adj)
    jam::launch_adj_small(ctx->d_geoms, p->d_models, p->d_adj, p->n_adj, pd, pix, st_ws, sens, st);
  if (timed) ctx->t_sens.end(st);
  if (p->n_chain)
    jam::launch_chain(ctx->d_geoms, p->d_models, p->d_chain, p->n_chain, pd, sens, st_ws, st);
  jam::launch_grads(ctx->d_geoms, p->d_models, p->n, pd, sens, sbp, st_ws, gd, st);
}

// ---------------------------------------------------------------------------
// Autotuner.  Candidates differ in the numerator schedule only (variant rule,
// 64x64-tile threshold, items' term granularity, persistent or one workgroup
// per item); each is timed on the batch composition with fixed valid
// parameters (edge-on, isotropic, unit mass scale) in a scratch workspace.
// Results are cached per composition signature, in memory and optionally in
// a text file (one "key rule tau gran launch" line per entry).
// ---------------------------------------------------------------------------
std::string tune_key(const jam_ctx *ctx, int n, const int32_t *geom_idx) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  for (int m = 0; m < n; ++m) {
    const GeomHost &g = ctx->gh[geom_idx[m]];
    mix((uint64_t)g.n_ux | ((uint64_t)g.n_uy << 20) | ((uint64_t)g.T << 40));
  }
  char buf[128];
  snprintf(buf, sizeof buf, "gfx950/v2/n%d/%016llx", n, (unsigned long long)h);
  return buf;
}

void load_tune_file(jam_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  FILE *f = fopen(ctx->tune_path.c_str(), "r");
  if (!f) return;
  char key[160];
  Tune t;
  while (fscanf(f, "%159s %d %d %d %d", key, &t.rule, &t.tau, &t.gran, &t.launch) == 5)
    ctx->tuned.push_back({key, t});
  fclose(f);
}

void save_tune_file(const jam_ctx *ctx) {
  if (ctx->tune_path.empty()) return;
  FILE *f = fopen(ctx->tune_path.c_str(), "w");
  if (!f) return;
  for (auto &e : ctx->tuned)
    fprintf(f, "%s %d %d %d %d\n", e.first.c_str(), e.second.rule, e.second.tau, e.second.gran,
            e.second.launch);
  fclose(f);
}

jam_status autotune(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, Tune &best) {
  std::vector<Tune> cands;
  Tune base;
  const int g0 = default_gran(ctx, n, geom_idx, base);
  for (int launch = 0; launch < 2; ++launch)
    for (int tau : {0, 1 << 30})
      for (double mul : {0.5, 0.75, 1.0, 1.5, 2.0}) {
        Tune t;
        t.rule = 1;
        t.tau = tau;
        t.gran = std::max(1, (int)std::lround(g0 * mul));
        t.launch = launch;
        cands.push_back(t);
      }
  {
    Tune t;
    t.rule = 0;
    t.gran = 0;
    cands.push_back(t);
  }
  std::vector<std::unique_ptr<Plan>> plans(cands.size());
  size_t ws_max = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    const jam_status s = build_plan(ctx, n, geom_idx, cands[i], plans[i]);
    if (s != JAM_OK) return s;
    ws_max = std::max(ws_max, plans[i]->ws_fwd);
  }
  int64_t nl = 0;
  for (int m = 0; m < n; ++m) nl += ctx->gh[geom_idx[m]].K;
  void *ws = nullptr, *prm = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    if (prm) (void)hipFree(prm);
    if (ws) (void)hipFree(ws);
  };
  std::vector<double> host(3 * (size_t)n + nl, 0.0);
  for (int m = 0; m < n; ++m) {
    host[m] = kPi / 2;                 // inclination
    host[n + m] = 1.0;                 // mass scale
    host[2 * n + m] = 1.0e8;           // BH mass
  }
  if (hipMalloc(&ws, ws_max) != hipSuccess || hipMalloc(&prm, host.size() * 8) != hipSuccess ||
      hipStreamCreate(&st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess ||
      hipMemcpy(prm, host.data(), host.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    cleanup();
    return fail(JAM_E_DEVICE, "autotune: device allocation failed");
  }
  const double *pp = (const double *)prm;
  const jam::ParamsDev pd{pp, pp + n, pp + 2 * n, pp + 3 * n, nullptr, nullptr};
  double best_ms = 1e300;
  size_t best_i = 0;
  for (size_t i = 0; i < cands.size(); ++i) {
    Plan *p = plans[i].get();
    char *w = (char *)ws;
    float ms = 0.f, tot = 0.f;
    for (int rep = 0; rep < 3; ++rep) {
      launch_forward_maps(ctx, p, pd, nullptr, w, st, false, true);
      (void)hipEventRecord(e0, st);
      if (p->tune.map)
        jam::launch_num_map(ctx->d_geoms, p->d_models, p->d_num, p->n_num,
                            (const float4 *)(w + p->off_terms), (const int *)(w + p->off_status),
                            (double *)(w + p->off_part),
                            p->tune.launch == 1 ? (int *)(w + p->off_queue) : nullptr,
                            p->grid_num, st);
      else
        jam::launch_num(ctx->d_geoms, p->d_models, p->d_num, p->n_num,
                        (const float4 *)(w + p->off_terms), (const double *)(w + p->off_gauss),
                        (const int *)(w + p->off_status),
                        (double *)(w + p->off_part), p->tune.launch == 1 ? (int *)(w + p->off_queue) : nullptr,
                        p->grid_num, p->tune.rule == 1, st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        cleanup();
        return fail(JAM_E_DEVICE, "autotune: timing failed");
      }
      if (rep > 0) tot += ms;    // first run warms caches and clocks
    }
    if (tot < best_ms) {
      best_ms = tot;
      best_i = i;
    }
  }
  const hipError_t e = hipGetLastError();
  cleanup();
  if (e != hipSuccess) return fail(JAM_E_DEVICE, "autotune: %s", hipGetErrorString(e));
  best = plans[best_i]->tune;
  return JAM_OK;
}

jam_status get_plan_impl(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, Plan *&out) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  if (n < 1) return fail(JAM_E_INVALID_ARG, "batch size must be >= 1");
  if (!geom_idx) return fail(JAM_E_INVALID_ARG, "geom_idx is NULL");
  for (int m = 0; m < n; ++m)
    if (geom_idx[m] < 0 || geom_idx[m] >= (int)ctx->gh.size())
      return fail(JAM_E_INVALID_ARG, "geom_idx[%d] = %d out of range", m, geom_idx[m]);
  for (auto itp = ctx->plans.begin(); itp != ctx->plans.end(); ++itp) {
    Plan *p = itp->get();
    if (p->n == n && std::equal(p->key.begin(), p->key.end(), geom_idx)) {
      if (itp != ctx->plans.begin()) ctx->plans.splice(ctx->plans.begin(), ctx->plans, itp);
      out = p;
      return JAM_OK;
    }
  }
  Tune t;
  if (ctx->opt.form == 1) t.rule = 0;
  if (ctx->opt.launch == 1) t.launch = 1;
  if (ctx->opt.form == 0 && ctx->opt.autotune) {
    const std::string key = tune_key(ctx, n, geom_idx);
    bool found = false;
    for (auto &e : ctx->tuned)
      if (e.first == key) {
        t = e.second;
        found = true;
        break;
      }
    if (!found) {
      const jam_status s = autotune(ctx, n, geom_idx, t);
      if (s != JAM_OK) return s;
      ctx->tuned.push_back({key, t});
      save_tune_file(ctx);
    }
  }
  std::unique_ptr<Plan> p;
  const jam_status s = build_plan(ctx, n, geom_idx, t, p);
  if (s != JAM_OK) return s;
  out = p.get();
  ctx->plans.push_front(std::move(p));
  while (ctx->plans.size() > kMaxPlans) ctx->plans.pop_back();
  return JAM_OK;
}

// The plan of a batch composition, built (and autotuned) at its first use;
// host memory exhaustion while building it is returned as a status.
jam_status get_plan(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, Plan *&out) {
  try {
    return get_plan_impl(ctx, n, geom_idx, out);
  } catch (const std::bad_alloc &) {
    return fail(JAM_E_UNSUPPORTED, "host memory exhausted while preparing a batch of %d", n);
  } catch (...) {
    return fail(JAM_E_UNSUPPORTED, "unexpected host error while preparing a batch of %d", n);
  }
}

// A prepared plan of this composition, or NULL; builds nothing.
Plan *find_plan(jam_ctx *ctx, int32_t n, const int32_t *geom_idx) {
  for (auto &pl : ctx->plans)
    if (pl->n == n && std::equal(pl->key.begin(), pl->key.end(), geom_idx)) return pl.get();
  return nullptr;
}

// Switch to the context's device for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

jam_status check_batch(const jam_batch *b) {
  if (!b) return fail(JAM_E_INVALID_ARG, "batch is NULL");
  if (!b->inc || !b->mass_scale || !b->m_bh || !b->beta)
    return fail(JAM_E_INVALID_ARG, "batch inc, mass_scale, m_bh and beta are required");
  return JAM_OK;
}

jam_status check_ws(void *ws, size_t ws_bytes, size_t need) {
  if (need > ws_bytes) return fail(JAM_E_WORKSPACE, "workspace of %zu bytes < %zu needed", ws_bytes, need);
  if (!ws) return fail(JAM_E_WORKSPACE, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(JAM_E_WORKSPACE, "workspace must be 256-byte aligned");
  return JAM_OK;
}

// Replay the plan's captured graph `which` (0 forward, 1 adjoint) if it was
// recorded with exactly these pointers; otherwise record it first on the
// context's capture stream.  `record` launches the sequence on a stream.
template <typename F>
jam_status run_graph(jam_ctx *ctx, Plan *p, int which, const GraphKey &key, hipStream_t st,
                     F record) {
  if (!p->gexec[which] || !(p->gkey[which] == key)) {
    if (p->gexec[which]) {
      HIP_TRY(hipGraphExecDestroy(p->gexec[which]));
      p->gexec[which] = nullptr;
    }
    if (!ctx->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    record(ctx->cap_stream);
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamEndCapture(ctx->cap_stream, &graph));
    const hipError_t e = hipGraphInstantiate(&p->gexec[which], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      p->gexec[which] = nullptr;
      return fail(JAM_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    p->gkey[which] = key;
  }
  HIP_TRY(hipGraphLaunch(p->gexec[which], st));
  return JAM_OK;
}

// Inverse of a symmetric positive definite n x n matrix (row-major) by its
// Cholesky factor C = L L^T: L^-1 by forward substitution, then
// C^-1 = L^-T L^-1, written symmetric.  False if C is not positive definite.
bool spd_inverse(int n, const double *c, std::vector<double> &inv) {
  std::vector<long double> L((size_t)n * n, 0.0L), Li((size_t)n * n, 0.0L);
  for (int j = 0; j < n; ++j) {
    long double d = c[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
    if (!(d > 0.0L)) return false;
    const long double ljj = std::sqrt(d);
    L[(size_t)j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      long double v = c[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
      L[(size_t)i * n + j] = v / ljj;
    }
  }
  for (int j = 0; j < n; ++j) {          // column j of L^-1
    Li[(size_t)j * n + j] = 1.0L / L[(size_t)j * n + j];
    for (int i = j + 1; i < n; ++i) {
      long double v = 0.0L;
      for (int k = j; k < i; ++k) v += L[(size_t)i * n + k] * Li[(size_t)k * n + j];
      Li[(size_t)i * n + j] = -v / L[(size_t)i * n + i];
    }
  }
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = i; j < n; ++j) {
      long double v = 0.0L;
      for (int k = j; k < n; ++k) v += Li[(size_t)k * n + i] * Li[(size_t)k * n + j];
      inv[(size_t)i * n + j] = inv[(size_t)j * n + i] = (double)v;
    }
  return true;
}

// Constants of the one-dimensional MGE transform: Euler nodes
// beta_k = P ln(10)/3 + i pi k and signed binomial weights (-1)^k xi_k,
// k = 0..2P, and per Gaussian the factor w_n dlog(sigma) 2 10^(P/3) that,
// with the transform's 2 sqrt(2 pi) and the expansion's 1/sqrt(2 pi), turns
// sum_k (-1)^k xi_k Re F(sigma_n chi_k) into the peak amplitude.
jam_status mge_constants(int32_t n_comp, int32_t n_sigma, const double *sigma, int32_t P,
                         jam::MgeConst &k) {
  if (n_comp < 1 || n_comp > jam::kMgeMaxComp)
    return fail(JAM_E_INVALID_ARG, "n_comp must be in [1, %d]", jam::kMgeMaxComp);
  if (n_sigma < 1 || n_sigma > jam::kMgeMaxSigma)
    return fail(JAM_E_INVALID_ARG, "n_sigma must be in [1, %d]", jam::kMgeMaxSigma);
  if (P < 1 || 2 * P + 1 > jam::kMgeMaxTerms)
    return fail(JAM_E_INVALID_ARG, "euler_p must be in [1, %d]", (jam::kMgeMaxTerms - 1) / 2);
  if (!sigma) return fail(JAM_E_INVALID_ARG, "sigma is NULL");
  for (int n = 0; n < n_sigma; ++n) {
    if (!(sigma[n] > 0.0) || !std::isfinite(sigma[n]))
      return fail(JAM_E_INVALID_ARG, "sigma[%d] must be positive and finite", n);
    if (n > 0 && !(sigma[n] > sigma[n - 1]))
      return fail(JAM_E_INVALID_ARG, "sigma must be strictly increasing");
  }
  std::memset(&k, 0, sizeof k);
  k.n_terms = 2 * P + 1;
  k.n_sigma = n_sigma;
  const long double pi = 3.141592653589793238462643383279502884L;
  k.beta_re = (double)(P * std::log(10.0L) / 3.0L);
  long double xi[jam::kMgeMaxTerms] = {};
  xi[0] = 0.5L;
  for (int j = 1; j <= P; ++j) xi[j] = 1.0L;
  const long double pw = std::ldexp(1.0L, -P);
  xi[2 * P] = pw;
  long double binom = 1.0L;   // binom(P, j), built up with j
  for (int j = 1; j < P; ++j) {
    binom = binom * (P - j + 1) / j;
    xi[2 * P - j] = xi[2 * P - j + 1] + pw * binom;
  }
  for (int j = 0; j <= 2 * P; ++j) {
    k.beta_im[j] = (double)(pi * j);
    k.eta[j] = (double)((j % 2 ? -xi[j] : xi[j]));
  }
  const long double dlog =
      n_sigma > 1 ? (std::log((long double)sigma[n_sigma - 1]) - std::log((long double)sigma[0])) /
                        (n_sigma - 1)
                  : 1.0L;
  const long double f = 2.0L * std::pow(10.0L, P / 3.0L) * dlog;
  for (int n = 0; n < n_sigma; ++n) {
    k.sigma2[n] = sigma[n] * sigma[n];
    const long double w = (n_sigma > 1 && (n == 0 || n == n_sigma - 1)) ? 0.5L : 1.0L;
    k.scale[n] = (double)(w * f);
  }
  return JAM_OK;
}

jam_status check_kinematics(const jam_ctx *ctx, const jam_batch *b) {
  for (int m = 0; m < b->n; ++m) {
    const int gi = b->geom_idx[m];
    if (gi < 0 || gi >= (int)ctx->kin_host.size())
      return fail(JAM_E_INVALID_ARG, "geom_idx[%d] out of range", m);
    if (!ctx->kin_host[gi].prec)
      return fail(JAM_E_INVALID_ARG, "no kinematics set for geometry %d (model %d)", gi, m);
  }
  return JAM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI.
// ---------------------------------------------------------------------------
extern "C" {

const char *jam_last_error(void) { return g_err.c_str(); }

jam_status jam_timing(jam_ctx *ctx, int32_t enable, double *numerator_ms,
                      int64_t *numerator_launches, double *sens_ms, int64_t *sens_launches) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  KernelTimer *ts[2] = {&ctx->t_num, &ctx->t_sens};
  if (enable) {
    for (KernelTimer *t : ts) {
      if (t->start.empty()) {
        t->start.resize(KernelTimer::kCap);
        t->stop.resize(KernelTimer::kCap);
        for (int i = 0; i < KernelTimer::kCap; ++i) {
          HIP_TRY(hipEventCreate(&t->start[i]));
          HIP_TRY(hipEventCreate(&t->stop[i]));
        }
      }
      t->used = 0;
      t->on = true;
    }
    return JAM_OK;
  }
  double ms[2] = {0.0, 0.0};
  for (int k = 0; k < 2; ++k) {
    KernelTimer *t = ts[k];
    t->on = false;
    for (int i = 0; i < t->used; ++i) {
      HIP_TRY(hipEventSynchronize(t->stop[i]));
      float e = 0.f;
      HIP_TRY(hipEventElapsedTime(&e, t->start[i], t->stop[i]));
      ms[k] += e;
    }
  }
  if (numerator_ms) *numerator_ms = ms[0];
  if (numerator_launches) *numerator_launches = ctx->t_num.used;
  if (sens_ms) *sens_ms = ms[1];
  if (sens_launches) *sens_launches = ctx->t_sens.used;
  return JAM_OK;
}

jam_status jam_gauss_legendre(int32_t n, double *nodes, double *weights) {
  if (n < 1 || n > kMaxNu) return fail(JAM_E_INVALID_ARG, "n must be in [1, 1024]");
  if (!nodes || !weights) return fail(JAM_E_INVALID_ARG, "output arrays are NULL");
  gauss_legendre01(n, nodes, weights);
  return JAM_OK;
}

jam_status jam_create(int32_t n_geom, const jam_geometry *geoms, const jam_options *opt,
                      jam_ctx **out) {
  g_err.clear();
  if (!out) return fail(JAM_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_geom < 1 || !geoms) return fail(JAM_E_INVALID_ARG, "need at least one geometry");
  for (int i = 0; i < n_geom; ++i) {
    const jam_status s = validate(geoms[i], i);
    if (s != JAM_OK) return s;
  }
  if (opt && (opt->form < 0 || opt->form > 2))
    return fail(JAM_E_INVALID_ARG, "options.form must be 0, 1 or 2");
  if (opt && (opt->launch < 0 || opt->launch > 1))
    return fail(JAM_E_INVALID_ARG, "options.launch must be 0 or 1");
  if (opt && (opt->alignment < 0 || opt->alignment > 1))
    return fail(JAM_E_INVALID_ARG, "options.alignment must be 0 or 1");
  auto ctx = std::make_unique<jam_ctx>();
  if (opt) ctx->opt = *opt;
  if (opt && opt->tune_cache) ctx->tune_path = opt->tune_cache;
  ctx->opt.tune_cache = nullptr;   // the path is copied
  HIP_TRY(hipGetDevice(&ctx->device));
  HIP_TRY(hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device));
  ctx->occ_num_pix = jam::occupancy_num(false);
  ctx->occ_num_mfma = jam::occupancy_num(true);
  ctx->occ_sens = jam::occupancy_sens();
  {
    const jam_status s = scratch_address(ctx->device, &ctx->scratch);
    if (s != JAM_OK) return s;
  }
  load_tune_file(ctx.get());
  ctx->gh.resize(n_geom);
  {
    const unsigned nt = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    std::vector<int> failed(nt, -1);
    for (unsigned t = 0; t < nt; ++t)
      pool.emplace_back([&, t] {
        for (int i = (int)t; i < n_geom; i += (int)nt) {
          try {
            build_geometry(geoms[i], ctx->gh[i]);
            build_spherical(ctx->gh[i]);
          } catch (...) {   // out of host memory: reported below, never past the thread
            failed[t] = i;
            return;
          }
        }
      });
    for (auto &th : pool) th.join();
    for (unsigned t = 0; t < nt; ++t)
      if (failed[t] >= 0)
        return fail(JAM_E_UNSUPPORTED, "geometry %d: host memory exhausted while building it",
                    failed[t]);
  }
  // device arena: GeomDev array then every geometry's arrays
  size_t off = align256(sizeof(jam::GeomDev) * n_geom);
  struct Offs { size_t ls, lq, li, ms, mq, mS, u, w, xs, ys, ux, uy, bp, bpix, bw, pp, pb, pw; };
  std::vector<Offs> offs(n_geom);
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + std::max<size_t>(bytes, 8)); return o; };
  for (int i = 0; i < n_geom; ++i) {
    const GeomHost &g = ctx->gh[i];
    Offs &o = offs[i];
    o.ls = take(8 * g.K); o.lq = take(8 * g.K); o.li = take(8 * g.K);
    o.ms = take(8 * g.J); o.mq = take(8 * g.J); o.mS = take(8 * g.J);
    o.u = take(8 * g.n_u); o.w = take(8 * g.n_u);
    o.xs = take(8 * g.n_ux); o.ys = take(8 * g.n_uy);
    o.ux = take(4 * g.nxp); o.uy = take(4 * g.nyp);
    o.bp = take(4 * g.bin_ptr.size()); o.bpix = take(4 * g.bin_pix.size()); o.bw = take(8 * g.bin_w.size());
    o.pp = take(4 * g.pix_ptr.size()); o.pb = take(4 * g.pix_bin.size()); o.pw = take(8 * g.pix_w.size());
  }
  std::vector<char> stage(off, 0);
  HIP_TRY(hipMalloc(&ctx->arena, off));
  char *base = (char *)ctx->arena;
  std::vector<jam::GeomDev> gd(n_geom);
  auto put = [&](size_t o, const void *src, size_t bytes) {
    if (bytes) std::memcpy(stage.data() + o, src, bytes);
    return base + o;
  };
  for (int i = 0; i < n_geom; ++i) {
    const GeomHost &g = ctx->gh[i];
    const Offs &o = offs[i];
    jam::GeomDev &d = gd[i];
    d.K = g.K; d.J1 = g.J1; d.n_u = g.n_u; d.T = g.T;
    d.n_ux = g.n_ux; d.n_uy = g.n_uy; d.n_pix = g.n_pix; d.n_bins = g.n_bins;
    d.nxp = g.nxp; d.nyp = g.nyp; d.pad0 = d.pad1 = 0;
    d.s_pc = g.s_pc; d.bh_sigma = g.bh_sigma;
    d.lum_sigma = (const double *)put(o.ls, g.lum_sigma.data(), 8 * g.K);
    d.lum_q = (const double *)put(o.lq, g.lum_q.data(), 8 * g.K);
    d.lum_I0 = (const double *)put(o.li, g.lum_I0.data(), 8 * g.K);
    d.mass_sigma = (const double *)put(o.ms, g.mass_sigma.data(), 8 * g.J);
    d.mass_q = (const double *)put(o.mq, g.mass_q.data(), 8 * g.J);
    d.mass_S0 = (const double *)put(o.mS, g.mass_S0.data(), 8 * g.J);
    d.u = (const double *)put(o.u, g.u.data(), 8 * g.n_u);
    d.w = (const double *)put(o.w, g.w.data(), 8 * g.n_u);
    d.xs = (const double *)put(o.xs, g.xs.data(), 8 * g.n_ux);
    d.ys = (const double *)put(o.ys, g.ys.data(), 8 * g.n_uy);
    d.ux = (const int *)put(o.ux, g.ux.data(), 4 * g.nxp);
    d.uy = (const int *)put(o.uy, g.uy.data(), 4 * g.nyp);
    d.bin_ptr = (const int *)put(o.bp, g.bin_ptr.data(), 4 * g.bin_ptr.size());
    d.bin_pix = (const int *)put(o.bpix, g.bin_pix.data(), 4 * g.bin_pix.size());
    d.bin_w = (const double *)put(o.bw, g.bin_w.data(), 8 * g.bin_w.size());
    d.pix_ptr = (const int *)put(o.pp, g.pix_ptr.data(), 4 * g.pix_ptr.size());
    d.pix_bin = (const int *)put(o.pb, g.pix_bin.data(), 4 * g.pix_bin.size());
    d.pix_w = (const double *)put(o.pw, g.pix_w.data(), 8 * g.pix_w.size());
    d.sph_lnr0 = g.sph_lnr0;
    d.sph_dlnr = g.sph_dlnr;
    d.sph_sig_max = g.sph_sig_max;
    for (int q = 0; q < 8; ++q) {
      d.gl8_x[q] = g.gl8_x[q];
      d.gl8_w[q] = g.gl8_w[q];
    }
  }
  std::memcpy(stage.data(), gd.data(), sizeof(jam::GeomDev) * n_geom);
  HIP_TRY(hipMemcpy(ctx->arena, stage.data(), off, hipMemcpyHostToDevice));
  ctx->d_geoms = (jam::GeomDev *)ctx->arena;
  ctx->kin_buf.assign(n_geom, nullptr);
  ctx->kin_host.assign(n_geom, jam::KinDev{nullptr, nullptr});
  HIP_TRY(hipMalloc(&ctx->d_kin, sizeof(jam::KinDev) * n_geom));
  HIP_TRY(hipMemcpy(ctx->d_kin, ctx->kin_host.data(), sizeof(jam::KinDev) * n_geom,
                    hipMemcpyHostToDevice));
  *out = ctx.release();
  return JAM_OK;
}

void jam_destroy(jam_ctx *ctx) { delete ctx; }

jam_status jam_batch_sizes(const jam_ctx *ctx, int32_t n, const int32_t *geom_idx,
                           int64_t *n_bins_total, int64_t *n_lum_total, int64_t *n_mass_total) {
  if (!ctx || n < 1 || !geom_idx) return fail(JAM_E_INVALID_ARG, "invalid arguments");
  int64_t b = 0, l = 0, ms = 0;
  for (int m = 0; m < n; ++m) {
    if (geom_idx[m] < 0 || geom_idx[m] >= (int)ctx->gh.size())
      return fail(JAM_E_INVALID_ARG, "geom_idx[%d] out of range", m);
    const GeomHost &g = ctx->gh[geom_idx[m]];
    b += g.n_bins;
    l += g.K;
    ms += g.J;
  }
  if (n_bins_total) *n_bins_total = b;
  if (n_lum_total) *n_lum_total = l;
  if (n_mass_total) *n_mass_total = ms;
  return JAM_OK;
}

jam_status jam_prepare(jam_ctx *ctx, int32_t n, const int32_t *geom_idx) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  return get_plan(ctx, n, geom_idx, p);
}

jam_status jam_workspace_size(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, int32_t with_vjp,
                              size_t *bytes) {
  if (!bytes) return fail(JAM_E_INVALID_ARG, "bytes is NULL");
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  const jam_status s = get_plan(ctx, n, geom_idx, p);
  if (s != JAM_OK) return s;
  *bytes = with_vjp ? p->ws_vjp : p->ws_fwd;
  return JAM_OK;
}

jam_status jam_eval_batch(jam_ctx *ctx, const jam_batch *batch, double *vrms2, int32_t *status,
                          void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!vrms2) return fail(JAM_E_INVALID_ARG, "vrms2 is NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  if ((s = check_ws(ws, ws_bytes, p->ws_fwd)) != JAM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if (ctx->opt.graph) {
    const GraphKey k({batch->inc, batch->mass_scale, batch->m_bh, batch->beta, batch->lum_I0,
                      batch->mass_S0, vrms2, status, ws}, ws_bytes);
    const jam_batch b = *batch;
    s = run_graph(ctx, p, 0, k, st, [&](hipStream_t cs) {
      launch_eval(ctx, p, &b, vrms2, status, w, cs, true);
    });
    if (s != JAM_OK) return s;
  } else {
    launch_eval(ctx, p, batch, vrms2, status, w, st, false);
  }
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_eval(jam_ctx *ctx, const jam_batch *one, double *vrms2, int32_t *status, void *ws,
                    size_t ws_bytes, void *stream) {
  if (one && one->n != 1) return fail(JAM_E_INVALID_ARG, "jam_eval takes exactly one model");
  return jam_eval_batch(ctx, one, vrms2, status, ws, ws_bytes, stream);
}

jam_status jam_eval_batch_noalloc(jam_ctx *ctx, const jam_batch *batch, double *vrms2,
                                  int32_t *status, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!vrms2) return fail(JAM_E_INVALID_ARG, "vrms2 is NULL");
  if (batch->n < 1 || !batch->geom_idx) return fail(JAM_E_INVALID_ARG, "invalid batch");
  if (!ctx->scratch) return fail(JAM_E_DEVICE, "fixed scratch memory is not available");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = find_plan(ctx, batch->n, batch->geom_idx);
  if (!p)
    return fail(JAM_E_INVALID_ARG,
                "batch composition not prepared: call jam_prepare (which allocates) first");
  if (p->ws_fwd > kScratchBytes)
    return fail(JAM_E_WORKSPACE, "composition needs %zu bytes of workspace, above the %zu bytes "
                "of fixed scratch", p->ws_fwd, kScratchBytes);
  // eager launches only (instantiating a graph allocates); no timing events
  launch_eval(ctx, p, batch, vrms2, status, (char *)ctx->scratch, (hipStream_t)stream, true);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_eval_maps(jam_ctx *ctx, const jam_batch *batch, double *N_map, double *I_map,
                         int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!N_map || !I_map) return fail(JAM_E_INVALID_ARG, "map outputs are NULL");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  if ((s = check_ws(ws, ws_bytes, p->ws_fwd)) != JAM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  launch_forward_maps(ctx, p, params_of(batch), status, w, st, true, false);
  jam::launch_maps(ctx->d_geoms, p->d_models, p->d_maps, p->n_maps, (const double *)(w + p->off_pix),
                   (const int *)(w + p->off_status), N_map, I_map, st);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_vjp(jam_ctx *ctx, const jam_batch *batch, const double *vrms2, const double *cot,
                   jam_grads *grads, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!cot || !grads) return fail(JAM_E_INVALID_ARG, "cot and grads are required");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  if ((s = check_ws(ws, ws_bytes, p->ws_vjp)) != JAM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if (ctx->opt.graph) {
    // gradient outputs are part of the recorded launches
    const GraphKey k({batch->inc, batch->mass_scale, batch->m_bh, batch->beta, batch->lum_I0,
                      batch->mass_S0, vrms2, cot, ws, grads->inc, grads->mass_scale, grads->m_bh,
                      grads->beta, grads->lum_I0, grads->mass_S0},
                     ws_bytes);
    const jam_batch b = *batch;
    const jam_grads g = *grads;
    s = run_graph(ctx, p, 1, k, st, [&](hipStream_t cs) {
      launch_vjp(ctx, p, &b, vrms2, cot, &g, w, cs, true);
    });
    if (s != JAM_OK) return s;
  } else {
    launch_vjp(ctx, p, batch, vrms2, cot, grads, w, st, false);
  }
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

static jam_status set_kinematics_impl(jam_ctx *ctx, int32_t geom, const double *vrms_obs,
                                      const double *cov) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  if (geom < 0 || geom >= (int)ctx->gh.size()) return fail(JAM_E_INVALID_ARG, "geometry %d out of range", geom);
  if (!vrms_obs || !cov) return fail(JAM_E_INVALID_ARG, "vrms_obs and cov are required");
  const int nb = ctx->gh[geom].n_bins;
  if (nb > jam::kChi2MaxBins)
    return fail(JAM_E_UNSUPPORTED, "chi^2 supports at most %d bins (geometry %d has %d)",
                jam::kChi2MaxBins, geom, nb);
  double cmax = 0.0;
  for (int i = 0; i < nb; ++i) {
    if (!std::isfinite(vrms_obs[i])) return fail(JAM_E_INVALID_ARG, "vrms_obs[%d] is not finite", i);
    for (int j = 0; j < nb; ++j) {
      const double v = cov[(size_t)i * nb + j];
      if (!std::isfinite(v)) return fail(JAM_E_INVALID_ARG, "cov[%d][%d] is not finite", i, j);
      cmax = std::max(cmax, std::fabs(v));
    }
  }
  for (int i = 0; i < nb; ++i)
    for (int j = i + 1; j < nb; ++j)
      if (std::fabs(cov[(size_t)i * nb + j] - cov[(size_t)j * nb + i]) > 1e-12 * cmax)
        return fail(JAM_E_INVALID_ARG, "cov is not symmetric at (%d, %d)", i, j);
  std::vector<double> host((size_t)nb + (size_t)nb * nb);
  std::vector<double> inv;
  if (!spd_inverse(nb, cov, inv)) return fail(JAM_E_INVALID_ARG, "cov is not positive definite");
  std::copy(vrms_obs, vrms_obs + nb, host.begin());
  std::copy(inv.begin(), inv.end(), host.begin() + nb);
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  HIP_TRY(hipDeviceSynchronize());      // no evaluation may still read the old buffer
  void *buf = nullptr;
  HIP_TRY(hipMalloc(&buf, host.size() * sizeof(double)));
  if (hipMemcpy(buf, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(buf);
    return fail(JAM_E_DEVICE, "copy of the kinematics failed");
  }
  const jam::KinDev kd{(const double *)buf, (const double *)buf + nb};
  if (hipMemcpy(ctx->d_kin + geom, &kd, sizeof kd, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(buf);
    return fail(JAM_E_DEVICE, "copy of the kinematics table failed");
  }
  if (ctx->kin_buf[geom]) HIP_TRY(hipFree(ctx->kin_buf[geom]));
  ctx->kin_buf[geom] = buf;
  ctx->kin_host[geom] = kd;
  return JAM_OK;
}

jam_status jam_set_kinematics(jam_ctx *ctx, int32_t geom, const double *vrms_obs,
                              const double *cov) {
  try {
    return set_kinematics_impl(ctx, geom, vrms_obs, cov);
  } catch (...) {
    return fail(JAM_E_UNSUPPORTED, "host memory exhausted while setting the kinematics");
  }
}

jam_status jam_chi2(jam_ctx *ctx, const jam_batch *batch, const double *vrms2, double *chi2,
                    double *dchi2, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  if (!batch || batch->n < 1 || !batch->geom_idx) return fail(JAM_E_INVALID_ARG, "invalid batch");
  if (!vrms2 || !chi2) return fail(JAM_E_INVALID_ARG, "vrms2 and chi2 are required");
  jam_status s = check_kinematics(ctx, batch);
  if (s != JAM_OK) return s;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  jam::launch_chi2(ctx->d_geoms, p->d_models, p->n, ctx->d_kin, vrms2, nullptr, chi2, nullptr,
                   dchi2, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_eval_chi2(jam_ctx *ctx, const jam_batch *batch, double *chi2, double *vrms2,
                         int32_t *status, void *ws, size_t ws_bytes, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!chi2) return fail(JAM_E_INVALID_ARG, "chi2 is NULL");
  if ((s = check_kinematics(ctx, batch)) != JAM_OK) return s;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  if ((s = check_ws(ws, ws_bytes, p->ws_fwd)) != JAM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  double *V = vrms2 ? vrms2 : (double *)(w + p->off_vfwd);
  auto record = [&](const jam_batch *b, hipStream_t cs, bool capturing) {
    launch_eval(ctx, p, b, V, status, w, cs, capturing);
    jam::launch_chi2(ctx->d_geoms, p->d_models, p->n, ctx->d_kin, V,
                     (const int *)(w + p->off_status), chi2, nullptr, nullptr, cs);
  };
  if (ctx->opt.graph) {
    const GraphKey k({batch->inc, batch->mass_scale, batch->m_bh, batch->beta, batch->lum_I0,
                      batch->mass_S0, V, status, ws, chi2, ctx->d_kin},
                     ws_bytes);
    const jam_batch b = *batch;
    s = run_graph(ctx, p, 2, k, st, [&](hipStream_t cs) { record(&b, cs, true); });
    if (s != JAM_OK) return s;
  } else {
    record(batch, st, false);
  }
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_vjp_chi2(jam_ctx *ctx, const jam_batch *batch, const double *vrms2,
                        const double *cot, jam_grads *grads, void *ws, size_t ws_bytes,
                        void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  jam_status s = check_batch(batch);
  if (s != JAM_OK) return s;
  if (!cot || !grads) return fail(JAM_E_INVALID_ARG, "cot and grads are required");
  if ((s = check_kinematics(ctx, batch)) != JAM_OK) return s;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  if ((s = get_plan(ctx, batch->n, batch->geom_idx, p)) != JAM_OK) return s;
  if ((s = check_ws(ws, ws_bytes, p->ws_vjp)) != JAM_OK) return s;
  hipStream_t st = (hipStream_t)stream;
  char *w = (char *)ws;
  if (ctx->opt.graph) {
    const GraphKey k({batch->inc, batch->mass_scale, batch->m_bh, batch->beta, batch->lum_I0,
                      batch->mass_S0, vrms2, cot, ws, grads->inc, grads->mass_scale, grads->m_bh,
                      grads->beta, grads->lum_I0, grads->mass_S0, ctx->d_kin},
                     ws_bytes);
    const jam_batch b = *batch;
    const jam_grads g = *grads;
    s = run_graph(ctx, p, 3, k, st, [&](hipStream_t cs) {
      launch_vjp(ctx, p, &b, vrms2, nullptr, &g, w, cs, true, cot);
    });
    if (s != JAM_OK) return s;
  } else {
    launch_vjp(ctx, p, batch, vrms2, nullptr, grads, w, st, false, cot);
  }
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_mge1d(int32_t n_prof, int32_t n_comp, const double *comp, int32_t n_sigma,
                     const double *sigma, int32_t euler_p, double *amp, void *stream) {
  if (n_prof < 1 || n_prof > (1 << 24)) return fail(JAM_E_INVALID_ARG, "n_prof must be in [1, 2^24]");
  if (!comp || !amp) return fail(JAM_E_INVALID_ARG, "comp and amp are required");
  jam::MgeConst k;
  const jam_status s = mge_constants(n_comp, n_sigma, sigma, euler_p, k);
  if (s != JAM_OK) return s;
  jam::launch_mge1d(n_prof, n_comp, comp, k, amp, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_mge1d_vjp(int32_t n_prof, int32_t n_comp, const double *comp, int32_t n_sigma,
                         const double *sigma, int32_t euler_p, const double *cot, double *grad,
                         void *stream) {
  if (n_prof < 1 || n_prof > (1 << 24)) return fail(JAM_E_INVALID_ARG, "n_prof must be in [1, 2^24]");
  if (!comp || !cot || !grad) return fail(JAM_E_INVALID_ARG, "comp, cot and grad are required");
  jam::MgeConst k;
  const jam_status s = mge_constants(n_comp, n_sigma, sigma, euler_p, k);
  if (s != JAM_OK) return s;
  jam::launch_mge1d_vjp(n_prof, n_comp, comp, k, cot, grad, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_beta_logistic(jam_ctx *ctx, const jam_batch *batch, const double *prof, double *beta,
                             void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  if (!batch || batch->n < 1 || !batch->geom_idx) return fail(JAM_E_INVALID_ARG, "invalid batch");
  if (!prof || !beta) return fail(JAM_E_INVALID_ARG, "prof and beta are required");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  const jam_status s = get_plan(ctx, batch->n, batch->geom_idx, p);
  if (s != JAM_OK) return s;
  jam::launch_beta_logistic(ctx->d_geoms, p->d_models, p->n, prof, beta, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_beta_logistic_vjp(jam_ctx *ctx, const jam_batch *batch, const double *prof,
                                 const double *cot, double *grad, void *stream) {
  if (!ctx) return fail(JAM_E_INVALID_ARG, "ctx is NULL");
  if (!batch || batch->n < 1 || !batch->geom_idx) return fail(JAM_E_INVALID_ARG, "invalid batch");
  if (!prof || !cot || !grad) return fail(JAM_E_INVALID_ARG, "prof, cot and grad are required");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  const jam_status s = get_plan(ctx, batch->n, batch->geom_idx, p);
  if (s != JAM_OK) return s;
  jam::launch_beta_logistic_vjp(ctx->d_geoms, p->d_models, p->n, prof, cot, grad,
                                (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return JAM_OK;
}

jam_status jam_plan_info(jam_ctx *ctx, int32_t n, const int32_t *geom_idx, int32_t *info) {
  if (!ctx || !info) return fail(JAM_E_INVALID_ARG, "invalid arguments");
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return fail(JAM_E_DEVICE, "cannot select the context's device");
  Plan *p = nullptr;
  const jam_status s = get_plan(ctx, n, geom_idx, p);
  if (s != JAM_OK) return s;
  info[0] = p->tune.rule;
  info[1] = p->tune.tau;
  info[2] = p->tune.gran;
  info[3] = p->tune.launch;
  info[4] = p->n_num;
  info[5] = p->grid_num;
  info[6] = p->n_sens + p->n_sensw + p->n_adj;
  info[7] = (p->n_sens ? p->grid_sens : 0) + p->n_sensw + p->n_adj;
  info[8] = p->spherical ? 3 : (p->tune.rule == 0 ? 0 : (p->tune.map ? 2 : 1));
  return JAM_OK;
}

}  // extern "C"
