// C-ABI of the mcrt library: context set-up (FP64 tables built on the host),
// entry points and error handling.  The kernels live in trace_*.hip and
// pda.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mcrt_internal.h"

namespace {

// CODATA 2018, cgs
constexpr double H_PL = 6.62607015e-27;
constexpr double K_B = 1.380649e-16;
constexpr double C_L = 2.99792458e10;
constexpr double SIG_SB = 5.670374419e-5;
constexpr double PI = 3.14159265358979323846;

thread_local std::string g_last_error;

// ------------------------------------------------------------------------
// Planck bin integrals in closed series form.  With x = h nu / (k T),
//   int_{nu_a}^{nu_b} B_nu dnu = 2 k^4 T^4 / (h^3 c^2) * F,
//   F = int_{x_a}^{x_b} t^3 / (e^t - 1) dt.
// For small arguments I(x) = int_0^x t^3/(e^t-1) dt = sum_n a_n x^(n+3)/(n+3)
// with t/(e^t-1) = sum_n a_n t^n (a_0 = 1, a_1 = -1/2,
// a_2m = (-1)^(m+1) 2 zeta(2m) / (2 pi)^(2m), odd a_n = 0 beyond n = 1);
// for x >= 2 the tail J(x) = int_x^inf = sum_n e^(-n x) (x^3/n + 3x^2/n^2 +
// 6x/n^3 + 6/n^4).  The T-derivative follows from d/dT [T^4 F(x_a, x_b)].
// ------------------------------------------------------------------------
struct Planck {
  double a[64];
  Planck() {
    for (int n = 0; n < 64; ++n) a[n] = 0.0;
    a[0] = 1.0;
    a[1] = -0.5;
    for (int m = 1; 2 * m < 64; ++m) {
      double zeta;
      if (m == 1) zeta = PI * PI / 6.0;
      else if (m == 2) zeta = PI * PI * PI * PI / 90.0;
      else {
        zeta = 0.0;
        for (int k = 2000; k >= 1; --k) zeta += std::pow((double)k, -2.0 * m);
      }
      double v = 2.0 * zeta / std::pow(2.0 * PI, 2.0 * m);
      a[2 * m] = (m % 2 == 1) ? v : -v;
    }
  }
  double I_small(double x) const {  // x <= 2
    double s = 0.0, xp = x * x * x;
    for (int n = 0; n < 64; ++n) {
      s += a[n] * xp / (n + 3);
      xp *= x;
    }
    return s;
  }
  static double J_tail(double x) {  // x >= 2
    double s = 0.0;
    for (int n = 1; n < 200; ++n) {
      double e = std::exp(-n * x);
      if (e == 0.0) break;
      double dn = n;
      double t = e * (x * x * x / dn + 3.0 * x * x / (dn * dn) + 6.0 * x / (dn * dn * dn) +
                      6.0 / (dn * dn * dn * dn));
      s += t;
      if (t < 1e-18 * s) break;
    }
    return s;
  }
  double F(double xa, double xb) const {  // xa < xb
    const double x0 = 2.0;
    if (xa >= x0) return J_tail(xa) - J_tail(xb);
    if (xb <= x0) return I_small(xb) - I_small(xa);
    return (I_small(x0) - I_small(xa)) + (J_tail(x0) - J_tail(xb));
  }
  static double f(double x) {  // x^3 / (e^x - 1)
    if (x > 700.0) return 0.0;
    return x * x * x * std::exp(-x) / (-std::expm1(-x));
  }
  // bin [lam_lo, lam_hi] (cm): B-bar and dB-bar/dT
  void bin(double lam_lo, double lam_hi, double T, double& B, double& dB) const {
    if (!(T > 0.0)) {
      B = dB = 0.0;
      return;
    }
    double xa = H_PL * C_L / (lam_hi * K_B * T);
    double xb = H_PL * C_L / (lam_lo * K_B * T);
    double pre = 2.0 * std::pow(K_B * T, 4) / (H_PL * H_PL * H_PL * C_L * C_L);
    double Fv = F(xa, xb);
    B = pre * Fv;
    dB = pre / T * (4.0 * Fv - xb * f(xb) + xa * f(xa));
  }
};

// MRW escape-time law: survival P(s) and its complement 1 - P (s = D c t / R0^2).
double mrw_P(double s) {
  double sum = 0.0;
  for (int n = 1; n < 100; ++n) {
    double e = std::exp(-(double)n * n * PI * PI * s);
    sum += (n & 1) ? e : -e;
    if (e < 1e-20) break;
  }
  return 2.0 * sum;
}
double mrw_Q(double s) {  // 1 - P(s), theta-function form
  double sum = 0.0;
  for (int k = 0; k < 100; ++k) {
    double a = (2.0 * k + 1.0) * (2.0 * k + 1.0) / 4.0;
    double e = std::exp(-a / s);
    sum += e;
    if (e < 1e-20 * sum || e == 0.0) break;
  }
  return 2.0 / std::sqrt(PI * s) * sum;
}
// s with P(s) = P0, P0 = exp(-exp(v)), by bisection in log s
double mrw_solve_v(double v) {
  double q = std::exp(v);                // -ln P0
  double P0 = std::exp(-q);
  double Q0 = -std::expm1(-q);           // 1 - P0
  bool use_Q = Q0 < 0.5;
  double lo = 1e-4, hi = 1.0;
  auto above = [&](double s) {  // true if s is below the solution (P(s) > P0)
    return use_Q ? (mrw_Q(s) < Q0) : (mrw_P(s) > P0);
  };
  while (!above(lo)) lo *= 0.5;
  while (above(hi)) hi *= 2.0;
  for (int it = 0; it < 300; ++it) {
    double mid = std::sqrt(lo * hi);
    if (above(mid)) lo = mid; else hi = mid;
    if (hi / lo - 1.0 < 1e-15) break;
  }
  return std::sqrt(lo * hi);
}

int fail(mcrt_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_last_error = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                          \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(ctx, MCRT_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace mcrt {
void set_error(mcrt_ctx* ctx, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_last_error = msg;
}
int launch_trace_fp64(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s);
int launch_raytrace_image(mcrt_ctx* ctx, const double* T, const double* J, int n_inc,
                          const double* cos_i_host, int n_sub, int n_phi, double* img,
                          hipStream_t s);
int launch_visibility(mcrt_ctx* ctx, const double* img, int n_inc, const double* cos_i_host,
                      int n_sub, int n_phi, int n_base, const double* base_host, double distance,
                      double* V, hipStream_t s);
int launch_trace_fp32(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s);

TraceArgs make_trace_args(mcrt_ctx* ctx, uint64_t n_packets, uint64_t n_total, uint64_t seed,
                          uint64_t offset, const double* frozen_T, mcrt_packet_rec* recs,
                          int64_t n_recs) {
  TraceArgs a{};
  a.m = ctx->m;
  a.t = ctx->t;
  if (!ctx->opt.conv_split) a.t.E_half = nullptr;
  a.eps = ctx->L_star / (double)n_total;
  a.key0 = (uint32_t)seed;
  a.key1 = (uint32_t)(seed >> 32);
  a.offset = offset;
  a.n_packets = n_packets;
  a.next = ctx->d_next;
  a.mrw = ctx->opt.mrw;
  a.n_int_min = ctx->opt.n_int_min;
  a.gamma = ctx->opt.gamma;
  a.max_events = ctx->opt.max_events;
  a.frozen_T = frozen_T;
  a.T_coef = (ctx->opt.mrw_coef_T == 1 && ctx->have_T_prev) ? ctx->d_T_prev : nullptr;
  a.recs = recs;
  a.n_recs = n_recs;
  a.wave_events = ctx->opt.wave_events;
  a.g_asym = ctx->opt.g_asym;
  a.runahead = ctx->opt.wave_runahead != 0 && ctx->opt.g_asym == 0.0 && a.t.path == nullptr;
  if (ctx->opt.wave_events > 0 && ctx->d_tail) {
    a.tail = ctx->d_tail;
    a.tail_count = (unsigned int*)((char*)ctx->d_tail + (size_t)mcrt::TAIL_CAP * mcrt::TAIL_STATE_BYTES);
    a.tail_next = a.tail_count + 1;
    a.tail_cap = mcrt::TAIL_CAP;
    a.live_handoff = (unsigned)ctx->opt.handoff_live;  // 0: the launch's wavefronts
    // after the two counters: the live count (8-byte aligned) and the
    // wavefronts counted into it; the launch sets n_waves and live_handoff
    a.live = (long long*)(a.tail_count + 2);
    a.waves_in = (unsigned int*)(a.live + 1);
  }
  return a;
}

int launch_trace(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s) {
  if (ctx->opt.precision == MCRT_FP32) return launch_trace_fp32(ctx, a, s);
  return launch_trace_fp64(ctx, a, s);
}
}  // namespace mcrt

namespace mcrt {
double hydro_A(double M_star, double mu_mol) {
  const double G = 6.67430e-8, M_P = 1.67262192369e-24;
  return mu_mol * M_P * G * M_star / K_B;
}
}  // namespace mcrt

extern "C" {

void mcrt_default_options(mcrt_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->precision = MCRT_FP64;
  o->mrw = 0;
  o->gamma = 3.0;
  o->n_int_min = 20;
  o->n_T = 256;
  o->T_lo = 1.0;
  o->T_hi = 1.0e4;
  o->n_inc = 10;
  o->max_events = (int64_t)1 << 30;
  o->pda_visits = 100;
  o->pda_max_sweeps = 50;
  o->pda_tol = 1e-8;
  o->cg_max_iter = 20000;
  o->cg_tol = 1e-12;
  o->mrw_coef_T = 0;
  o->block_size = 0;
  o->blocks_per_cu = 0;
  o->pda_solver = 0;
  o->pda_precond = 1;
  o->wave_events = 2048;
  o->g_asym = 0.0;
  o->hydro_M_star = 0.0;
  o->hydro_mu = 2.3;
  o->pda_sigma = 0.0;
  o->conv_split = 0;
  o->j_tally = 0;
  o->wave_runahead = 0;
  o->handoff_live = 0;
}

static_assert(mcrt::TAIL_CAP == MCRT_TAIL_CAP, "hand-off buffer size as declared");

int mcrt_setup(mcrt_ctx** out, const mcrt_grid* grid, const mcrt_star* star,
               const mcrt_dust* dust, const double* rho, const mcrt_options* opt) {
  if (!out || !grid || !star || !dust || !rho || !opt) return fail(nullptr, MCRT_E_ARG, "null argument");
  *out = nullptr;
  const int n_r = grid->n_r, n_mu = grid->n_mu, nl = dust->n_lambda, ns = dust->n_species;
  if (n_r < 1 || n_mu < 1 || nl < 1 || ns < 1 || !grid->r_edges || !grid->mu_edges ||
      !dust->lambda_edges || !dust->kappa_abs || !dust->kappa_sca || !dust->mass_frac)
    return fail(nullptr, MCRT_E_ARG, "bad grid or dust descriptor");
  if ((long long)n_r * n_mu > (1ll << 30)) return fail(nullptr, MCRT_E_ARG, "grid too large");
  for (int i = 0; i < n_r; ++i)
    if (!(grid->r_edges[i + 1] > grid->r_edges[i])) return fail(nullptr, MCRT_E_ARG, "r_edges not increasing");
  if (!(grid->r_edges[0] > 0.0)) return fail(nullptr, MCRT_E_ARG, "r_edges[0] must be > 0");
  if (grid->mu_edges[0] != 0.0 || grid->mu_edges[n_mu] != 1.0)
    return fail(nullptr, MCRT_E_ARG, "mu_edges must run from 0 to 1");
  for (int j = 0; j < n_mu; ++j)
    if (!(grid->mu_edges[j + 1] > grid->mu_edges[j])) return fail(nullptr, MCRT_E_ARG, "mu_edges not increasing");
  for (int k = 0; k < nl; ++k)
    if (!(dust->lambda_edges[k + 1] > dust->lambda_edges[k]) || !(dust->lambda_edges[k] > 0.0))
      return fail(nullptr, MCRT_E_ARG, "lambda_edges not positive increasing");
  if (!(star->T_star > 0.0) || !(star->R_star > 0.0) || !(star->R_star < grid->r_edges[0]))
    return fail(nullptr, MCRT_E_ARG, "star must be hot and inside the inner hole");
  if (opt->n_T < 3 || !(opt->T_lo > 0.0) || !(opt->T_hi > opt->T_lo) || opt->n_inc < 1 ||
      opt->max_events < 1 || opt->n_int_min < 0 || !(opt->gamma >= 0.0) ||
      (opt->precision != MCRT_FP64 && opt->precision != MCRT_FP32) || opt->pda_solver < 0 ||
      opt->pda_solver > 2 || opt->pda_precond < 0 || opt->pda_precond > 1 || opt->wave_events < 0 ||
      !(opt->g_asym > -1.0 && opt->g_asym < 1.0) || !(opt->hydro_M_star >= 0.0) ||
      !(opt->hydro_mu > 0.0) || !(opt->pda_sigma >= 0.0) || opt->blocks_per_cu < 0 ||
      opt->wave_runahead < 0 || opt->wave_runahead > 1 || opt->handoff_live < 0 ||
      opt->handoff_live > mcrt::TAIL_CAP)
    return fail(nullptr, MCRT_E_ARG, "bad options");
  if (!(opt->block_size == 0 || opt->block_size == 512 ||
        ((opt->block_size == 256 || opt->block_size == 768) && opt->precision == MCRT_FP32)))
    return fail(nullptr, MCRT_E_ARG, "block_size: 0 or 512, or 256 or 768 with FP32 tracking");
  const int nc = n_r * n_mu;
  for (int c = 0; c < nc; ++c)
    if (!(rho[c] >= 0.0) || !std::isfinite(rho[c])) return fail(nullptr, MCRT_E_ARG, "rho must be finite and >= 0");

  mcrt_ctx* ctx = new mcrt_ctx();
  ctx->opt = *opt;
  ctx->n_r = n_r;
  ctx->n_mu = n_mu;
  ctx->n_lambda = nl;
  ctx->n_cells = nc;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return fail(nullptr, MCRT_E_HIP, "no HIP device");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) != hipSuccess) {
    delete ctx;
    return fail(nullptr, MCRT_E_HIP, "device properties");
  }
  ctx->n_cu = prop.multiProcessorCount;

  // ---------------- host tables (FP64)
  const int nT = opt->n_T;
  std::vector<double> kabs(nl, 0.0), ksca(nl, 0.0);
  double fsum = 0.0;
  for (int s = 0; s < ns; ++s) fsum += dust->mass_frac[s];
  if (!(fsum > 0.0)) {
    delete ctx;
    return fail(nullptr, MCRT_E_ARG, "mass fractions must sum to > 0");
  }
  for (int s = 0; s < ns; ++s)
    for (int k = 0; k < nl; ++k) {
      kabs[k] += dust->mass_frac[s] / fsum * dust->kappa_abs[(size_t)s * nl + k];
      ksca[k] += dust->mass_frac[s] / fsum * dust->kappa_sca[(size_t)s * nl + k];
    }
  std::vector<double> chi(nl), omega(nl);
  for (int k = 0; k < nl; ++k) {
    if (!(kabs[k] > 0.0) || !(ksca[k] >= 0.0)) {
      delete ctx;
      return fail(nullptr, MCRT_E_ARG, "absorption opacity must be > 0 in every bin");
    }
    chi[k] = kabs[k] + ksca[k];
    omega[k] = ksca[k] / chi[k];
  }
  Planck pl;
  std::vector<double> Tn(nT), cdf((size_t)nT * nl), G(nT), Drho(nT), kbar(nT), star_cdf(nl);
  std::vector<double> B(nl), dB(nl);
  const double lr = std::log(opt->T_hi / opt->T_lo);
  for (int n = 0; n < nT; ++n) {
    double T = n == 0 ? 0.0 : opt->T_lo * std::exp(lr * (double)(n - 1) / (double)(nT - 2));
    if (n == 1) T = opt->T_lo;
    if (n == nT - 1) T = opt->T_hi;
    Tn[n] = T;
    for (int k = 0; k < nl; ++k) pl.bin(dust->lambda_edges[k], dust->lambda_edges[k + 1], T, B[k], dB[k]);
    double acc = 0.0;
    for (int k = 0; k < nl; ++k) {
      acc += kabs[k] * B[k];
      cdf[(size_t)n * nl + k] = acc;
    }
    G[n] = acc;
    if (n == 0) continue;
    // The emission-weighted means of Sect. 2.2.3 at the fixed point of the
    // eta equation, eta ~ chi dB/dT: D rho = 1/(3 chi_R) with the Rosseland
    // mean of the extinction, and kappa-bar = <kappa> weighted by dB/dT.
    // Anisotropic scattering enters as the isotropic-equivalent scattering
    // opacity (1 - g) sigma.
    double s_dB = 0.0, s_dBchi = 0.0, s_kdB = 0.0;
    for (int k = 0; k < nl; ++k) {
      s_dB += dB[k];
      s_dBchi += dB[k] / (kabs[k] + ksca[k] * (1.0 - opt->g_asym));
      s_kdB += kabs[k] * dB[k];
    }
    Drho[n] = s_dBchi / s_dB / 3.0;
    kbar[n] = s_kdB / s_dB;
  }
  Drho[0] = Drho[1];
  kbar[0] = kbar[1];
  {
    double tot = 0.0;
    for (int k = 0; k < nl; ++k) {
      pl.bin(dust->lambda_edges[k], dust->lambda_edges[k + 1], star->T_star, B[k], dB[k]);
      tot += B[k];
    }
    double acc = 0.0;
    for (int k = 0; k < nl; ++k) {
      acc += B[k];
      star_cdf[k] = acc / tot;
    }
    star_cdf[nl - 1] = 1.0;
  }
  ctx->L_star = 4.0 * PI * star->R_star * star->R_star * SIG_SB * std::pow(star->T_star, 4.0);
  for (int n = 1; n < nT; ++n)
    if (!(G[n] > G[n - 1])) {
      delete ctx;
      return fail(nullptr, MCRT_E_ARG, "emission table not increasing: raise T_lo");
    }
  std::vector<double> mrw_tab(mcrt::MRW_TAB_N);
  for (int q = 0; q < mcrt::MRW_TAB_N; ++q) {
    double v = mcrt::MRW_TAB_V0 + (mcrt::MRW_TAB_V1 - mcrt::MRW_TAB_V0) * q / (mcrt::MRW_TAB_N - 1);
    mrw_tab[q] = mrw_solve_v(v);
  }
  // guide over u = ln g: bin b starts at exp(lnG0 + b / inv_du)
  const double lnG0 = std::log(G[1]);
  const double inv_du = (mcrt::N_GUIDE - 1) / (std::log(G[nT - 1]) - lnG0);
  std::vector<int> guide(mcrt::N_GUIDE);
  {
    int n = 1;
    for (int b = 0; b < mcrt::N_GUIDE; ++b) {
      double g = std::exp(lnG0 + b / inv_du);
      while (n < nT - 2 && G[n + 1] <= g) ++n;
      guide[b] = n;
    }
  }
  std::vector<double> inv_dT(nT, 0.0), g_slope(nT, 0.0);
  for (int n = 0; n + 1 < nT; ++n) {
    inv_dT[n] = 1.0 / (Tn[n + 1] - Tn[n]);
    g_slope[n] = (Tn[n + 1] - Tn[n]) / (G[n + 1] - G[n]);
  }
  std::vector<double> r2(n_r + 1), mu2(n_mu + 1), smu(n_mu + 1), inv4pim(nc);
  for (int e = 0; e <= n_r; ++e) r2[e] = grid->r_edges[e] * grid->r_edges[e];
  for (int e = 0; e <= n_mu; ++e) {
    mu2[e] = grid->mu_edges[e] * grid->mu_edges[e];
    smu[e] = std::sqrt(1.0 - grid->mu_edges[e] * grid->mu_edges[e]);
  }
  std::vector<double> cell_len(nc);
  for (int i = 0; i < n_r; ++i) {
    double a = grid->r_edges[i], b = grid->r_edges[i + 1];
    double dr3 = b * b * b - a * a * a;
    for (int j = 0; j < n_mu; ++j) {
      double V = 4.0 * PI / 3.0 * dr3 * (grid->mu_edges[j + 1] - grid->mu_edges[j]);
      double mass = rho[i * n_mu + j] * V;
      inv4pim[i * n_mu + j] = mass > 0.0 ? 1.0 / (4.0 * PI * mass) : 0.0;
      const double rc = 0.5 * (a + b), wr = b - a;
      const double wt = rc * (std::acos(grid->mu_edges[j]) - std::acos(grid->mu_edges[j + 1])) *
                        (j == 0 ? 2.0 : 1.0);
      cell_len[i * n_mu + j] = wr > wt ? wr : wt;
    }
  }
  double chi_max = 0.0;
  for (int k = 0; k < nl; ++k) chi_max = std::max(chi_max, chi[k]);

  // ---------------- device blob
  struct Part {
    const void* src;
    size_t bytes;
    void** dst;
  };
  std::vector<float> cdf32(cdf.begin(), cdf.end()), star32(star_cdf.begin(), star_cdf.end()),
      chi32(chi.begin(), chi.end()), om32(omega.begin(), omega.end());
  mcrt::DevModel& M = ctx->m;
  M.n_r = n_r;
  M.n_mu = n_mu;
  M.n_lambda = nl;
  M.n_T = nT;
  M.n_inc = opt->n_inc;
  M.lnT_lo = std::log(opt->T_lo);
  M.inv_dlnT = (double)(nT - 2) / std::log(opt->T_hi / opt->T_lo);
  M.lnG0 = lnG0;
  M.inv_du = inv_du;
  M.R_star = star->R_star;
  M.L_star = ctx->L_star;
  M.chi_max = chi_max;
  std::vector<Part> parts = {
      {grid->r_edges, (n_r + 1) * sizeof(double), (void**)&M.r_edges},
      {r2.data(), (n_r + 1) * sizeof(double), (void**)&M.r2},
      {grid->mu_edges, (n_mu + 1) * sizeof(double), (void**)&M.mu_edges},
      {mu2.data(), (n_mu + 1) * sizeof(double), (void**)&M.mu2},
      {smu.data(), (n_mu + 1) * sizeof(double), (void**)&M.smu},
      {rho, nc * sizeof(double), (void**)&M.rho},
      {inv4pim.data(), nc * sizeof(double), (void**)&M.inv4pim},
      {Tn.data(), nT * sizeof(double), (void**)&M.Tn},
      {cdf.data(), cdf.size() * sizeof(double), (void**)&M.cdf},
      {G.data(), nT * sizeof(double), (void**)&M.G},
      {Drho.data(), nT * sizeof(double), (void**)&M.Drho},
      {kbar.data(), nT * sizeof(double), (void**)&M.kbar},
      {star_cdf.data(), nl * sizeof(double), (void**)&M.star_cdf},
      {chi.data(), nl * sizeof(double), (void**)&M.chi},
      {omega.data(), nl * sizeof(double), (void**)&M.omega},
      {mrw_tab.data(), mrw_tab.size() * sizeof(double), (void**)&M.mrw_tab},
      {cdf32.data(), cdf32.size() * sizeof(float), (void**)&M.cdf32},
      {star32.data(), nl * sizeof(float), (void**)&M.star_cdf32},
      {chi32.data(), nl * sizeof(float), (void**)&M.chi32},
      {om32.data(), nl * sizeof(float), (void**)&M.omega32},
      {guide.data(), guide.size() * sizeof(int), (void**)&M.g_guide},
      {inv_dT.data(), nT * sizeof(double), (void**)&M.inv_dT},
      {g_slope.data(), nT * sizeof(double), (void**)&M.g_slope},
      {cell_len.data(), nc * sizeof(double), (void**)&M.cell_len},
      {dust->lambda_edges, (nl + 1) * sizeof(double), (void**)&M.lam},
      {pl.a, sizeof(pl.a), (void**)&M.planck_a},
  };
  size_t total = 0;
  for (auto& p : parts) total += al(p.bytes);
  if (hipMalloc(&ctx->d_blob, total) != hipSuccess) {
    delete ctx;
    return fail(nullptr, MCRT_E_OOM, "device allocation of the model failed");
  }
  {
    std::vector<char> host(total, 0);
    size_t off = 0;
    for (auto& p : parts) {
      std::memcpy(host.data() + off, p.src, p.bytes);
      *p.dst = (char*)ctx->d_blob + off;
      off += al(p.bytes);
    }
    if (hipMemcpy(ctx->d_blob, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
      mcrt_destroy(ctx);
      return fail(nullptr, MCRT_E_HIP, "upload of the model failed");
    }
  }
  // tallies + state
  size_t nd = nc * sizeof(double), nu = nc * sizeof(uint32_t);
  size_t tb = al(nd) + 3 * al(nu) + al((size_t)nl * opt->n_inc * sizeof(double)) + al(8) +
              al(mcrt::N_COUNTERS * 8) + al(nd) + al(8) + 2 * al(nd) + al(nc) +
              al(sizeof(mcrt::DevHealth)) + 2 * al(nd) + al(8 * sizeof(double));
  if (hipMalloc(&ctx->d_tally_blob, tb) != hipSuccess) {
    mcrt_destroy(ctx);
    return fail(nullptr, MCRT_E_OOM, "device allocation of the tallies failed");
  }
  char* q = (char*)ctx->d_tally_blob;
  ctx->t.E_abs = (double*)q; q += al(nd);
  ctx->t.visits = (uint32_t*)q; q += al(nu);
  ctx->t.n_abs = (uint32_t*)q; q += al(nu);
  ctx->t.n_mrw = (uint32_t*)q; q += al(nu);
  ctx->t.sed = (double*)q; q += al((size_t)nl * opt->n_inc * sizeof(double));
  ctx->t.E_star = (double*)q; q += al(8);
  ctx->t.counters = (unsigned long long*)q; q += al(mcrt::N_COUNTERS * 8);
  ctx->d_E_half = (double*)q; q += al(nd);   // inside the span that clearing covers
  ctx->t.E_half = ctx->d_E_half;
  ctx->d_next = (unsigned long long*)q; q += al(8);
  ctx->d_T = (double*)q; q += al(nd);
  ctx->d_T_prev = (double*)q; q += al(nd);
  ctx->d_region = (uint8_t*)q; q += al(nc);
  ctx->d_health = (mcrt::DevHealth*)q; q += al(sizeof(mcrt::DevHealth));
  ctx->d_conv = (double*)q;
  if (hipMalloc(&ctx->d_tail, (size_t)mcrt::TAIL_CAP * mcrt::TAIL_STATE_BYTES + 256) != hipSuccess) {
    mcrt_destroy(ctx);
    return fail(nullptr, MCRT_E_OOM, "device allocation of the hand-off buffer failed");
  }
  if (opt->j_tally) {
    const size_t pb = al((size_t)nc * nl * sizeof(double)) + al(nd);
    if (hipMalloc(&ctx->d_paths, pb) != hipSuccess) {
      mcrt_destroy(ctx);
      return fail(nullptr, MCRT_E_OOM, "device allocation of the path tallies failed");
    }
    ctx->t.path = (double*)ctx->d_paths;
    ctx->t.mrw_path = (double*)((char*)ctx->d_paths + al((size_t)nc * nl * sizeof(double)));
    if (hipMemset(ctx->d_paths, 0, pb) != hipSuccess) {
      mcrt_destroy(ctx);
      return fail(nullptr, MCRT_E_HIP, "clearing the path tallies failed");
    }
  }
  if (hipMemset(ctx->d_tally_blob, 0, tb) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    mcrt_destroy(ctx);
    return fail(nullptr, MCRT_E_HIP, "clearing the tallies failed");
  }
  *out = ctx;
  return MCRT_OK;
}

void mcrt_destroy(mcrt_ctx* ctx) {
  if (!ctx) return;
  if (ctx->d_blob) hipFree(ctx->d_blob);
  if (ctx->d_tally_blob) hipFree(ctx->d_tally_blob);
  if (ctx->d_pda_blob) hipFree(ctx->d_pda_blob);
  if (ctx->d_lin_args) hipFree(ctx->d_lin_args);
  if (ctx->d_nl) hipFree(ctx->d_nl);
  if (ctx->d_tail) hipFree(ctx->d_tail);
  if (ctx->d_paths) hipFree(ctx->d_paths);
  if (ctx->d_src) hipFree(ctx->d_src);
  delete ctx;
}

int mcrt_reset(mcrt_ctx* ctx, hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  // tallies are contiguous from E_abs up to (excluding) the work counter
  size_t bytes = (size_t)((char*)ctx->d_next - (char*)ctx->t.E_abs);
  int rc = mcrt::launch_zero(ctx->t.E_abs, bytes, stream);
  if (!rc && ctx->t.path)
    rc = mcrt::launch_zero(ctx->d_paths, (size_t)((char*)(ctx->t.mrw_path + ctx->n_cells) -
                                                  (char*)ctx->d_paths), stream);
  return rc;
}

int mcrt_trace(mcrt_ctx* ctx, uint64_t n_packets, uint64_t n_total, uint64_t seed,
               uint64_t offset, const double* frozen_T_dev, mcrt_packet_rec* rec_dev,
               int64_t n_recs, hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  if (n_total == 0 || n_packets > n_total || offset > n_total - n_packets)
    return fail(ctx, MCRT_E_ARG, "packets [offset, offset+n) must lie in [0, n_total)");
  if (n_recs < 0 || (n_recs > 0 && !rec_dev)) return fail(ctx, MCRT_E_ARG, "bad record buffer");
  if (n_packets == 0) return MCRT_OK;
  mcrt::TraceArgs a = mcrt::make_trace_args(ctx, n_packets, n_total, seed, offset, frozen_T_dev,
                                            rec_dev, n_recs);
  int rc = mcrt::launch_zero(ctx->d_next, 8, stream);
  // tail_count, tail_next, live and waves_in
  if (!rc && a.tail_count) rc = mcrt::launch_zero(a.tail_count, 24, stream);
  if (rc) return fail(ctx, rc, "clearing the work counters failed");
  // the MRW coefficients take the temperature the context holds now (the
  // last pass's, PDA included, or one set by the caller), kept apart from
  // the T that a later update overwrites
  if (a.T_coef) {
    rc = mcrt::launch_copy(ctx->d_T_prev, ctx->d_T, (size_t)ctx->n_cells, stream);
    if (rc) return fail(ctx, rc, "copying the MRW temperature failed");
  }
  return mcrt::launch_trace(ctx, a, stream);
}

int mcrt_update_T(mcrt_ctx* ctx, double* T_dev, hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  int rc = mcrt::launch_update_T(ctx, stream);
  if (rc) return rc;
  if (ctx->opt.mrw_coef_T == 1) ctx->have_T_prev = true;
  if (T_dev)
    HIPCHK(ctx, hipMemcpyAsync(T_dev, ctx->d_T, ctx->n_cells * sizeof(double),
                               hipMemcpyDeviceToDevice, stream));
  return MCRT_OK;
}

int mcrt_pda_solve(mcrt_ctx* ctx, const uint8_t* mask_dev, mcrt_pda_stats* stats,
                   hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  if (!mask_dev && ctx->opt.pda_visits <= 0 && !(ctx->opt.pda_sigma > 0.0))
    return fail(ctx, MCRT_E_ARG, "no PDA mask, pda_visits <= 0 and pda_sigma = 0");
  return mcrt::pda_solve(ctx, mask_dev, stats, stream);
}

int mcrt_pda_linear(mcrt_ctx* ctx, const uint8_t* mask_dev, const double* rho_dev,
                    const double* kscale_dev, const double* T_D_dev, const double* T_bc_dev,
                    double* T_out_dev, mcrt_pda_stats* stats, hipStream_t stream) {
  if (!ctx || !mask_dev || !T_D_dev || !T_bc_dev || !T_out_dev)
    return fail(ctx, MCRT_E_ARG, "mcrt_pda_linear: null argument");
  return mcrt::pda_linear(ctx, mask_dev, rho_dev, kscale_dev, T_D_dev, T_bc_dev, T_out_dev, stats,
                          stream);
}

int mcrt_pda_adjoint(mcrt_ctx* ctx, const double* dJdT_dev, double* g_logrho_dev,
                     double* g_kscale_dev, hipStream_t stream) {
  if (!ctx || !dJdT_dev || !g_logrho_dev) return fail(ctx, MCRT_E_ARG, "mcrt_pda_adjoint: null argument");
  return mcrt::pda_adjoint(ctx, dJdT_dev, g_logrho_dev, g_kscale_dev, nullptr, stream);
}

int mcrt_pda_nonlinear(mcrt_ctx* ctx, const uint8_t* mask_dev, const double* rho_dev,
                       const double* kscale_dev, const double* T_bc_dev, double* T_out_dev,
                       mcrt_pda_stats* stats, hipStream_t stream) {
  if (!ctx || !mask_dev || !T_bc_dev || !T_out_dev)
    return fail(ctx, MCRT_E_ARG, "mcrt_pda_nonlinear: null argument");
  return mcrt::pda_nonlinear(ctx, mask_dev, rho_dev, kscale_dev, T_bc_dev, T_out_dev, stats,
                             stream);
}

int mcrt_pda_nonlinear_adjoint(mcrt_ctx* ctx, const double* dJdT_dev, double* g_logrho_dev,
                               double* g_kscale_dev, mcrt_pda_stats* stats, hipStream_t stream) {
  if (!ctx || !dJdT_dev || !g_logrho_dev)
    return fail(ctx, MCRT_E_ARG, "mcrt_pda_nonlinear_adjoint: null argument");
  return mcrt::pda_nl_adjoint(ctx, dJdT_dev, g_logrho_dev, g_kscale_dev, stats, stream);
}

int mcrt_sed(mcrt_ctx* ctx, double* sed_dev, hipStream_t stream) {
  if (!ctx || !sed_dev) return fail(ctx, MCRT_E_ARG, "null argument");
  HIPCHK(ctx, hipMemcpyAsync(sed_dev, ctx->t.sed,
                             (size_t)ctx->n_lambda * ctx->opt.n_inc * sizeof(double),
                             hipMemcpyDeviceToDevice, stream));
  return MCRT_OK;
}

int mcrt_locate(mcrt_ctx* ctx, const double* xyz_dev, int64_t n, int32_t* cell_dev,
                hipStream_t stream) {
  if (!ctx || n < 0 || (n > 0 && (!xyz_dev || !cell_dev))) return fail(ctx, MCRT_E_ARG, "bad locate arguments");
  return mcrt::launch_locate(ctx, xyz_dev, n, cell_dev, stream);
}

int64_t mcrt_get_size(mcrt_ctx* ctx, int what) {
  if (!ctx) return -1;
  int64_t nc = ctx->n_cells;
  int64_t nT = ctx->opt.n_T, nl = ctx->n_lambda;
  switch (what) {
    case MCRT_GET_E_ABS: return nc * 8;
    case MCRT_GET_VISITS:
    case MCRT_GET_N_ABS:
    case MCRT_GET_N_MRW: return nc * 4;
    case MCRT_GET_T: return nc * 8;
    case MCRT_GET_REGION: return nc;
    case MCRT_GET_COUNTERS: return mcrt::N_COUNTERS * 8;
    case MCRT_GET_E_STAR: return 8;
    case MCRT_GET_TABLES: return (nT + nT * nl + nT + nT + nl + 1) * 8;
    case MCRT_GET_RHO: return nc * 8;
    case MCRT_GET_HYDRO_COLD: return 4;
    case MCRT_GET_E_HALF: return nc * 8;
    case MCRT_GET_PATH: return ctx->t.path ? nc * nl * 8 : -1;
    case MCRT_GET_MRW_PATH: return ctx->t.path ? nc * 8 : -1;
    default: return -1;
  }
}

int mcrt_get(mcrt_ctx* ctx, int what, void* dst_dev, hipStream_t stream) {
  if (!ctx || !dst_dev) return fail(ctx, MCRT_E_ARG, "null argument");
  const void* src = nullptr;
  switch (what) {
    case MCRT_GET_E_ABS: src = ctx->t.E_abs; break;
    case MCRT_GET_VISITS: src = ctx->t.visits; break;
    case MCRT_GET_N_ABS: src = ctx->t.n_abs; break;
    case MCRT_GET_N_MRW: src = ctx->t.n_mrw; break;
    case MCRT_GET_T: src = ctx->d_T; break;
    case MCRT_GET_REGION: src = ctx->d_region; break;
    case MCRT_GET_COUNTERS: src = ctx->t.counters; break;
    case MCRT_GET_RHO: src = ctx->m.rho; break;
    case MCRT_GET_HYDRO_COLD: src = &ctx->d_health->hydro_cold; break;
    case MCRT_GET_E_HALF: src = ctx->d_E_half; break;
    case MCRT_GET_PATH: src = ctx->t.path; break;
    case MCRT_GET_MRW_PATH: src = ctx->t.mrw_path; break;
    case MCRT_GET_E_STAR: src = ctx->t.E_star; break;
    case MCRT_GET_TABLES: {
      int64_t nT = ctx->opt.n_T, nl = ctx->n_lambda;
      char* d = (char*)dst_dev;
      const mcrt::DevModel& M = ctx->m;
      HIPCHK(ctx, hipMemcpyAsync(d, M.Tn, nT * 8, hipMemcpyDeviceToDevice, stream));
      d += nT * 8;
      HIPCHK(ctx, hipMemcpyAsync(d, M.cdf, nT * nl * 8, hipMemcpyDeviceToDevice, stream));
      d += nT * nl * 8;
      HIPCHK(ctx, hipMemcpyAsync(d, M.Drho, nT * 8, hipMemcpyDeviceToDevice, stream));
      d += nT * 8;
      HIPCHK(ctx, hipMemcpyAsync(d, M.kbar, nT * 8, hipMemcpyDeviceToDevice, stream));
      d += nT * 8;
      HIPCHK(ctx, hipMemcpyAsync(d, M.star_cdf, nl * 8, hipMemcpyDeviceToDevice, stream));
      d += nl * 8;
      HIPCHK(ctx, hipMemcpyAsync(d, &ctx->L_star, 8, hipMemcpyHostToDevice, stream));
      return MCRT_OK;
    }
    default: return fail(ctx, MCRT_E_ARG, "unknown quantity");
  }
  if (!src) return fail(ctx, MCRT_E_ARG, "this context does not keep that quantity");
  HIPCHK(ctx, hipMemcpyAsync(dst_dev, src, (size_t)mcrt_get_size(ctx, what),
                             hipMemcpyDeviceToDevice, stream));
  return MCRT_OK;
}

int mcrt_hydrostatic(mcrt_ctx* ctx, double M_star, double mu_mol, double* rho_dev,
                     hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  if (!(M_star >= 0.0) || !(mu_mol > 0.0))
    return fail(ctx, MCRT_E_ARG, "need M_star >= 0 and mu_mol > 0");
  int rc = mcrt::launch_hydrostatic(ctx, mcrt::hydro_A(M_star, mu_mol), ctx->opt.T_lo, stream);
  if (rc) return rc;
  ctx->lin_ready = false;
  if (rho_dev)
    HIPCHK(ctx, hipMemcpyAsync(rho_dev, ctx->m.rho, ctx->n_cells * sizeof(double),
                               hipMemcpyDeviceToDevice, stream));
  return MCRT_OK;
}

int mcrt_convergence(mcrt_ctx* ctx, int32_t n_min, int32_t first, double* out_host,
                     hipStream_t stream) {
  if (!ctx) return fail(nullptr, MCRT_E_ARG, "null context");
  if (n_min < 1) return fail(ctx, MCRT_E_ARG, "n_min must be >= 1");
  int rc = mcrt::launch_convergence(ctx, n_min, first ? 1 : 0, stream);
  if (rc) return fail(ctx, rc, "convergence statistic launch failed");
  if (out_host) {
    HIPCHK(ctx, hipMemcpyAsync(out_host, mcrt::conv_result(ctx), 4 * sizeof(double),
                               hipMemcpyDeviceToHost, stream));
    HIPCHK(ctx, hipStreamSynchronize(stream));
  }
  return MCRT_OK;
}

int mcrt_region_mask(mcrt_ctx* ctx, int32_t visits_min, double sigma_max, uint8_t* mask_dev,
                     hipStream_t stream) {
  if (!ctx || !mask_dev) return fail(ctx, MCRT_E_ARG, "null argument");
  if (!(sigma_max >= 0.0)) return fail(ctx, MCRT_E_ARG, "sigma_max must be >= 0");
  int rc = mcrt::launch_region_mask(ctx, visits_min, sigma_max, mask_dev, stream);
  return rc ? fail(ctx, rc, "region mask launch failed") : MCRT_OK;
}

int mcrt_mean_intensity(mcrt_ctx* ctx, const double* T_dev, double* J_dev, hipStream_t stream) {
  if (!ctx || !J_dev) return fail(ctx, MCRT_E_ARG, "null argument");
  if (!ctx->t.path) return fail(ctx, MCRT_E_ARG, "the context keeps no path tallies (j_tally)");
  int rc = mcrt::launch_mean_intensity(ctx, T_dev ? T_dev : ctx->d_T, J_dev, stream);
  return rc ? fail(ctx, rc, "mean intensity launch failed") : MCRT_OK;
}

namespace {
// Checks shared by the ray-traced spectrum and image; allocates the
// context's source-function buffer on first use.
int raytrace_checks(mcrt_ctx* ctx, const double* out, const double* cos_i_host, int32_t n_inc,
                    int32_t n_sub, int32_t n_phi) {
  if (!ctx || !out || !cos_i_host) return fail(ctx, MCRT_E_ARG, "null argument");
  if (n_inc < 1 || n_sub < 1 || n_phi < 1) return fail(ctx, MCRT_E_ARG, "n_inc, n_sub, n_phi >= 1");
  for (int q = 0; q < n_inc; ++q)
    if (!(cos_i_host[q] >= 0.0 && cos_i_host[q] <= 1.0))
      return fail(ctx, MCRT_E_ARG, "cos_i must lie in [0, 1]");
  if (ctx->opt.g_asym != 0.0)
    return fail(ctx, MCRT_E_ARG, "the ray tracer's source function scatters isotropically");
  if (!ctx->d_src &&
      hipMalloc((void**)&ctx->d_src, (size_t)ctx->n_cells * ctx->n_lambda * sizeof(double)) !=
          hipSuccess) {
    ctx->d_src = nullptr;
    return fail(ctx, MCRT_E_OOM, "source-function buffer");
  }
  return MCRT_OK;
}
}  // namespace

int mcrt_raytrace_sed(mcrt_ctx* ctx, const double* T_dev, const double* J_dev, int32_t n_inc,
                      const double* cos_i_host, int32_t n_sub, int32_t n_phi, double* L_dev,
                      hipStream_t stream) {
  int rc = raytrace_checks(ctx, L_dev, cos_i_host, n_inc, n_sub, n_phi);
  if (rc) return rc;
  rc = mcrt::launch_raytrace(ctx, T_dev ? T_dev : ctx->d_T, J_dev, n_inc, cos_i_host, n_sub,
                             n_phi, L_dev, stream);
  return rc ? fail(ctx, rc, "ray tracing launch failed") : MCRT_OK;
}

int mcrt_raytrace_image(mcrt_ctx* ctx, const double* T_dev, const double* J_dev, int32_t n_inc,
                        const double* cos_i_host, int32_t n_sub, int32_t n_phi, double* I_dev,
                        hipStream_t stream) {
  int rc = raytrace_checks(ctx, I_dev, cos_i_host, n_inc, n_sub, n_phi);
  if (rc) return rc;
  rc = mcrt::launch_raytrace_image(ctx, T_dev ? T_dev : ctx->d_T, J_dev, n_inc, cos_i_host,
                                   n_sub, n_phi, I_dev, stream);
  return rc ? fail(ctx, rc, "ray tracing launch failed") : MCRT_OK;
}

int mcrt_visibility(mcrt_ctx* ctx, const double* I_dev, int32_t n_inc, const double* cos_i_host,
                    int32_t n_sub, int32_t n_phi, int32_t n_base, const double* baselines_host,
                    double distance, double* V_dev, hipStream_t stream) {
  if (!ctx || !I_dev || !V_dev || !cos_i_host || !baselines_host)
    return fail(ctx, MCRT_E_ARG, "null argument");
  if (n_inc < 1 || n_sub < 1 || n_phi < 1 || n_base < 1)
    return fail(ctx, MCRT_E_ARG, "n_inc, n_sub, n_phi, n_base >= 1");
  if (!(distance > 0.0) || !std::isfinite(distance))
    return fail(ctx, MCRT_E_ARG, "distance must be positive");
  for (int q = 0; q < n_inc; ++q)
    if (!(cos_i_host[q] >= 0.0 && cos_i_host[q] <= 1.0))
      return fail(ctx, MCRT_E_ARG, "cos_i must lie in [0, 1]");
  for (int j = 0; j < n_base; ++j)
    if (!(baselines_host[2 * j] >= 0.0) || !std::isfinite(baselines_host[2 * j]) ||
        !std::isfinite(baselines_host[2 * j + 1]))
      return fail(ctx, MCRT_E_ARG, "baseline lengths >= 0 and finite angles");
  if (!ctx->d_src &&
      hipMalloc((void**)&ctx->d_src, (size_t)ctx->n_cells * ctx->n_lambda * sizeof(double)) !=
          hipSuccess) {
    ctx->d_src = nullptr;
    return fail(ctx, MCRT_E_OOM, "source-function buffer");
  }
  int rc = mcrt::launch_visibility(ctx, I_dev, n_inc, cos_i_host, n_sub, n_phi, n_base,
                                   baselines_host, distance, V_dev, stream);
  return rc ? fail(ctx, rc, rc == MCRT_E_ARG ? ctx->err : "visibility launch failed") : MCRT_OK;
}

int mcrt_set_T(mcrt_ctx* ctx, const double* T_dev, hipStream_t stream) {
  if (!ctx || !T_dev) return fail(ctx, MCRT_E_ARG, "null argument");
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_T, T_dev, ctx->n_cells * sizeof(double),
                             hipMemcpyDeviceToDevice, stream));
  if (ctx->opt.mrw_coef_T == 1) ctx->have_T_prev = true;
  return MCRT_OK;
}

const char* mcrt_strerror(int code) {
  switch (code) {
    case MCRT_OK: return "ok";
    case MCRT_E_ARG: return "invalid argument";
    case MCRT_E_OOM: return "device out of memory";
    case MCRT_E_HIP: return "HIP runtime error";
    case MCRT_E_NOT_CONVERGED: return "PDA solver did not converge";
    case MCRT_E_STUCK: return "packets hit the event cap";
    case MCRT_E_SINGULAR_REGION: return "PDA region part without Dirichlet neighbour";
    default: return "unknown error";
  }
}

const char* mcrt_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
