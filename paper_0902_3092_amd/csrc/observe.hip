// Observables by integration of the source function (Sect. 2.3; from the
// Monte Carlo temperature before the PDA, Sect. 3.3): the mean intensity of
// the radiation field from the path-length tallies, the source function of
// isotropic scattering, and the spectral energy distribution from the
// formal solution of the transfer equation along parallel rays.
//
// Work split: one thread per cell (mean intensity), one per (cell, bin)
// (source function), and one wavefront per ray, the ray's cell-to-cell
// traversal uniform across the wavefront (FP64) and the wavelength bins
// spread over its lanes: every segment costs each lane one exponential per
// bin it holds, and the source-function reads of a segment are contiguous
// across the lanes.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "mcrt_internal.h"
#include "trace_common.h"

namespace mcrt {
namespace {

constexpr double H_PL = 6.62607015e-27;
constexpr double K_BZ = 1.380649e-16;
constexpr double C_LT = 2.99792458e10;
constexpr int RAY_BS = 256;       // four rays per workgroup
constexpr int MAX_BINS = 512;     // bins a wavefront holds, eight per lane

// Planck bin integrals (the closed series of the setup tables): with
// x = h nu / (k T), int B_nu dnu = 2 (kT)^4 / (h^3 c^2) F(x_a, x_b),
// F = int t^3 / (e^t - 1) dt, by the power series of t / (e^t - 1) below
// x = 2 and the exponential series of the tail above.
__device__ double planck_I_small(const double* a, double x) {
  double s = 0.0, xp = x * x * x;
  for (int n = 0; n < 64; ++n) {
    s += a[n] * xp / (n + 3);
    xp *= x;
  }
  return s;
}

__device__ double planck_J_tail(double x) {
  double s = 0.0;
  for (int n = 1; n < 200; ++n) {
    const double e = exp(-n * x);
    if (e == 0.0) break;
    const double dn = n;
    const double t = e * (x * x * x / dn + 3.0 * x * x / (dn * dn) + 6.0 * x / (dn * dn * dn) +
                          6.0 / (dn * dn * dn * dn));
    s += t;
    if (t < 1e-18 * s) break;
  }
  return s;
}

__device__ double planck_F(const double* a, double xa, double xb) {
  const double x0 = 2.0;
  if (xa >= x0) return planck_J_tail(xa) - planck_J_tail(xb);
  if (xb <= x0) return planck_I_small(a, xb) - planck_I_small(a, xa);
  return (planck_I_small(a, x0) - planck_I_small(a, xa)) + (planck_J_tail(x0) - planck_J_tail(xb));
}

__device__ double planck_f(double x) {  // x^3 / (e^x - 1)
  if (x > 700.0) return 0.0;
  return x * x * x * exp(-x) / (-expm1(-x));
}

// bin [lam_lo, lam_hi] (cm): B-bar and dB-bar/dT at T (0 for T <= 0)
__device__ void planck_bin(const double* a, double lam_lo, double lam_hi, double T, double& B,
                           double& dB) {
  if (!(T > 0.0)) {
    B = dB = 0.0;
    return;
  }
  const double xa = H_PL * C_LT / (lam_hi * K_BZ * T);
  const double xb = H_PL * C_LT / (lam_lo * K_BZ * T);
  const double kT = K_BZ * T;
  const double pre = 2.0 * kT * kT * kT * kT / (H_PL * H_PL * H_PL * C_LT * C_LT);
  const double Fv = planck_F(a, xa, xb);
  B = pre * Fv;
  dB = pre / T * (4.0 * Fv - xb * planck_f(xb) + xa * planck_f(xa));
}

// J_k = (P_k + w_k P_mrw) / (4 pi V), w_k = dB_k/dT / sum dB/dT at T (the
// fixed point of the eta equation makes eta_k / chi_k proportional to dB_k/dT)
__global__ void mean_intensity_kernel(DevModel M, const double* __restrict__ T,
                                      const double* __restrict__ path,
                                      const double* __restrict__ mrw_path, double* __restrict__ J,
                                      int nc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const int nl = M.n_lambda;
  // 1 / (4 pi V) from the cell's geometry (packets cross empty cells too)
  const int i = c / M.n_mu, j = c % M.n_mu;
  const double ra = M.r_edges[i], rb = M.r_edges[i + 1];
  const double V = 4.0 * KPI / 3.0 * (rb * rb * rb - ra * ra * ra) *
                   (M.mu_edges[j + 1] - M.mu_edges[j]);
  const double iv = 1.0 / (4.0 * KPI * V);
  const double pm = mrw_path[c];
  const double Tc = T[c];
  double sum_dB = 0.0;
  if (pm > 0.0 && Tc > 0.0)
    for (int k = 0; k < nl; ++k) {
      double B, dB;
      planck_bin(M.planck_a, M.lam[k], M.lam[k + 1], Tc, B, dB);
      sum_dB += dB;
    }
  for (int k = 0; k < nl; ++k) {
    double v = path[(size_t)c * nl + k];
    if (sum_dB > 0.0) {
      double B, dB;
      planck_bin(M.planck_a, M.lam[k], M.lam[k + 1], Tc, B, dB);
      v += pm * dB / sum_dB;
    }
    J[(size_t)c * nl + k] = v * iv;
  }
}

// S_k = (kappa_abs,k Bbar_k(T) + kappa_sca,k J_k) / chi_k = (1 - omega) Bbar + omega J
__global__ void source_kernel(DevModel M, const double* __restrict__ T,
                              const double* __restrict__ J, double* __restrict__ S, int nc) {
  const int nl = M.n_lambda;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)nc * nl) return;
  const int c = (int)(idx / nl), k = (int)(idx % nl);
  double B, dB;
  planck_bin(M.planck_a, M.lam[k], M.lam[k + 1], T[c], B, dB);
  const double om = M.omega[k];
  S[idx] = (1.0 - om) * B + (J ? om * J[idx] : 0.0);
}

constexpr int MAX_INC = 64;        // inclinations per call (kernel arguments)

struct RayGeom {
  int n_inc, n_rings, n_sub, n_phi;
  double cos_i[MAX_INC];
};

// One wavefront per ray: ring (hole and radial cells, n_sub each), azimuth,
// inclination from the ray index; traversal from the far side of the outer
// sphere to the near one; each lane holds bins lane, lane + 64, ...  The
// ray's intensity goes into the spectrum L (4 pi I times its area), or, for
// an image, to img[ray][bin].
__global__ void __launch_bounds__(RAY_BS) ray_kernel(DevModel M, RayGeom G,
                                                     const double* __restrict__ S,
                                                     double* __restrict__ L,
                                                     double* __restrict__ img) {
  const int lane = __lane_id();
  const long long ray = (long long)blockIdx.x * (RAY_BS / 64) + threadIdx.x / 64;
  const long long per_inc = (long long)G.n_rings * G.n_phi;
  if (ray >= per_inc * G.n_inc) return;  // the whole wavefront
  const int q = (int)(ray / per_inc);
  const int ring = (int)((ray % per_inc) / G.n_phi);
  const int ph = (int)(ray % G.n_phi);
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda;
  const int cell_r = ring / G.n_sub, part = ring % G.n_sub;
  const double lo = cell_r == 0 ? 0.0 : M.r_edges[cell_r - 1];
  const double hi = M.r_edges[cell_r];
  const double b_lo = lo + (hi - lo) * part / G.n_sub;
  const double b_hi = lo + (hi - lo) * (part + 1) / G.n_sub;
  const double bm = 0.5 * (b_lo + b_hi);
  const double area = KPI * (b_hi * b_hi - b_lo * b_lo) / G.n_phi;
  const double ci = G.cos_i[q], si = sqrt(fmax(0.0, 1.0 - ci * ci));
  double sp, cp;
  sincos((ph + 0.5) * KPI / G.n_phi, &sp, &cp);
  // towards the observer n = (si, 0, ci); image-plane axes (ci, 0, -si), (0, 1, 0)
  const double n[3] = {si, 0.0, ci};
  const double b[3] = {bm * cp * ci, bm * sp, -bm * cp * si};
  const double bb = bm * bm;
  double I[MAX_BINS / 64];
  const int nq = (nl + 63) / 64;
  for (int m = 0; m < nq; ++m) I[m] = 0.0;
  const double ro2 = M.r2[n_r];
  if (bb < ro2) {
    const double s0 = -sqrt(ro2 - bb);
    double p[3] = {b[0] + s0 * n[0], b[1] + s0 * n[1], b[2] + s0 * n[2]};
    int i = n_r - 1;
    int j = mu_row(M.mu2, n_mu, p[0] * p[0] + p[1] * p[1] + p[2] * p[2], p[2] * p[2]);
    const int max_steps = 4 * (n_r + n_mu) + 16;
    for (int step = 0; step < max_steps; ++step) {
      const double pd = p[0] * n[0] + p[1] * n[1] + p[2] * n[2];
      const double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      double best = exit_sphere<double>(pd, rr - M.r2[i + 1]);
      int face = 1;
      double s = enter_sphere<double>(pd, rr - M.r2[i]);
      if (s >= 0.0 && s < best) { best = s; face = 0; }
      if (j >= 1) {
        const double m2 = M.mu2[j];
        s = exit_cone<double>(n[2] * n[2] - m2, p[2] * n[2] - m2 * pd, p[2] * p[2] - m2 * rr,
                              false);
        if (s >= 0.0 && s < best) { best = s; face = 2; }
      }
      if (j + 1 < n_mu) {
        const double m2 = M.mu2[j + 1];
        s = exit_cone<double>(n[2] * n[2] - m2, p[2] * n[2] - m2 * pd, p[2] * p[2] - m2 * rr,
                              true);
        if (s >= 0.0 && s < best) { best = s; face = 3; }
      }
      const int c = i * n_mu + j;
      const double rho = M.rho[c];
      if (rho > 0.0 && best > 0.0) {
        for (int m = 0; m < nq; ++m) {
          const int k = lane + 64 * m;
          if (k < nl) {
            const double at = exp(-rho * M.chi[k] * best);
            I[m] = I[m] * at + S[(size_t)c * nl + k] * (1.0 - at);
          }
        }
      }
      p[0] += best * n[0];
      p[1] += best * n[1];
      p[2] += best * n[2];
      if (face == 1) {
        if (i + 1 == n_r) break;
        ++i;
      } else if (face == 0) {
        if (i == 0) {
          // through the empty hole to its far side
          const double pd2 = p[0] * n[0] + p[1] * n[1] + p[2] * n[2];
          const double chord = pd2 < 0.0 ? -2.0 * pd2 : 0.0;
          p[0] += chord * n[0];
          p[1] += chord * n[1];
          p[2] += chord * n[2];
          j = mu_row(M.mu2, n_mu, p[0] * p[0] + p[1] * p[1] + p[2] * p[2], p[2] * p[2]);
        } else {
          --i;
        }
      } else if (face == 2) {
        --j;
      } else {
        ++j;
      }
    }
  }
  for (int m = 0; m < nq; ++m) {
    const int k = lane + 64 * m;
    if (k >= nl) continue;
    if (img) img[(size_t)ray * nl + k] = I[m];
    else if (I[m] != 0.0) unsafeAtomicAdd(&L[(size_t)q * nl + k], 4.0 * KPI * I[m] * area);
  }
}

// The star per inclination: its luminosity in each bin (the launch spectrum)
// dimmed by the dust along the line of sight from its centre, which runs
// radially at |mu| = cos i and so stays in one row (the row of cos i).
__global__ void star_kernel(DevModel M, RayGeom G, double* __restrict__ L) {
  const int q = blockIdx.x;
  const int nl = M.n_lambda, n_mu = M.n_mu;
  const double ci = G.cos_i[q];
  const int j = mu_row(M.mu2, n_mu, 1.0, ci * ci);
  for (int k = threadIdx.x; k < nl; k += blockDim.x) {
    double tau = 0.0;
    for (int i = 0; i < M.n_r; ++i)
      tau += M.rho[i * n_mu + j] * M.chi[k] * (M.r_edges[i + 1] - M.r_edges[i]);
    const double share = M.star_cdf[k] - (k ? M.star_cdf[k - 1] : 0.0);
    L[(size_t)q * nl + k] += M.L_star * share * exp(-tau);
  }
}

// Visibility amplitudes of a ray-traced image (Sect. 3.4), in two steps.
// Partial sums: workgroup (pair, chunk) takes a contiguous range of the rays
// of one (inclination, baseline) pair; its four wavefronts take every fourth
// ray of it, each lane the bins lane, lane + 64, ...; the four meet in LDS
// and the chunk's sums of A I cos, A I sin and A I per bin go to `part`.
// Then one thread per (pair, bin) adds the chunks in order and the star.
constexpr int MAX_BASE = 64;
constexpr int VIS_BS = 256;

struct VisGeom {
  int n_inc, n_rings, n_sub, n_phi, n_base, n_chunk;
  double distance;
  double cos_i[MAX_INC];
  double B[MAX_BASE], theta[MAX_BASE];
};

__global__ void __launch_bounds__(VIS_BS) vis_partial_kernel(DevModel M, VisGeom G,
                                                             const double* __restrict__ img,
                                                             double* __restrict__ part) {
  __shared__ double red[VIS_BS / 64][3][MAX_BINS];
  const int pair = blockIdx.x / G.n_chunk, chunk = blockIdx.x % G.n_chunk;
  const int q = pair / G.n_base, jb = pair % G.n_base;
  const int lane = __lane_id(), w = threadIdx.x / 64;
  const int nl = M.n_lambda, nq = (nl + 63) / 64;
  const double ct = cos(G.theta[jb]), st = sin(G.theta[jb]);
  double re[MAX_BINS / 64], im[MAX_BINS / 64], tot[MAX_BINS / 64], sf[MAX_BINS / 64];
  for (int m = 0; m < nq; ++m) {
    re[m] = im[m] = tot[m] = 0.0;
    const int k = min(lane + 64 * m, nl - 1);
    sf[m] = G.B[jb] / (sqrt(M.lam[k] * M.lam[k + 1]) * G.distance);
  }
  const long long rays = (long long)G.n_rings * G.n_phi;
  const long long r0 = rays * chunk / G.n_chunk, r1 = rays * (chunk + 1) / G.n_chunk;
  for (long long r = r0 + w; r < r1; r += VIS_BS / 64) {
    const int ring = (int)(r / G.n_phi), p = (int)(r % G.n_phi);
    const int cell = ring / G.n_sub, sub = ring % G.n_sub;
    const double lo = cell == 0 ? 0.0 : M.r_edges[cell - 1];
    const double hi = M.r_edges[cell];
    const double b_lo = lo + (hi - lo) * sub / G.n_sub;
    const double b_hi = lo + (hi - lo) * (sub + 1) / G.n_sub;
    const double bm = 0.5 * (b_lo + b_hi);
    const double half = 0.5 * KPI * (b_hi * b_hi - b_lo * b_lo) / G.n_phi;
    double sp, cp;
    sincos((p + 0.5) * KPI / G.n_phi, &sp, &cp);
    const double x = bm * cp, y = bm * sp;
    const double* row = img + ((size_t)q * rays + r) * nl;
    for (int m = 0; m < nq; ++m) {
      const int k = lane + 64 * m;
      if (k >= nl) continue;
      const double a = half * row[k];
      if (a == 0.0) continue;
      // the ray and its mirror image at -y
      double s1, c1, s2, c2;
      sincos(-2.0 * KPI * sf[m] * (x * ct + y * st), &s1, &c1);
      sincos(-2.0 * KPI * sf[m] * (x * ct - y * st), &s2, &c2);
      re[m] += a * (c1 + c2);
      im[m] += a * (s1 + s2);
      tot[m] += 2.0 * a;
    }
  }
  for (int m = 0; m < nq; ++m) {
    const int k = lane + 64 * m;
    if (k < nl) {
      red[w][0][k] = re[m];
      red[w][1][k] = im[m];
      red[w][2][k] = tot[m];
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nl; k += VIS_BS) {
    double* dst = part + ((size_t)blockIdx.x * 3) * nl;
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int u = 0; u < VIS_BS / 64; ++u) v += red[u][c][k];
      dst[(size_t)c * nl + k] = v;
    }
  }
}

// The star, a point at the centre dimmed along the line of sight (which
// stays in the row of |mu| = cos i), and the amplitude.
__global__ void vis_final_kernel(DevModel M, VisGeom G, const double* __restrict__ part,
                                 double* __restrict__ V) {
  const int nl = M.n_lambda;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)G.n_inc * G.n_base * nl) return;
  const int pair = (int)(idx / nl), k = (int)(idx % nl);
  const int q = pair / G.n_base;
  const double ci = G.cos_i[q];
  const int jr = mu_row(M.mu2, M.n_mu, 1.0, ci * ci);
  double tau = 0.0;
  for (int i = 0; i < M.n_r; ++i)
    tau += M.rho[i * M.n_mu + jr] * M.chi[k] * (M.r_edges[i + 1] - M.r_edges[i]);
  const double share = M.star_cdf[k] - (k ? M.star_cdf[k - 1] : 0.0);
  const double fs = M.L_star * share * exp(-tau) / (4.0 * KPI);
  double R = fs, I = 0.0, F = fs;
  for (int c = 0; c < G.n_chunk; ++c) {
    const double* src = part + ((size_t)(pair * G.n_chunk + c) * 3) * nl;
    R += src[k];
    I += src[nl + k];
    F += src[2 * nl + k];
  }
  V[idx] = F > 0.0 ? sqrt(R * R + I * I) / F : 0.0;
}

}  // namespace

int launch_visibility(mcrt_ctx* ctx, const double* img, int n_inc, const double* cos_i_host,
                      int n_sub, int n_phi, int n_base, const double* base_host, double distance,
                      double* V, hipStream_t s) {
  const DevModel& M = ctx->m;
  if (M.n_lambda > MAX_BINS || n_inc > MAX_INC || n_base > MAX_BASE) {
    set_error(ctx, "visibilities: at most 512 bins, 64 inclinations and 64 baselines per call");
    return MCRT_E_ARG;
  }
  VisGeom G{};
  G.n_inc = n_inc;
  G.n_rings = (M.n_r + 1) * n_sub;
  G.n_sub = n_sub;
  G.n_phi = n_phi;
  G.n_base = n_base;
  G.distance = distance;
  for (int q = 0; q < n_inc; ++q) G.cos_i[q] = cos_i_host[q];
  for (int j = 0; j < n_base; ++j) {
    G.B[j] = base_host[2 * j];
    G.theta[j] = base_host[2 * j + 1];
  }
  // the partial sums live in the source-function buffer (n_cells x n_lambda
  // doubles): chunks per pair as that holds, about 512 workgroups in all
  const int pairs = n_inc * n_base;
  const long long rays = (long long)G.n_rings * n_phi;
  long long nch = ctx->n_cells / (3LL * pairs);
  nch = std::min<long long>(nch, std::max<long long>(1, 512 / pairs));
  nch = std::min<long long>(nch, rays);
  if (nch < 1) {
    set_error(ctx, "visibilities: too many inclinations x baselines for this grid's buffer");
    return MCRT_E_ARG;
  }
  G.n_chunk = (int)nch;
  hipLaunchKernelGGL(vis_partial_kernel, dim3((unsigned)(pairs * nch)), dim3(VIS_BS), 0, s, M, G,
                     img, ctx->d_src);
  const long long outs = (long long)pairs * M.n_lambda;
  hipLaunchKernelGGL(vis_final_kernel, dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, M,
                     G, ctx->d_src, V);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

int launch_mean_intensity(mcrt_ctx* ctx, const double* T, double* J, hipStream_t s) {
  const int nc = ctx->n_cells;
  hipLaunchKernelGGL(mean_intensity_kernel, dim3((nc + 255) / 256), dim3(256), 0, s, ctx->m, T,
                     ctx->t.path, ctx->t.mrw_path, J, nc);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

namespace {
// The spectrum (L: per inclination and bin, with the star) or the image
// (img: per ray and bin, without it) of the same rays.
int raytrace(mcrt_ctx* ctx, const double* T, const double* J, int n_inc,
             const double* cos_i_host, int n_sub, int n_phi, double* L, double* img,
             hipStream_t s) {
  const DevModel& M = ctx->m;
  if (M.n_lambda > MAX_BINS) {
    set_error(ctx, "the ray tracer holds at most 512 bins");
    return MCRT_E_ARG;
  }
  if (n_inc > MAX_INC) {
    set_error(ctx, "at most 64 inclinations per call");
    return MCRT_E_ARG;
  }
  const long long cells_bins = (long long)ctx->n_cells * M.n_lambda;
  hipLaunchKernelGGL(source_kernel, dim3((unsigned)((cells_bins + 255) / 256)), dim3(256), 0, s,
                     M, T, J, ctx->d_src, ctx->n_cells);
  if (L) {
    int rc = launch_zero(L, (size_t)n_inc * M.n_lambda * sizeof(double), s);
    if (rc) return rc;
  }
  RayGeom G{};
  G.n_inc = n_inc;
  G.n_rings = (M.n_r + 1) * n_sub;
  G.n_sub = n_sub;
  G.n_phi = n_phi;
  for (int q = 0; q < n_inc; ++q) G.cos_i[q] = cos_i_host[q];
  const long long rays = (long long)n_inc * G.n_rings * n_phi;
  hipLaunchKernelGGL(ray_kernel, dim3((unsigned)((rays + 3) / 4)), dim3(RAY_BS), 0, s, M, G,
                     ctx->d_src, img ? nullptr : L, img);
  if (!img) hipLaunchKernelGGL(star_kernel, dim3(n_inc), dim3(64), 0, s, M, G, L);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}
}  // namespace

int launch_raytrace(mcrt_ctx* ctx, const double* T, const double* J, int n_inc,
                    const double* cos_i_host, int n_sub, int n_phi, double* L, hipStream_t s) {
  return raytrace(ctx, T, J, n_inc, cos_i_host, n_sub, n_phi, L, nullptr, s);
}

int launch_raytrace_image(mcrt_ctx* ctx, const double* T, const double* J, int n_inc,
                          const double* cos_i_host, int n_sub, int n_phi, double* img,
                          hipStream_t s) {
  return raytrace(ctx, T, J, n_inc, cos_i_host, n_sub, n_phi, nullptr, img, s);
}

}  // namespace mcrt
