// Packet transport on gfx950, FP64 throughout ("plain" path).
//
// One packet per lane in persistent wavefronts: a lane whose packet ends
// takes the next packet id from a global counter (one atomic per wavefront
// per refill), so lanes stay busy while packet lengths vary by orders of
// magnitude (the optically thick midplane).  Each loop iteration performs
// one event of the lane's packet: a flight through the central hole, a face
// crossing, or an interaction (scattering or absorption with immediate
// reemission, Sect. 2.1) optionally followed by modified-random-walk steps
// (Sect. 2.2.2).  Small tables (grid edges, temperature nodes, emission
// per unit mass G(T), D*rho(T), kappa-bar(T), opacities, star spectrum, MRW
// escape table) are staged in LDS; the emission CDF joins them when it fits.
//
// FP64 code in this file is compiled without contraction into fused
// multiply-adds so that cell location is bit-exact and event sequences match
// the CPU reference packet by packet.
#include <hip/hip_runtime.h>

#include "mcrt_internal.h"
#include "rng.h"

#pragma clang fp contract(off)

namespace mcrt {
namespace {

constexpr double PI = 3.14159265358979323846;

struct Lds {
  double *r_edges, *r2, *mu_edges, *mu2, *smu, *Tn, *G, *Drho, *kbar, *star_cdf, *chi, *omega,
      *mrw_tab, *cdf;
};

__host__ __device__ inline size_t lds_small_doubles(int n_r, int n_mu, int n_T, int n_lambda) {
  return (size_t)3 * (n_r + 1) + (size_t)3 * (n_mu + 1) + (size_t)4 * n_T + (size_t)3 * n_lambda +
         MRW_TAB_N;
}

// ---------------------------------------------------------------- geometry
// Leave a sphere from inside; c = r^2 - R^2, pd = p.d.
__device__ inline double exit_sphere(double pd, double c) {
  double disc = pd * pd - c;
  if (c >= 0.0 && (pd > 0.0 || disc < 0.0)) return 0.0;
  disc = disc < 0.0 ? 0.0 : disc;
  double sq = sqrt(disc);
  return pd > 0.0 ? -c / (pd + sq) : -pd + sq;
}

// Reach a sphere from outside; returns a negative value if it is missed.
__device__ inline double enter_sphere(double pd, double c) {
  if (c <= 0.0 && pd < 0.0) return 0.0;
  if (pd >= 0.0) return -1.0;
  double disc = pd * pd - c;
  if (disc < 0.0) return -1.0;
  return c / (-pd + sqrt(disc));
}

// Leave across the cone pair |z| = mu r, f(s) = A s^2 + 2 B s + C.  toward_pole:
// the cell is on the wedge side (f < 0) and is left when f turns positive;
// otherwise on the pole side, left when f turns negative.  < 0: never.
__device__ inline double exit_cone(double A, double B, double C, bool toward_pole) {
  if (toward_pole) {
    if (C >= 0.0 && B > 0.0) return 0.0;
  } else {
    if (C <= 0.0 && B < 0.0) return 0.0;
  }
  double disc = B * B - A * C;
  if (disc < 0.0) return -1.0;
  double sq = sqrt(disc);
  double v;
  if (toward_pole)
    v = (B > 0.0) ? C / (-B - sq) : (-B + sq) / A;
  else
    v = (B < 0.0) ? C / (-B + sq) : (-B - sq) / A;
  if (!(v > 0.0) || __builtin_isinf(v)) return -1.0;
  return v;
}

// Distance to the cell boundary along d and the face: 0 inner sphere,
// 1 outer sphere, 2 cone toward the midplane, 3 cone toward the pole.
__device__ inline double boundary(const Lds& L, int n_mu, int i, int j, const double p[3],
                                  const double d[3], int& face) {
  double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double best = exit_sphere(pd, rr - L.r2[i + 1]);
  face = 1;
  double s = enter_sphere(pd, rr - L.r2[i]);
  if (s >= 0.0 && s < best) { best = s; face = 0; }
  double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (j >= 1) {
    double m2 = L.mu2[j];
    s = exit_cone(d[2] * d[2] - m2 * dd, p[2] * d[2] - m2 * pd, p[2] * p[2] - m2 * rr, false);
    if (s >= 0.0 && s < best) { best = s; face = 2; }
  }
  if (j + 1 < n_mu) {
    double m2 = L.mu2[j + 1];
    s = exit_cone(d[2] * d[2] - m2 * dd, p[2] * d[2] - m2 * pd, p[2] * p[2] - m2 * rr, true);
    if (s >= 0.0 && s < best) { best = s; face = 3; }
  }
  return best;
}

// Row of mu for a point (largest e with mu_e^2 r^2 <= z^2), r2 = (x x + y y) + z z.
__device__ inline int mu_row(const double* mu2, int n_mu, double r2, double z2) {
  int lo = 0, hi = n_mu;  // mu2[lo]*r2 <= z2 holds for lo = 0
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (mu2[mid] * r2 <= z2) lo = mid; else hi = mid;
  }
  return lo;
}

// Lower bound of the distance to the cell boundary (spheres and full cones).
__device__ inline double min_boundary_distance(const Lds& L, int n_mu, int i, int j,
                                               const double p[3]) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double dmin = fmin(r - L.r_edges[i], L.r_edges[i + 1] - r);
  double mu = fabs(p[2]) / r;
  double sm = sqrt(fmax(0.0, 1.0 - mu * mu));
  if (j >= 1) dmin = fmin(dmin, r * (L.smu[j] * mu - L.mu_edges[j] * sm));
  if (j + 1 < n_mu) dmin = fmin(dmin, r * (L.mu_edges[j + 1] * sm - L.smu[j + 1] * mu));
  return dmin > 0.0 ? dmin : 0.0;
}

// ------------------------------------------------------------ T tables
__device__ inline int seg_of(const double* x, int n, double v) {
  if (v >= x[n - 1]) return n - 2;
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ inline double T_of_g(const Lds& L, int n_T, double g) {
  if (g <= 0.0) return 0.0;
  int n = seg_of(L.G, n_T, g);
  double Ga = L.G[n], Gb = L.G[n + 1];
  return L.Tn[n] + (g - Ga) / (Gb - Ga) * (L.Tn[n + 1] - L.Tn[n]);
}

__device__ inline double interp_T(const Lds& L, int n_T, const double* tab, double T) {
  int n = seg_of(L.Tn, n_T, T);
  double f = (T - L.Tn[n]) / (L.Tn[n + 1] - L.Tn[n]);
  return tab[n] + f * (tab[n + 1] - tab[n]);
}

// Reemission bin: smallest k whose cumulative difference spectrum exceeds
// xi times the total.  T_old < 0: full spectrum at T_new.
__device__ inline int reemit(const Lds& L, const double* cdf, int n_T, int nl, double T_old,
                             double T_new, double xi) {
  int nn = seg_of(L.Tn, n_T, T_new);
  double fn = (T_new - L.Tn[nn]) / (L.Tn[nn + 1] - L.Tn[nn]);
  bool diff = (T_old >= 0.0) && (T_new > T_old);
  int no = 0;
  double fo = 0.0;
  if (diff) {
    no = seg_of(L.Tn, n_T, T_old);
    fo = (T_old - L.Tn[no]) / (L.Tn[no + 1] - L.Tn[no]);
  }
  const double* an = cdf + (size_t)nn * nl;
  const double* bn = an + nl;
  const double* ao = cdf + (size_t)no * nl;
  const double* bo = ao + nl;
  bool same = diff && (no == nn);
  double df = fn - fo;
  auto Dk = [&](int k) -> double {
    if (same) return df * (bn[k] - an[k]);
    double cn = an[k] + fn * (bn[k] - an[k]);
    if (!diff) return cn;
    return cn - (ao[k] + fo * (bo[k] - ao[k]));
  };
  double tot = Dk(nl - 1);
  if (!(tot > 0.0)) {
    diff = false;
    same = false;
    tot = Dk(nl - 1);
  }
  double target = xi * tot;
  int lo = 0, hi = nl - 1;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (Dk(mid) > target) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// ------------------------------------------------------------- MRW law
// Survival P(s) in a sphere with an absorbing edge (s = D c t / R0^2) and
// dP/ds; the theta-function form below s = 0.1.
__device__ inline void survival(double s, double& P, double& dP) {
  if (s >= 0.1) {
    double x = PI * PI * s, sum = 0.0, dsum = 0.0;
    for (int n = 1; n <= 7; ++n) {
      double n2 = (double)(n * n);
      double e = exp(-n2 * x);
      double sg = (n & 1) ? 1.0 : -1.0;
      sum += sg * e;
      dsum -= sg * n2 * PI * PI * e;
    }
    P = 2.0 * sum;
    dP = 2.0 * dsum;
  } else {
    // 1 - P = 2 sqrt(pi/x) sum_k exp(-a_k / s), a_k = (2k+1)^2 / 4, x = pi^2 s
    double sum = 0.0, dsum = 0.0;
    for (int k = 0; k < 3; ++k) {
      double a = (double)((2 * k + 1) * (2 * k + 1)) * 0.25;
      double e = exp(-a / s);
      sum += e;
      dsum += e * a / (s * s);
    }
    double pre = 2.0 / (sqrt(PI) * sqrt(s));  // 2 sqrt(pi / (pi^2 s))
    P = 1.0 - pre * sum;
    dP = -(pre * dsum - 0.5 * pre / s * sum);
  }
}

__device__ inline double escape_s(const Lds& L, double P0) {
  double v = log(-log(P0));
  double t = (v - MRW_TAB_V0) / (MRW_TAB_V1 - MRW_TAB_V0) * (MRW_TAB_N - 1);
  t = fmin(fmax(t, 0.0), (double)(MRW_TAB_N - 1) - 1e-9);
  int q = (int)t;
  double f = t - q;
  double s = L.mrw_tab[q] + f * (L.mrw_tab[q + 1] - L.mrw_tab[q]);
  for (int it = 0; it < 3; ++it) {
    double P, dP;
    survival(s, P, dP);
    double step = (P - P0) / dP;
    double sn = s - step;
    s = sn > 0.5 * s ? sn : 0.5 * s;
  }
  return s;
}

__device__ inline void iso_dir(Rng64& r, double d[3]) {
  double w = 2.0 * r.next() - 1.0;
  double ph = 2.0 * PI * r.next();
  double st = sqrt(fmax(0.0, 1.0 - w * w));
  double sn, cs;
  sincos(ph, &sn, &cs);
  d[0] = st * cs;
  d[1] = st * sn;
  d[2] = w;
}

template <bool CDF_LDS>
__global__ void __launch_bounds__(256) trace_fp64_kernel(TraceArgs A) {
  extern __shared__ double smem[];
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda, n_T = M.n_T;
  Lds L;
  {
    double* q = smem;
    auto take = [&](double*& dst, const double* src, int n) {
      dst = q;
      for (int a = threadIdx.x; a < n; a += blockDim.x) q[a] = src[a];
      q += n;
    };
    take(L.r_edges, M.r_edges, n_r + 1);
    take(L.r2, M.r2, n_r + 1);
    take(L.mu_edges, M.mu_edges, n_mu + 1);
    take(L.mu2, M.mu2, n_mu + 1);
    take(L.smu, M.smu, n_mu + 1);
    take(L.Tn, M.Tn, n_T);
    take(L.G, M.G, n_T);
    take(L.Drho, M.Drho, n_T);
    take(L.kbar, M.kbar, n_T);
    take(L.star_cdf, M.star_cdf, nl);
    take(L.chi, M.chi, nl);
    take(L.omega, M.omega, nl);
    take(L.mrw_tab, M.mrw_tab, MRW_TAB_N);
    if (CDF_LDS) take(L.cdf, M.cdf, n_T * nl);
    else L.cdf = nullptr;
  }
  __syncthreads();
  const double* cdf = CDF_LDS ? L.cdf : M.cdf;

  const int lane = __lane_id();
  bool alive = false, exhausted = false;
  // packet state
  Rng64 rng;
  double p[3] = {0, 0, 0}, d[3] = {0, 0, 1}, tau = 0.0;
  int k = 0, i = -1, j = 0, n_int = 0;
  long long events = 0;
  uint64_t pid = 0;
  uint32_t pc_cross = 0, pc_scat = 0, pc_abs = 0, pc_mrw = 0;
  // lane totals
  unsigned long long tot[N_COUNTERS] = {0, 0, 0, 0, 0, 0, 0, 0};

  for (;;) {
    // ---- refill idle lanes (one atomic per wavefront)
    unsigned long long idle = __ballot(!alive);
    if (idle != 0ull && !exhausted) {
      int cnt = __popcll(idle);
      int leader = __ffsll((long long)idle) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.next, (unsigned long long)cnt);
      base = __shfl(base, leader);
      if (base + cnt >= A.n_packets) exhausted = true;
      if (!alive) {
        unsigned long long below = idle & ((1ull << lane) - 1ull);
        unsigned long long q = base + (unsigned long long)__popcll(below);
        if (q < A.n_packets) {
          // ---- launch (Sect. 2.1): uniform point on the star at azimuth 0,
          // Lambertian outward direction, bin from the stellar spectrum
          pid = A.offset + q;
          rng.init(A.key0, A.key1, pid);
          double ws = 2.0 * rng.next() - 1.0;
          double st = sqrt(fmax(0.0, 1.0 - ws * ws));
          p[0] = M.R_star * st;
          p[1] = 0.0;
          p[2] = M.R_star * ws;
          double mup = sqrt(rng.next());
          double php = 2.0 * PI * rng.next();
          double sp = sqrt(fmax(0.0, 1.0 - mup * mup));
          double sn, cs;
          sincos(php, &sn, &cs);
          d[0] = mup * st + sp * cs * ws;
          d[1] = sp * sn;
          d[2] = mup * ws - sp * cs * st;
          double xs = rng.next();
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (L.star_cdf[mid] > xs) hi = mid; else lo = mid + 1;
          }
          k = lo;
          tau = -log(rng.next());
          i = -1;
          j = 0;
          n_int = 0;
          events = 0;
          pc_cross = pc_scat = pc_abs = pc_mrw = 0;
          tot[C_LAUNCH]++;
          alive = true;
        }
      }
    }
    if (__ballot(alive) == 0ull) {
      if (exhausted) break;
      continue;
    }
    if (!alive) continue;

    // ---- one event of this lane's packet
    int fate = 0;
    if (++events > A.max_events) {
      fate = 3;
    } else if (i < 0) {
      // central hole: free flight to the star or to the inner grid sphere
      double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
      double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      double s = enter_sphere(pd, rr - M.R_star * M.R_star);
      if (s >= 0.0) {
        p[0] += s * d[0]; p[1] += s * d[1]; p[2] += s * d[2];
        fate = 2;
      } else {
        s = exit_sphere(pd, rr - L.r2[0]);
        p[0] += s * d[0]; p[1] += s * d[1]; p[2] += s * d[2];
        i = 0;
        double r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2];
        j = mu_row(L.mu2, n_mu, r2, p[2] * p[2]);
        atomicAdd(&A.t.visits[j], 1u);
        n_int = 0;
        ++pc_cross;
      }
    } else {
      const int c = i * n_mu + j;
      const double rho = M.rho[c];
      const double alpha = rho * L.chi[k];
      int face;
      double sb = boundary(L, n_mu, i, j, p, d, face);
      double tau_b = alpha * sb;
      if (tau_b <= tau) {
        p[0] += sb * d[0]; p[1] += sb * d[1]; p[2] += sb * d[2];
        tau -= tau_b;
        ++pc_cross;
        bool entered = true;
        if (face == 1) {
          if (i + 1 == n_r) {
            int m = (int)(fabs(d[2]) * M.n_inc);
            m = m < M.n_inc ? m : M.n_inc - 1;
            unsafeAtomicAdd(&A.t.sed[k * M.n_inc + m], A.eps);
            fate = 1;
            entered = false;
          } else {
            ++i;
          }
        } else if (face == 0) {
          --i;
          if (i < 0) entered = false;
        } else if (face == 2) {
          --j;
        } else {
          ++j;
        }
        if (entered) atomicAdd(&A.t.visits[i * n_mu + j], 1u);
        n_int = 0;
      } else {
        // interaction in the cell
        double sint = tau / alpha;
        p[0] += sint * d[0]; p[1] += sint * d[1]; p[2] += sint * d[2];
        const double* fz = A.frozen_T;
        if (rng.next() < L.omega[k]) {
          ++pc_scat;
        } else {
          ++pc_abs;
          atomicAdd(&A.t.n_abs[c], 1u);
          double E_old = unsafeAtomicAdd(&A.t.E_abs[c], A.eps);
          double xb = rng.next();
          if (fz) {
            k = reemit(L, cdf, n_T, nl, -1.0, fz[c], xb);
          } else {
            double im = M.inv4pim[c];
            double T_old = T_of_g(L, n_T, E_old * im);
            double T_new = T_of_g(L, n_T, (E_old + A.eps) * im);
            k = reemit(L, cdf, n_T, nl, T_old, T_new, xb);
          }
        }
        iso_dir(rng, d);
        ++n_int;
        if (A.mrw) {
          // modified random walk while the start criterion holds
          while (n_int >= A.n_int_min) {
            double Tc;
            if (fz) Tc = fz[c];
            else if (A.T_coef) Tc = A.T_coef[c];
            else Tc = T_of_g(L, n_T, __hip_atomic_load(&A.t.E_abs[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) * M.inv4pim[c]);
            double Drho = interp_T(L, n_T, L.Drho, Tc);
            double lam_R = 3.0 * Drho / rho;
            double dmin = min_boundary_distance(L, n_mu, i, j, p);
            if (!(dmin > A.gamma * lam_R)) break;
            if (++events > A.max_events) break;
            double R0 = dmin * (1.0 - 1e-6);
            double s = escape_s(L, rng.next());
            double D = Drho / rho;
            double ell = s * R0 * R0 / D;
            double dE = A.eps * rho * interp_T(L, n_T, L.kbar, Tc) * ell;
            double nrm[3];
            iso_dir(rng, nrm);
            p[0] += R0 * nrm[0]; p[1] += R0 * nrm[1]; p[2] += R0 * nrm[2];
            double E_old = unsafeAtomicAdd(&A.t.E_abs[c], dE);
            double xb = rng.next();
            if (fz) {
              k = reemit(L, cdf, n_T, nl, -1.0, fz[c], xb);
            } else {
              double im = M.inv4pim[c];
              double T_old = T_of_g(L, n_T, E_old * im);
              double T_new = T_of_g(L, n_T, (E_old + dE) * im);
              k = reemit(L, cdf, n_T, nl, T_old, T_new, xb);
            }
            iso_dir(rng, d);
            ++pc_mrw;
            atomicAdd(&A.t.n_mrw[c], 1u);
          }
        }
        tau = -log(rng.next());
      }
    }
    if (fate != 0) {
      if (fate == 1) tot[C_ESCAPED]++;
      else if (fate == 2) { tot[C_STAR]++; unsafeAtomicAdd(A.t.E_star, A.eps); }
      else tot[C_CAPPED]++;
      tot[C_CROSS] += pc_cross;
      tot[C_SCAT] += pc_scat;
      tot[C_ABS] += pc_abs;
      tot[C_MRW] += pc_mrw;
      if (A.recs) {
        int64_t r = (int64_t)(pid - A.offset);
        if (r >= 0 && r < A.n_recs) {
          mcrt_packet_rec& R = A.recs[r];
          R.fate = fate;
          R.k = k;
          R.n_cross = pc_cross;
          R.n_scat = pc_scat;
          R.n_abs = pc_abs;
          R.n_mrw = pc_mrw;
          R.n_draws = (int64_t)rng.d;
          R.x = p[0]; R.y = p[1]; R.z = p[2];
          R.u = d[0]; R.v = d[1]; R.w = d[2];
        }
      }
      alive = false;
    }
  }
  // wavefront totals, one atomic per counter per wavefront
  for (int q = 0; q < N_COUNTERS; ++q) {
    unsigned long long v = tot[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0 && v) atomicAdd(&A.t.counters[q], v);
  }
}

__global__ void locate_kernel(const double* r2e, const double* mu2e, int n_r, int n_mu,
                              const double* xyz, int64_t n, int32_t* cell) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double x = xyz[3 * t], y = xyz[3 * t + 1], z = xyz[3 * t + 2];
  double r2 = (x * x + y * y) + z * z;
  double z2 = z * z;
  if (!(r2 >= r2e[0]) || !(r2 < r2e[n_r])) {
    cell[t] = -1;
    return;
  }
  int lo = 0, hi = n_r;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (r2e[mid] <= r2) lo = mid; else hi = mid;
  }
  cell[t] = lo * n_mu + mu_row(mu2e, n_mu, r2, z2);
}

}  // namespace

int launch_locate(mcrt_ctx* ctx, const double* xyz, int64_t n, int32_t* cell, hipStream_t s) {
  if (n <= 0) return MCRT_OK;
  int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  hipLaunchKernelGGL(locate_kernel, dim3((unsigned)nb), dim3(bs), 0, s, ctx->m.r2, ctx->m.mu2,
                     ctx->n_r, ctx->n_mu, xyz, n, cell);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("locate launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

int launch_trace_fp64(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s) {
  const DevModel& M = ctx->m;
  size_t small = lds_small_doubles(M.n_r, M.n_mu, M.n_T, M.n_lambda) * sizeof(double);
  size_t cdfb = (size_t)M.n_T * M.n_lambda * sizeof(double);
  const size_t lds_cap = 64 * 1024;
  bool cdf_lds = small + cdfb <= lds_cap;
  size_t lds = small + (cdf_lds ? cdfb : 0);
  int bs = ctx->opt.block_size > 0 ? ctx->opt.block_size : 256;
  if (bs > 256) bs = 256;
  int occ = 0;
  hipError_t e;
  if (cdf_lds)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, trace_fp64_kernel<true>, bs, lds);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, trace_fp64_kernel<false>, bs, lds);
  if (e != hipSuccess || occ < 1) occ = 1;
  int per_cu = ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : occ;
  long long nb = (long long)ctx->n_cu * per_cu;
  long long need = ((long long)a.n_packets + bs - 1) / bs;
  if (nb > need) nb = need < 1 ? 1 : need;
  if (cdf_lds)
    hipLaunchKernelGGL(trace_fp64_kernel<true>, dim3((unsigned)nb), dim3(bs), lds, s, a);
  else
    hipLaunchKernelGGL(trace_fp64_kernel<false>, dim3((unsigned)nb), dim3(bs), lds, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

}  // namespace mcrt
