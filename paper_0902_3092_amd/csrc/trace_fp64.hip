// Packet transport on gfx950 in FP64 throughout (the "plain" path).
//
// One packet per lane in persistent wavefronts: a lane whose packet ends
// takes the next packet id from a global counter (one atomic per wavefront
// per refill), so lanes stay busy while packet lengths vary by orders of
// magnitude (the optically thick midplane).  Each loop iteration performs
// one event of the lane's packet: a flight through the central hole, a face
// crossing, or an interaction (scattering, or absorption with immediate
// reemission, Sect. 2.1) optionally followed by modified-random-walk steps
// (Sect. 2.2.2, eqs. modified RW .. criterion).
//
// Run time is set by the longest packets (a packet caught in the optically
// thick rim takes ~1e6 events one after another), so the kernel is built
// for the latency of one event: the tables live in LDS (emission CDF in
// FP64 when it fits, else an FP32 copy that locates the bin before two FP64
// probes in L2 confirm it), table indices come from arithmetic guesses plus
// fix-ups instead of binary searches, the cell density and the running cell
// temperature stay in registers while the packet stays in the cell.
//
// FP64 code in this file is compiled without contraction into fused
// multiply-adds so that cell location is bit-exact and event sequences match
// the CPU reference packet by packet.
#include <hip/hip_runtime.h>

#include "mcrt_internal.h"
#include "rng.h"
#include "trace_common.h"

#pragma clang fp contract(off)

namespace mcrt {
namespace {

constexpr int BS64 = 512;

struct Lds64 {
  double *r_edges, *r2, *mu_edges, *mu2, *smu, *star_cdf, *chi, *omega, *mrw_tab;
  TabView tv;
  const double* cdf64;   // LDS or global
  const float* cdf32;    // LDS guess table (nullptr: search cdf64 directly)
  uint32_t* vis;         // per-workgroup visit histogram [n_cells], or null
};

__host__ __device__ inline size_t lds_small_bytes(int n_r, int n_mu, int n_T, int nl) {
  return sizeof(double) * ((size_t)2 * (n_r + 1) + (size_t)3 * (n_mu + 1) + (size_t)6 * n_T +
                           (size_t)3 * nl + MRW_TAB_N) +
         sizeof(int) * N_GUIDE;
}

__device__ __forceinline__ int reemit64(const Lds64& L, double T_old, double T_new, double xi) {
  const int nl = L.tv.nl;
  Reemit<double> R = reemit_setup<double>(L.tv, L.cdf64, T_old, T_new);
  if (L.cdf32 == nullptr) return reemit_search<double>(R, nl, xi);
  // locate with the FP32 copy, then confirm with the FP64 values
  Reemit<float> Rf;
  Rf.an = L.cdf32 + (R.an - L.cdf64);
  Rf.bn = Rf.an + nl;
  Rf.ao = L.cdf32 + (R.ao - L.cdf64);
  Rf.bo = Rf.ao + nl;
  Rf.fn = (float)R.fn;
  Rf.fo = (float)R.fo;
  Rf.df = (float)R.df;
  Rf.diff = R.diff;
  Rf.same = R.same;
  int k = reemit_search<float>(Rf, nl, (float)xi);
  double target = xi * R.D(nl - 1);
  while (k < nl - 1 && !(R.D(k) > target)) ++k;
  while (k > 0 && R.D(k - 1) > target) --k;
  return k;
}

__device__ __forceinline__ double boundary64(const Lds64& L, int n_mu, int i, int j,
                                             const double p[3], const double d[3], int& face) {
  double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double best = exit_sphere<double>(pd, rr - L.r2[i + 1]);
  face = 1;
  double s = enter_sphere<double>(pd, rr - L.r2[i]);
  if (s >= 0.0 && s < best) { best = s; face = 0; }
  double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (j >= 1) {
    double m2 = L.mu2[j];
    s = exit_cone<double>(d[2] * d[2] - m2 * dd, p[2] * d[2] - m2 * pd, p[2] * p[2] - m2 * rr,
                          false);
    if (s >= 0.0 && s < best) { best = s; face = 2; }
  }
  if (j + 1 < n_mu) {
    double m2 = L.mu2[j + 1];
    s = exit_cone<double>(d[2] * d[2] - m2 * dd, p[2] * d[2] - m2 * pd, p[2] * p[2] - m2 * rr,
                          true);
    if (s >= 0.0 && s < best) { best = s; face = 3; }
  }
  return best;
}

// lower bound of the distance to the cell boundary (spheres and full cones)
__device__ __forceinline__ double min_boundary64(const Lds64& L, int n_mu, int i, int j,
                                                 const double p[3]) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double dmin = fmin(r - L.r_edges[i], L.r_edges[i + 1] - r);
  double mu = fabs(p[2]) / r;
  double sm = sqrt(fmax(0.0, 1.0 - mu * mu));
  if (j >= 1) dmin = fmin(dmin, r * (L.smu[j] * mu - L.mu_edges[j] * sm));
  if (j + 1 < n_mu) dmin = fmin(dmin, r * (L.mu_edges[j + 1] * sm - L.smu[j + 1] * mu));
  return dmin > 0.0 ? dmin : 0.0;
}

__device__ __forceinline__ void iso64(Rng64& r, double d[3]) {
  double w = 2.0 * r.next() - 1.0;
  double ph = 2.0 * KPI * r.next();
  double st = sqrt(fmax(0.0, 1.0 - w * w));
  double sn, cs;
  sincos(ph, &sn, &cs);
  d[0] = st * cs;
  d[1] = st * sn;
  d[2] = w;
}

template <int CDF_MODE>  // 2: FP64 CDF in LDS; 1: FP32 guide copy in LDS; 0: global only
__global__ void __launch_bounds__(BS64) trace_fp64_kernel(TraceArgs A) {
  extern __shared__ double smem[];
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda, n_T = M.n_T;
  Lds64 L;
  {
    double* q = smem;
    auto take = [&](double*& dst, const double* src, int n) {
      dst = q;
      for (int a = threadIdx.x; a < n; a += blockDim.x) q[a] = src[a];
      q += n;
    };
    double *Tn, *G, *Drho, *kbar;
    take(L.r_edges, M.r_edges, n_r + 1);
    take(L.r2, M.r2, n_r + 1);
    take(L.mu_edges, M.mu_edges, n_mu + 1);
    take(L.mu2, M.mu2, n_mu + 1);
    take(L.smu, M.smu, n_mu + 1);
    take(Tn, M.Tn, n_T);
    take(G, M.G, n_T);
    take(Drho, M.Drho, n_T);
    take(kbar, M.kbar, n_T);
    double *invdT, *gslope;
    take(invdT, M.inv_dT, n_T);
    take(gslope, M.g_slope, n_T);
    take(L.star_cdf, M.star_cdf, nl);
    take(L.chi, M.chi, nl);
    take(L.omega, M.omega, nl);
    take(L.mrw_tab, M.mrw_tab, MRW_TAB_N);
    int* gq = (int*)q;
    for (int a = threadIdx.x; a < N_GUIDE; a += blockDim.x) gq[a] = M.g_guide[a];
    q = (double*)(gq + N_GUIDE);
    L.tv = TabView{n_T, nl, M.lnT_lo, M.inv_dlnT, M.lnG0, M.inv_du, N_GUIDE, Tn, G, Drho, kbar,
                   gq, invdT, gslope};
    L.cdf64 = M.cdf;
    L.cdf32 = nullptr;
    if (CDF_MODE == 2) {
      double* c = q;
      for (int a = threadIdx.x; a < n_T * nl; a += blockDim.x) c[a] = M.cdf[a];
      L.cdf64 = c;
    } else if (CDF_MODE == 1) {
      float* c = (float*)q;
      for (int a = threadIdx.x; a < n_T * nl; a += blockDim.x) c[a] = M.cdf32[a];
      L.cdf32 = c;
    }
    L.vis = nullptr;
    if (A.vis_lds) {
      size_t off = lds_small_bytes(n_r, n_mu, n_T, nl) +
                   (CDF_MODE == 2 ? (size_t)n_T * nl * 8 : CDF_MODE == 1 ? (size_t)n_T * nl * 4 : 0);
      L.vis = (uint32_t*)((char*)smem + off);
      for (int a = threadIdx.x; a < n_r * n_mu; a += blockDim.x) L.vis[a] = 0u;
    }
  }
  __syncthreads();

  const int lane = __lane_id();
  bool alive = false, exhausted = false;
  Rng64 rng;
  double p[3] = {0, 0, 0}, d[3] = {0, 0, 1}, tau = 0.0;
  int k = 0, i = -1, j = 0, n_int = 0;
  long long events = 0;
  uint64_t pid = 0;
  uint32_t pc_cross = 0, pc_scat = 0, pc_abs = 0, pc_mrw = 0;
  double rho = 0.0;    // density of the current cell
  double im = 0.0;     // 1 / (4 pi m) of the current cell
  double Tc = -1.0;    // running temperature of the current cell (< 0: not known)
  double Tfix = 0.0;   // the cell's fixed temperature (frozen field or MRW coefficient field)
  const double* fixT = A.frozen_T ? A.frozen_T : A.T_coef;
  double mrw_T = -2.0, mrw_Drho = 0.0, mrw_kbar = 0.0, mrw_lim = 0.0;  // MRW coefficients
  // bounds of the distance to the cell boundary: d_safe below (a flight
  // shorter than it stays in the cell, so the face distances are not needed),
  // dm_up above (the last computed distance plus the path flown since: while
  // it is within the MRW limit the criterion cannot hold)
  double d_safe = 0.0, dm_up = INFINITY;
  // absorptions and MRW steps in the current cell, added to the tallies when
  // the packet leaves it; the cell's tally after this lane's last deposit and
  // its temperature (reused when no other packet deposited in between)
  uint32_t cell_abs = 0, cell_mrw = 0;
  double E_seen = -1.0, T_seen = 0.0;
  uint32_t tot[N_COUNTERS] = {0, 0, 0, 0, 0, 0, 0, 0};

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
        unsigned long long q = base + (unsigned long long)__popcll(idle & ((1ull << lane) - 1ull));
        if (q < A.n_packets) {
          // launch (Sect. 2.1): uniform point on the star at azimuth 0,
          // Lambertian outward direction, bin from the stellar spectrum
          pid = A.offset + q;
          rng.init(A.key0, A.key1, pid);
          double ws = 2.0 * rng.next() - 1.0;
          double st = sqrt(fmax(0.0, 1.0 - ws * ws));
          p[0] = M.R_star * st;
          p[1] = 0.0;
          p[2] = M.R_star * ws;
          double mup = sqrt(rng.next());
          double php = 2.0 * KPI * rng.next();
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

    int fate = 0;
    if (++events > A.max_events) {
      fate = 3;
    } else if (i < 0) {
      // central hole: free flight to the star or to the inner grid sphere
      double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
      double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
      double s = enter_sphere<double>(pd, rr - M.R_star * M.R_star);
      if (s >= 0.0) {
        p[0] += s * d[0]; p[1] += s * d[1]; p[2] += s * d[2];
        fate = 2;
      } else {
        s = exit_sphere<double>(pd, rr - L.r2[0]);
        p[0] += s * d[0]; p[1] += s * d[1]; p[2] += s * d[2];
        i = 0;
        double r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2];
        j = mu_row(L.mu2, n_mu, r2, p[2] * p[2]);
        rho = M.rho[j];
        im = M.inv4pim[j];
        if (fixT) Tfix = fixT[j];
        if (L.vis) atomicAdd(&L.vis[j], 1u); else atomicAdd(&A.t.visits[j], 1u);
        Tc = -1.0;
        mrw_T = -2.0;
        d_safe = 0.0;
        dm_up = INFINITY;
        n_int = 0;
        ++pc_cross;
      }
    } else {
      const int c = i * n_mu + j;
      const double alpha = rho * L.chi[k];
      int face = 1;
      double sb = 0.0, tau_b = 0.0;
      const bool inside = tau < alpha * d_safe;
      if (!inside) {
        sb = boundary64(L, n_mu, i, j, p, d, face);
        tau_b = alpha * sb;
      }
      if (!inside && tau_b <= tau) {
        if (cell_abs) { atomicAdd(&A.t.n_abs[c], cell_abs); cell_abs = 0; }
        if (cell_mrw) { atomicAdd(&A.t.n_mrw[c], cell_mrw); cell_mrw = 0; }
        E_seen = -1.0;
        d_safe = 0.0;
        dm_up = INFINITY;
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
        if (entered) {
          int cn = i * n_mu + j;
          rho = M.rho[cn];
          im = M.inv4pim[cn];
          if (fixT) Tfix = fixT[cn];
          if (L.vis) atomicAdd(&L.vis[cn], 1u); else atomicAdd(&A.t.visits[cn], 1u);
        }
        Tc = -1.0;
        mrw_T = -2.0;
        n_int = 0;
      } else {
        // interaction in the cell
        double sint = tau / alpha;
        p[0] += sint * d[0]; p[1] += sint * d[1]; p[2] += sint * d[2];
        d_safe -= sint;
        dm_up += 1.000001 * sint;
        const double* fz = A.frozen_T;
        if (rng.next() < L.omega[k]) {
          ++pc_scat;
          iso64(rng, d);
        } else {
          ++pc_abs;
          ++cell_abs;
          // the tally update is in flight while the next draws are made
          double E_old = unsafeAtomicAdd(&A.t.E_abs[c], A.eps);
          double xb = rng.next();
          iso64(rng, d);
          if (fz) {
            k = reemit64(L, -1.0, Tfix, xb);
          } else {
            const double E_new = E_old + A.eps;
            double T_old = E_old == E_seen ? T_seen : T_of_g(L.tv, E_old * im);
            double T_new = T_of_g(L.tv, E_new * im);
            E_seen = E_new;
            T_seen = T_new;
            Tc = T_new;
            k = reemit64(L, T_old, T_new, xb);
          }
        }
        ++n_int;
        if (A.mrw) {
          // modified random walk while the start criterion holds
          while (n_int >= A.n_int_min) {
            double T_here;
            if (fixT) T_here = Tfix;
            else {
              if (Tc < 0.0)
                Tc = T_of_g(L.tv, __hip_atomic_load(&A.t.E_abs[c], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT) * im);
              T_here = Tc;
            }
            if (T_here != mrw_T) {  // MRW coefficients of this cell at this T
              mrw_T = T_here;
              mrw_Drho = interp_T(L.tv, L.tv.Drho, T_here);
              mrw_kbar = interp_T(L.tv, L.tv.kbar, T_here);
              double lam_R = 3.0 * mrw_Drho / rho;
              mrw_lim = A.gamma * lam_R;
            }
            const double Drho = mrw_Drho;
            if (dm_up <= mrw_lim) break;
            double dmin = min_boundary64(L, n_mu, i, j, p);
            d_safe = 0.999 * dmin;
            dm_up = 1.000001 * dmin;
            if (!(dmin > mrw_lim)) break;
            if (++events > A.max_events) break;
            double R0 = dmin * (1.0 - 1e-6);
            double s = mrw_escape_s(L.mrw_tab, rng.next());
            double ell = s * R0 * R0 * rho / Drho;  // c t = s R0^2 / D
            double dE = A.eps * rho * mrw_kbar * ell;
            double E_old = unsafeAtomicAdd(&A.t.E_abs[c], dE);
            double nrm[3];
            iso64(rng, nrm);
            p[0] += R0 * nrm[0]; p[1] += R0 * nrm[1]; p[2] += R0 * nrm[2];
            double xb = rng.next();
            iso64(rng, d);
            if (fz) {
              k = reemit64(L, -1.0, Tfix, xb);
            } else {
              const double E_new = E_old + dE;
              double T_old = E_old == E_seen ? T_seen : T_of_g(L.tv, E_old * im);
              double T_new = T_of_g(L.tv, E_new * im);
              E_seen = E_new;
              T_seen = T_new;
              Tc = T_new;
              k = reemit64(L, T_old, T_new, xb);
            }
            d_safe = 0.0;
            dm_up = INFINITY;
            ++pc_mrw;
            ++cell_mrw;
          }
        }
        tau = -log(rng.next());
      }
    }
    if (fate != 0) {
      if (cell_abs | cell_mrw) {  // the packet ended in a cell (capped)
        const int c = i * n_mu + j;
        if (i >= 0 && cell_abs) atomicAdd(&A.t.n_abs[c], cell_abs);
        if (i >= 0 && cell_mrw) atomicAdd(&A.t.n_mrw[c], cell_mrw);
        cell_abs = cell_mrw = 0;
      }
      E_seen = -1.0;
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
      // flush lane totals before they can overflow
      if (tot[C_CROSS] > 0x40000000u || tot[C_SCAT] > 0x40000000u || tot[C_ABS] > 0x40000000u ||
          tot[C_MRW] > 0x40000000u) {
        for (int q = 0; q < N_COUNTERS; ++q) {
          if (tot[q]) atomicAdd(&A.t.counters[q], (unsigned long long)tot[q]);
          tot[q] = 0;
        }
      }
    }
  }
  flush_counters(A.t.counters, tot, N_COUNTERS);
  if (L.vis) {
    __syncthreads();
    for (int a = threadIdx.x; a < n_r * n_mu; a += blockDim.x) {
      uint32_t v = L.vis[a];
      if (v) atomicAdd(&A.t.visits[a], v);
    }
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

template <int MODE>
int launch_mode(mcrt_ctx* ctx, const TraceArgs& a, size_t lds, hipStream_t s) {
  auto kern = trace_fp64_kernel<MODE>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) {
      set_error(ctx, std::string("LDS attribute: ") + hipGetErrorString(e));
      return MCRT_E_HIP;
    }
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, BS64, lds) != hipSuccess || occ < 1)
    occ = 1;
  int per_cu = ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : occ;
  long long nb = (long long)ctx->n_cu * per_cu;
  long long need = ((long long)a.n_packets + BS64 - 1) / BS64;
  if (nb > need) nb = need < 1 ? 1 : need;
  hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(BS64), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
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

// LDS: the small tables, the emission CDF in FP64, else its FP32 guide copy,
// else neither; then the visit histogram when that fits too.
int launch_trace_fp64(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s) {
  const DevModel& M = ctx->m;
  const size_t cap = 155 * 1024;
  size_t small = lds_small_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda);
  size_t c64 = (size_t)M.n_T * M.n_lambda * sizeof(double);
  size_t c32 = c64 / 2;
  const size_t vis = (size_t)4 * M.n_r * M.n_mu;
  TraceArgs b = a;
  if (small + c64 <= cap) {
    b.vis_lds = small + c64 + vis <= cap;
    return launch_mode<2>(ctx, b, small + c64 + (b.vis_lds ? vis : 0), s);
  }
  if (small + c32 <= cap) {
    b.vis_lds = small + c32 + vis <= cap;
    return launch_mode<1>(ctx, b, small + c32 + (b.vis_lds ? vis : 0), s);
  }
  b.vis_lds = small + vis <= cap;
  return launch_mode<0>(ctx, b, small + (b.vis_lds ? vis : 0), s);
}

}  // namespace mcrt
