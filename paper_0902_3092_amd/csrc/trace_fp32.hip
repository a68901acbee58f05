// Packet transport with FP32 cell-relative tracking.
//
// The packet position is an FP64 anchor A (set when the packet enters a cell
// and before each modified-random-walk jump) plus an FP32 offset q; the
// direction and the optical depth are FP32.  Face distances need
//   sphere e:  |p|^2 - r_e^2       = K_e + 2 A.q + q.q,   K_e = |A|^2 - r_e^2
//   cone   e:  z^2 - mu_e^2 |p|^2  = L_e + 2 (A_z q_z - mu_e^2 A.q) + (q_z^2 - mu_e^2 q.q),
//              L_e = A_z^2 - mu_e^2 |A|^2,
// where the constants K_e, L_e are formed in FP64 at the anchor and rounded
// once: the cancellation between |A|^2 and r_e^2 happens in FP64 and the
// FP32 terms scale with the offset (at most a cell) instead of the radius.
// In absolute FP32 coordinates a step in a cell of optical depth ~1e5 would
// be ~1e-4 of the cell, a few tens of ulps of the position: here it keeps
// FP32 relative precision of the cell size.
//
// Kept in FP64: the stellar launch and the flight through the central hole,
// the anchor, absorbed-energy tallies (atomics), temperature inversion, the
// MRW escape-time solve and deposit.  The reemission bin is searched in an
// FP32 copy of the emission CDF in LDS.
#include <hip/hip_runtime.h>

#include "mcrt_internal.h"
#include "rng.h"
#include "trace_common.h"

namespace mcrt {
namespace {

constexpr int BS32 = 512;

struct Lds32 {
  double *r2, *mu2, *mrw_tab;
  float *mu32, *smu32, *star_cdf, *chi, *omega;
  TabView tv;
  const float* cdf;
  uint32_t* vis;  // per-workgroup visit histogram [n_cells], or null
};

// Bytes of the tables; a visit histogram, when used, follows at this offset.
__host__ __device__ inline size_t lds32_bytes(int n_r, int n_mu, int n_T, int nl, bool with_cdf) {
  size_t dbl = (size_t)(n_r + 1) + (n_mu + 1) + MRW_TAB_N + 6 * (size_t)n_T;
  size_t flt = (size_t)2 * (n_mu + 1) + (size_t)3 * nl + (with_cdf ? (size_t)n_T * nl : 0);
  return dbl * 8 + N_GUIDE * 4 + ((flt * 4 + 7) & ~(size_t)7);
}

// Per-anchor constants of the four faces of cell (i, j).
struct Anchor {
  double A[3];
  float Af[3];
  float K_in, K_out, L_lo, L_hi;  // sphere r_i, r_i+1; cones mu_j, mu_j+1
};

__device__ __forceinline__ void set_anchor(Anchor& a, const Lds32& L, int n_mu, int i, int j) {
  double AA = a.A[0] * a.A[0] + a.A[1] * a.A[1] + a.A[2] * a.A[2];
  double Az2 = a.A[2] * a.A[2];
  a.K_in = (float)(AA - L.r2[i]);
  a.K_out = (float)(AA - L.r2[i + 1]);
  a.L_lo = j >= 1 ? (float)(Az2 - L.mu2[j] * AA) : 0.0f;
  a.L_hi = j + 1 < n_mu ? (float)(Az2 - L.mu2[j + 1] * AA) : 0.0f;
  a.Af[0] = (float)a.A[0];
  a.Af[1] = (float)a.A[1];
  a.Af[2] = (float)a.A[2];
}

__device__ __forceinline__ void reanchor(Anchor& a, float q[3], const Lds32& L, int n_mu, int i,
                                         int j) {
  a.A[0] += (double)q[0];
  a.A[1] += (double)q[1];
  a.A[2] += (double)q[2];
  q[0] = q[1] = q[2] = 0.0f;
  set_anchor(a, L, n_mu, i, j);
}

// Distance to the cell boundary along d and the face crossed.
__device__ __forceinline__ float boundary32(const Anchor& a, const Lds32& L, int n_mu, int i,
                                            int j, const float q[3], const float d[3], int& face) {
  float Ad = a.Af[0] * d[0] + a.Af[1] * d[1] + a.Af[2] * d[2];
  float qd = q[0] * d[0] + q[1] * d[1] + q[2] * d[2];
  float Aq = a.Af[0] * q[0] + a.Af[1] * q[1] + a.Af[2] * q[2];
  float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  float pd = Ad + qd;
  float best = exit_sphere<float>(pd, a.K_out + 2.0f * Aq + qq);
  face = 1;
  float s = enter_sphere<float>(pd, a.K_in + 2.0f * Aq + qq);
  if (s >= 0.0f && s < best) { best = s; face = 0; }
  float z = a.Af[2] + q[2];
  float dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  float zq = a.Af[2] * q[2];
  float qz2 = q[2] * q[2];
  if (j >= 1) {
    float m2 = (float)L.mu2[j];
    float C = a.L_lo + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    s = exit_cone<float>(d[2] * d[2] - m2 * dd, z * d[2] - m2 * pd, C, false);
    if (s >= 0.0f && s < best) { best = s; face = 2; }
  }
  if (j + 1 < n_mu) {
    float m2 = (float)L.mu2[j + 1];
    float C = a.L_hi + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    s = exit_cone<float>(d[2] * d[2] - m2 * dd, z * d[2] - m2 * pd, C, true);
    if (s >= 0.0f && s < best) { best = s; face = 3; }
  }
  return best;
}

// Lower bound of the distance to the cell boundary.  Spheres: (r^2 - r_e^2)/(r +
// r_e); cones: r sin|theta - theta_e| = (z^2 - mu_e^2 r^2) / (smu_e |z| + mu_e R),
// numerators from the anchored constants.
__device__ __forceinline__ float min_boundary32(const Anchor& a, const Lds32& L, int n_mu, int i,
                                                int j, const float q[3]) {
  float Aq = a.Af[0] * q[0] + a.Af[1] * q[1] + a.Af[2] * q[2];
  float qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
  float x = a.Af[0] + q[0], y = a.Af[1] + q[1], z = a.Af[2] + q[2];
  float R = sqrtf(x * x + y * y);
  float r = sqrtf(R * R + z * z);
  float ri = sqrtf((float)L.r2[i]), ro = sqrtf((float)L.r2[i + 1]);
  float dmin = fminf((a.K_in + 2.0f * Aq + qq) / (r + ri), -(a.K_out + 2.0f * Aq + qq) / (r + ro));
  float az = fabsf(z);
  float zq = a.Af[2] * q[2], qz2 = q[2] * q[2];
  if (j >= 1) {
    float m2 = (float)L.mu2[j];
    float f = a.L_lo + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    dmin = fminf(dmin, f / (L.smu32[j] * az + L.mu32[j] * R));
  }
  if (j + 1 < n_mu) {
    float m2 = (float)L.mu2[j + 1];
    float f = a.L_hi + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    dmin = fminf(dmin, -f / (L.smu32[j + 1] * az + L.mu32[j + 1] * R));
  }
  return dmin > 0.0f ? dmin : 0.0f;
}

__device__ __forceinline__ void iso32(Rng32& r, float d[3]) {
  float w = 2.0f * r.next() - 1.0f;
  float ph = 2.0f * (float)KPI * r.next();
  float st = sqrtf(fmaxf(0.0f, 1.0f - w * w));
  float sn, cs;
  __sincosf(ph, &sn, &cs);
  d[0] = st * cs;
  d[1] = st * sn;
  d[2] = w;
}

template <bool CDF_LDS>
__device__ __forceinline__ void trace_fp32_body(const TraceArgs& A) {
  extern __shared__ double smem[];
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda, n_T = M.n_T;
  Lds32 L;
  {
    double* q = smem;
    auto take = [&](double*& dst, const double* src, int n) {
      dst = q;
      for (int a = threadIdx.x; a < n; a += blockDim.x) q[a] = src[a];
      q += n;
    };
    double *Tn, *G, *Drho, *kbar;
    take(L.r2, M.r2, n_r + 1);
    take(L.mu2, M.mu2, n_mu + 1);
    take(L.mrw_tab, M.mrw_tab, MRW_TAB_N);
    take(Tn, M.Tn, n_T);
    take(G, M.G, n_T);
    take(Drho, M.Drho, n_T);
    take(kbar, M.kbar, n_T);
    double *invdT, *gslope;
    take(invdT, M.inv_dT, n_T);
    take(gslope, M.g_slope, n_T);
    int* gq = (int*)q;
    for (int a = threadIdx.x; a < N_GUIDE; a += blockDim.x) gq[a] = M.g_guide[a];
    float* f = (float*)(gq + N_GUIDE);
    auto takef = [&](float*& dst, int n, auto get) {
      dst = f;
      for (int a = threadIdx.x; a < n; a += blockDim.x) f[a] = get(a);
      f += n;
    };
    takef(L.mu32, n_mu + 1, [&](int a) { return (float)M.mu_edges[a]; });
    takef(L.smu32, n_mu + 1, [&](int a) { return (float)M.smu[a]; });
    takef(L.star_cdf, nl, [&](int a) { return M.star_cdf32[a]; });
    takef(L.chi, nl, [&](int a) { return M.chi32[a]; });
    takef(L.omega, nl, [&](int a) { return M.omega32[a]; });
    if (CDF_LDS) {
      float* c = f;
      for (int a = threadIdx.x; a < n_T * nl; a += blockDim.x) c[a] = M.cdf32[a];
      L.cdf = c;
    } else {
      L.cdf = M.cdf32;
    }
    L.tv = TabView{n_T, nl, M.lnT_lo, M.inv_dlnT, M.lnG0, M.inv_du, N_GUIDE, Tn, G, Drho, kbar,
                   gq, invdT, gslope};
    L.vis = nullptr;
    if (A.vis_lds) {
      L.vis = (uint32_t*)((char*)smem + lds32_bytes(n_r, n_mu, n_T, nl, CDF_LDS));
      for (int a = threadIdx.x; a < n_r * n_mu; a += blockDim.x) L.vis[a] = 0u;
    }
  }
  __syncthreads();

  const int lane = __lane_id();
  bool alive = false, exhausted = false;
  Rng32 rng;
  Anchor an;
  float q[3] = {0, 0, 0}, d[3] = {0, 0, 1}, tau = 0.0f;
  int k = 0, i = -1, j = 0, n_int = 0;
  long long events = 0;
  uint64_t pid = 0;
  uint32_t pc_cross = 0, pc_scat = 0, pc_abs = 0, pc_mrw = 0;
  double rho = 0.0;
  double Tc = -1.0;     // running temperature of the cell (lazily from its tally)
  double im = 0.0;      // 1 / (4 pi m) of the cell
  double Tfix = 0.0;    // the cell's fixed temperature (frozen field or MRW coefficient field)
  const double* fixT = A.frozen_T ? A.frozen_T : A.T_coef;
  double mrw_T = -2.0, mrw_Drho = 0.0, mrw_kbar = 0.0;  // MRW coefficients at mrw_T
  float mrw_lim = 0.0f;
  float d_safe = 0.0f;  // lower bound of the distance to every face of the cell
  // upper bound of that distance (the last computed one plus the path flown
  // since): while it is within the MRW limit the criterion cannot hold
  float dm_up = INFINITY;
  uint32_t tot[N_COUNTERS] = {0, 0, 0, 0, 0, 0, 0, 0};
  // absorptions and MRW steps in the current cell, added to the tallies when
  // the packet leaves it; the cell's tally after this lane's last deposit and
  // its temperature (reused when no other packet deposited in between)
  uint32_t cell_abs = 0, cell_mrw = 0;
  double E_seen = -1.0, T_seen = 0.0;

  for (;;) {
    unsigned long long idle = __ballot(!alive);
    if (idle != 0ull && !exhausted) {
      int cnt = __popcll(idle);
      int leader = __ffsll((long long)idle) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(A.next, (unsigned long long)cnt);
      base = __shfl(base, leader);
      if (base + cnt >= A.n_packets) exhausted = true;
      if (!alive) {
        unsigned long long qq = base + (unsigned long long)__popcll(idle & ((1ull << lane) - 1ull));
        if (qq < A.n_packets) {
          pid = A.offset + qq;
          rng.init(A.key0, A.key1, pid);
          // launch on the star (FP64 position), Lambertian outward direction
          float ws = 2.0f * rng.next() - 1.0f;
          float st = sqrtf(fmaxf(0.0f, 1.0f - ws * ws));
          an.A[0] = M.R_star * (double)st;
          an.A[1] = 0.0;
          an.A[2] = M.R_star * (double)ws;
          float mup = sqrtf(rng.next());
          float php = 2.0f * (float)KPI * rng.next();
          float sp = sqrtf(fmaxf(0.0f, 1.0f - mup * mup));
          float sn, cs;
          __sincosf(php, &sn, &cs);
          d[0] = mup * st + sp * cs * ws;
          d[1] = sp * sn;
          d[2] = mup * ws - sp * cs * st;
          float nrm = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
          d[0] *= nrm; d[1] *= nrm; d[2] *= nrm;
          float xs = rng.next();
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (L.star_cdf[mid] > xs) hi = mid; else lo = mid + 1;
          }
          k = lo;
          tau = -__logf(rng.next());
          q[0] = q[1] = q[2] = 0.0f;
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
      // central hole, FP64: the star or the inner grid sphere
      double P[3] = {an.A[0] + (double)q[0], an.A[1] + (double)q[1], an.A[2] + (double)q[2]};
      double D[3] = {(double)d[0], (double)d[1], (double)d[2]};
      double pd = P[0] * D[0] + P[1] * D[1] + P[2] * D[2];
      double rr = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
      double s = enter_sphere<double>(pd, rr - M.R_star * M.R_star);
      q[0] = q[1] = q[2] = 0.0f;
      if (s >= 0.0) {
        an.A[0] = P[0] + s * D[0]; an.A[1] = P[1] + s * D[1]; an.A[2] = P[2] + s * D[2];
        fate = 2;
      } else {
        s = exit_sphere<double>(pd, rr - L.r2[0]);
        an.A[0] = P[0] + s * D[0]; an.A[1] = P[1] + s * D[1]; an.A[2] = P[2] + s * D[2];
        i = 0;
        double r2 = (an.A[0] * an.A[0] + an.A[1] * an.A[1]) + an.A[2] * an.A[2];
        j = mu_row(L.mu2, n_mu, r2, an.A[2] * an.A[2]);
        set_anchor(an, L, n_mu, i, j);
        rho = M.rho[j];
        im = M.inv4pim[j];
        if (fixT) Tfix = fixT[j];
        if (L.vis) atomicAdd(&L.vis[j], 1u); else atomicAdd(&A.t.visits[j], 1u);
        Tc = -1.0;
        mrw_T = -2.0;
        d_safe = 0.0f;
        dm_up = INFINITY;
        n_int = 0;
        ++pc_cross;
      }
    } else {
      const int c = i * n_mu + j;
      const float alpha = (float)rho * L.chi[k];
      int face = 1;
      float sb = 0.0f, tau_b = 0.0f;
      // a flight shorter than the guaranteed distance to every face stays in
      // the cell: the face distances are not needed for it
      const bool inside = tau < alpha * d_safe;
      if (!inside) {
        sb = boundary32(an, L, n_mu, i, j, q, d, face);
        tau_b = alpha * sb;
      }
      if (!inside && tau_b <= tau) {
        d_safe = 0.0f;
        dm_up = INFINITY;
        if (cell_abs) { atomicAdd(&A.t.n_abs[c], cell_abs); cell_abs = 0; }
        if (cell_mrw) { atomicAdd(&A.t.n_mrw[c], cell_mrw); cell_mrw = 0; }
        E_seen = -1.0;
        q[0] += sb * d[0]; q[1] += sb * d[1]; q[2] += sb * d[2];
        tau -= tau_b;
        if (tau < 0.0f) tau = 0.0f;
        ++pc_cross;
        bool entered = true;
        if (face == 1) {
          if (i + 1 == n_r) {
            int m = (int)(fabsf(d[2]) * M.n_inc);
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
          reanchor(an, q, L, n_mu, i, j);
          if (L.vis) atomicAdd(&L.vis[cn], 1u); else atomicAdd(&A.t.visits[cn], 1u);
        } else if (fate == 0) {
          // into the hole: keep the FP64 position in the anchor
          an.A[0] += (double)q[0]; an.A[1] += (double)q[1]; an.A[2] += (double)q[2];
          q[0] = q[1] = q[2] = 0.0f;
        }
        Tc = -1.0;
        mrw_T = -2.0;
        n_int = 0;
      } else {
        float sint = tau / alpha;
        q[0] += sint * d[0]; q[1] += sint * d[1]; q[2] += sint * d[2];
        d_safe -= sint;
        dm_up += 1.00001f * sint;
        const double* fz = A.frozen_T;
        if (rng.next() < L.omega[k]) {
          ++pc_scat;
          iso32(rng, d);
        } else {
          ++pc_abs;
          ++cell_abs;
          // the tally update is in flight while the next draws are made
          double E_old = unsafeAtomicAdd(&A.t.E_abs[c], A.eps);
          float xb = rng.next();
          iso32(rng, d);
          double T_old = -1.0, T_new;
          if (fz) {
            T_new = Tfix;
          } else {
            const double E_new = E_old + A.eps;
            T_old = E_old == E_seen ? T_seen : T_of_g(L.tv, E_old * im);
            T_new = T_of_g(L.tv, E_new * im);
            E_seen = E_new;
            T_seen = T_new;
            Tc = T_new;
          }
          Reemit<float> R = reemit_setup<float>(L.tv, L.cdf, T_old, T_new);
          k = reemit_search<float>(R, nl, xb);
        }
        ++n_int;
        if (A.mrw) {
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
              mrw_lim = (float)(A.gamma * 3.0 * mrw_Drho / rho);
            }
            const double Drho = mrw_Drho;
            const float lim = mrw_lim;
            if (dm_up <= lim) break;
            {
              float dm = min_boundary32(an, L, n_mu, i, j, q);
              d_safe = 0.999f * dm;
              dm_up = 1.00001f * dm;
              if (!(dm > lim)) break;
            }
            // re-anchor so the sphere radius is exact to FP32 precision of itself
            reanchor(an, q, L, n_mu, i, j);
            float dmin = min_boundary32(an, L, n_mu, i, j, q);
            if (!(dmin > lim)) break;
            if (++events > A.max_events) break;
            double R0 = (double)dmin * (1.0 - 1e-5);
            double P0 = (double)rng.next();
            double s = mrw_escape_s(L.mrw_tab, P0);
            double ell = s * R0 * R0 * rho / Drho;
            double dE = A.eps * rho * mrw_kbar * ell;
            double E_old = unsafeAtomicAdd(&A.t.E_abs[c], dE);
            float nv[3];
            iso32(rng, nv);
            q[0] = (float)R0 * nv[0]; q[1] = (float)R0 * nv[1]; q[2] = (float)R0 * nv[2];
            float xb = rng.next();
            iso32(rng, d);
            double T_old = -1.0, T_new;
            if (fz) {
              T_new = Tfix;
            } else {
              const double E_new = E_old + dE;
              T_old = E_old == E_seen ? T_seen : T_of_g(L.tv, E_old * im);
              T_new = T_of_g(L.tv, E_new * im);
              E_seen = E_new;
              T_seen = T_new;
              Tc = T_new;
            }
            Reemit<float> R = reemit_setup<float>(L.tv, L.cdf, T_old, T_new);
            k = reemit_search<float>(R, nl, xb);
            d_safe = 0.0f;
            dm_up = INFINITY;
            ++pc_mrw;
            ++cell_mrw;
          }
        }
        tau = -__logf(rng.next());
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
          mcrt_packet_rec& Rr = A.recs[r];
          Rr.fate = fate;
          Rr.k = k;
          Rr.n_cross = pc_cross;
          Rr.n_scat = pc_scat;
          Rr.n_abs = pc_abs;
          Rr.n_mrw = pc_mrw;
          Rr.n_draws = (int64_t)rng.draws();
          Rr.x = an.A[0] + q[0]; Rr.y = an.A[1] + q[1]; Rr.z = an.A[2] + q[2];
          Rr.u = d[0]; Rr.v = d[1]; Rr.w = d[2];
        }
      }
      alive = false;
      if (tot[C_CROSS] > 0x40000000u || tot[C_SCAT] > 0x40000000u || tot[C_ABS] > 0x40000000u ||
          tot[C_MRW] > 0x40000000u) {
        for (int t = 0; t < N_COUNTERS; ++t) {
          if (tot[t]) atomicAdd(&A.t.counters[t], (unsigned long long)tot[t]);
          tot[t] = 0;
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

template <bool CDF_LDS>
__global__ void __launch_bounds__(BS32) trace_fp32_kernel(TraceArgs A) {
  trace_fp32_body<CDF_LDS>(A);
}

// Many disks in one launch: workgroup b works on disk block_disk[b] for the
// whole launch (its tables stay in LDS), taking packets from that disk's
// counter; workgroups are shared out in proportion to the disks' packets.
template <bool CDF_LDS>
__global__ void __launch_bounds__(BS32) trace_fp32_batch_kernel(const TraceArgs* __restrict__ As,
                                                                const int* __restrict__ block_disk) {
  trace_fp32_body<CDF_LDS>(As[block_disk[blockIdx.x]]);
}

template <bool CDF_LDS>
int launch32(mcrt_ctx* ctx, const TraceArgs& a, size_t lds, hipStream_t s) {
  auto kern = trace_fp32_kernel<CDF_LDS>;
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, BS32, lds) != hipSuccess || occ < 1)
    occ = 1;
  int per_cu = ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : occ;
  long long nb = (long long)ctx->n_cu * per_cu;
  long long need = ((long long)a.n_packets + BS32 - 1) / BS32;
  if (nb > need) nb = need < 1 ? 1 : need;
  hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(BS32), lds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

}  // namespace

// LDS: the tables (with the emission CDF when it fits), then the visit
// histogram when that fits too.
int launch_trace_fp32(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s) {
  const DevModel& M = ctx->m;
  const size_t cap = 155 * 1024;
  const size_t vis = (size_t)4 * M.n_r * M.n_mu;
  TraceArgs b = a;
  size_t with = lds32_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda, true);
  if (with <= cap) {
    b.vis_lds = with + vis <= cap;
    return launch32<true>(ctx, b, b.vis_lds ? with + vis : with, s);
  }
  size_t without = lds32_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda, false);
  b.vis_lds = without + vis <= cap;
  return launch32<false>(ctx, b, b.vis_lds ? without + vis : without, s);
}

size_t trace_fp32_lds(const DevModel& M, bool with_cdf) {
  return lds32_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda, with_cdf);
}

size_t trace_fp32_lds_cap() { return 155 * 1024; }

int trace_fp32_blocks_per_cu(size_t lds, bool cdf_lds) {
  int occ = 0;
  hipError_t e = cdf_lds ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, trace_fp32_batch_kernel<true>, BS32, lds)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &occ, trace_fp32_batch_kernel<false>, BS32, lds);
  return (e != hipSuccess || occ < 1) ? 1 : occ;
}

// Kernel attributes are set here, outside any stream capture.
int prepare_trace_fp32_batch(size_t lds, bool cdf_lds) {
  if (lds <= 64 * 1024) return MCRT_OK;
  hipError_t e = cdf_lds ? hipFuncSetAttribute((const void*)trace_fp32_batch_kernel<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
                         : hipFuncSetAttribute((const void*)trace_fp32_batch_kernel<false>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)e;  // not needed on every runtime; a real limit shows at launch
  (void)hipGetLastError();
  return MCRT_OK;
}

int launch_trace_fp32_batch(const TraceArgs* d_args, const int* d_block_disk, int n_blocks,
                            size_t lds, bool cdf_lds, hipStream_t s) {
  if (cdf_lds)
    hipLaunchKernelGGL(trace_fp32_batch_kernel<true>, dim3(n_blocks), dim3(BS32), lds, s, d_args,
                       d_block_disk);
  else
    hipLaunchKernelGGL(trace_fp32_batch_kernel<false>, dim3(n_blocks), dim3(BS32), lds, s, d_args,
                       d_block_disk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(nullptr, std::string("batched trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

}  // namespace mcrt
