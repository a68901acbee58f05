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

// nn / no >= 0: the segments of T_new / T_old, known from their inversion
__device__ __forceinline__ int reemit64(const Lds64& L, double T_old, double T_new, double xi,
                                        int nn = -1, int no = -1) {
  const int nl = L.tv.nl;
  Reemit<double> R = reemit_setup<double>(L.tv, L.cdf64, T_old, T_new, nn, no);
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

// Functions of one draw u used by the transport (both generators evaluate
// them with these functions, so they give the same values).
__device__ __forceinline__ double iso_mu64(double u) { return 2.0 * u - 1.0; }
__device__ __forceinline__ double iso_st64(double u) {
  const double w = iso_mu64(u);
  return sqrt(fmax(0.0, 1.0 - w * w));
}
__device__ __forceinline__ void iso_phi64(double u, double& sn, double& cs) {
  sincos(2.0 * KPI * u, &sn, &cs);
}
__device__ __forceinline__ double tau_of64(double u) { return -log(u); }

__device__ __forceinline__ void iso64(Rng64& r, double d[3]) {
  const double u1 = r.next();
  const double u2 = r.next();
  double sn, cs;
  iso_phi64(u2, sn, cs);
  const double st = iso_st64(u1);
  d[0] = st * cs;
  d[1] = st * sn;
  d[2] = iso_mu64(u1);
}
__device__ __forceinline__ double tau64(Rng64& r) { return tau_of64(r.next()); }
// the two draws of a scattering: the first raw (the scattering angle), the
// second as the sine and cosine of its azimuth
__device__ __forceinline__ void scat_draws(Rng64& r, double& u1, double& sn, double& cs) {
  u1 = r.next();
  iso_phi64(r.next(), sn, cs);
}

// Direction after a scattering by the Henyey-Greenstein phase function with
// asymmetry g != 0: the cosine of the scattering angle from the inverse of
// its cumulative distribution at u1, the azimuth (sine sn, cosine cs) about
// the old direction.
__device__ __forceinline__ void hg_turn64(double g, double u1, double sn, double cs, double d[3]) {
  const double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u1);
  const double mu = fmin(1.0, fmax(-1.0, (1.0 + g * g - q * q) / (2.0 * g)));
  const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  const double x = d[0], y = d[1], z = d[2];
  const double s = sqrt(x * x + y * y);  // sine of the polar angle of d
  if (s == 0.0) {
    d[0] = st * cs;
    d[1] = st * sn;
    d[2] = z > 0.0 ? mu : -mu;
  } else {
    d[0] = st * (x * z * cs - y * sn) / s + x * mu;
    d[1] = st * (y * z * cs + x * sn) / s + y * mu;
    d[2] = -st * cs * s + z * mu;
  }
}
__device__ __forceinline__ void ensure_draws(Rng64&, int) {}

// ------------------------------------------------------------------ packets
struct Pk64 {
  double p[3], d[3], tau;
  int k, i, j, n_int;
  long long events;
  uint32_t pc_cross, pc_scat, pc_abs, pc_mrw;
  double rho;                        // density of the cell
  double im;                         // 1 / (4 pi m) of the cell
  double Tc;                         // running temperature of the cell (< 0: not known)
  double Tfix;                       // the cell's fixed temperature (frozen or MRW field)
  double mrw_T, mrw_Drho, mrw_f, mrw_lim;  // MRW coefficients at mrw_T (mrw_f: its
  int mrw_seg, seg_seen;                    // fraction in segment mrw_seg); segment of T_seen
  double alpha, omega;  // extinction rho chi_k of the cell at bin k, and the albedo at k
  // bounds of the distance to the cell boundary: d_safe below (a flight
  // shorter than it stays in the cell, so the face distances are not needed),
  // dm_up above (the last computed distance plus the path flown since: while
  // it is within the MRW limit the criterion cannot hold)
  double d_safe, dm_up;
  // absorptions and MRW steps in this stay in the cell, added to the tallies
  // when the packet leaves it; the cell's tally after this packet's last
  // deposit (or as last read) and its temperature (reused when nobody
  // deposited in between)
  uint32_t cell_abs, cell_mrw;
  double E_seen, T_seen;
};

// A packet handed over to the whole-wavefront launch.
struct TailState64 {
  Pk64 P;
  Rng64 rng;
  uint64_t pid;
};
static_assert(sizeof(TailState64) <= TAIL_STATE_BYTES, "hand-off slot");

// ------------------------------------------------------ whole-wave mode
// As in the FP32 tracker: once all packets are handed out, long packets are
// continued by a second launch, a whole wavefront each (uniform control
// flow, one Philox pass for 64 draws with their logarithms, square roots
// and sines computed lane-parallel, 64-wide reemission search).
__device__ __forceinline__ double bcd0(double v) {
  const long long x = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 0);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)x >> 32), 0);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double bcd(double v, int l) {
  const long long x = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)x >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// One packet's stream (the same draws as Rng64) for a wavefront: the buffer is
// the 64 draws of Philox blocks blk0 .. blk0 + 31, draw p held by lane p
// (lanes 2b and 2b + 1 generate block blk0 + b and keep one draw each), so a
// draw is read from a fixed register at a uniform lane index.
struct WaveRng64 {
  uint64_t pid;
  uint32_t k0, k1;
  uint64_t blk0;
  int pos;        // next draw of the buffer, 0..63 (the stream's draw 2 blk0 + pos)
  double u, tau, st, sn, cs;  // this lane's draw

  __device__ __forceinline__ void fill() {
    const uint32_t lane = (uint32_t)__lane_id();
    const uint64_t blk = blk0 + (uint64_t)(lane >> 1);
    uint32_t c0 = (uint32_t)pid, c1 = (uint32_t)(pid >> 32), c2 = (uint32_t)blk,
             c3 = (uint32_t)(blk >> 32);
    philox4x32_10(c0, c1, c2, c3, k0, k1);
    u = (lane & 1u) ? Rng64::unit(c2, c3) : Rng64::unit(c0, c1);
    tau = tau_of64(u);
    st = iso_st64(u);
    iso_phi64(u, sn, cs);
  }
  __device__ __forceinline__ void init(const Rng64& r) {
    pid = r.pid;
    k0 = r.k0;
    k1 = r.k1;
    const uint64_t nd = r.d;  // index of the next draw
    blk0 = nd >> 1;
    pos = (int)(nd & 1);
    fill();
  }
  __device__ __forceinline__ double at(double x, int p) const { return bcd(x, p); }
  // at least n draws left in the buffer: else restart it at the block of
  // the next draw (the generator is inlined where a segment begins only)
  __device__ __forceinline__ void ensure(int n) {
    if (pos + n > 64) {
      blk0 += (uint64_t)(pos >> 1);
      pos &= 1;
      fill();
    }
  }
  __device__ __forceinline__ int take() { return pos++; }
  __device__ __forceinline__ double next() { return at(u, take()); }
  __device__ __forceinline__ double next_tau() { return at(tau, take()); }
  __device__ __forceinline__ void next_iso(double d[3]) {
    const int p1 = take();
    const double w = iso_mu64(at(u, p1)), s = at(st, p1);
    const int p2 = take();
    const double cs_ = at(cs, p2), sn_ = at(sn, p2);
    d[0] = s * cs_;
    d[1] = s * sn_;
    d[2] = w;
  }
  __device__ __forceinline__ void next_scat(double& u1, double& sn_, double& cs_) {
    const int p1 = take();
    u1 = at(u, p1);
    const int p2 = take();
    cs_ = at(cs, p2);
    sn_ = at(sn, p2);
  }
  __device__ __forceinline__ uint64_t nd_value() const { return blk0 * 2u + (uint64_t)pos; }
};

__device__ __forceinline__ void iso64(WaveRng64& r, double d[3]) { r.next_iso(d); }
__device__ __forceinline__ double tau64(WaveRng64& r) { return r.next_tau(); }
__device__ __forceinline__ void ensure_draws(WaveRng64& r, int n) { r.ensure(n); }
__device__ __forceinline__ void scat_draws(WaveRng64& r, double& u1, double& sn, double& cs) {
  r.next_scat(u1, sn, cs);
}

// smallest k with D(k) > xi D(nl-1) (nl - 1 if none), one bin per lane
__device__ __forceinline__ int reemit64_wave(const Lds64& L, double T_old, double T_new, double xi,
                                             int nn = -1, int no = -1) {
  const int nl = L.tv.nl;
  Reemit<double> R = reemit_setup<double>(L.tv, L.cdf64, T_old, T_new, nn, no);
  const double target = xi * R.D(nl - 1);
  const int lane = __lane_id();
  for (int base = 0; base < nl; base += 64) {
    const int kk = base + lane < nl ? base + lane : nl - 1;
    const unsigned long long m = __ballot(base + lane < nl && R.D(kk) > target);
    if (m) return base + __ffsll((long long)m) - 1;
  }
  return nl - 1;
}

// One event of packet P (see the FP32 tracker for the structure).  WAVE: all
// lanes hold P; lane 0 issues the memory updates.
template <bool WAVE, class RNG>
__device__ __forceinline__ int event64(Pk64& P, RNG& rng, const TraceArgs& A, const Lds64& L,
                                       const double* fixT, int lane) {
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu;
  const bool issuer = !WAVE || lane == 0;
  auto visit = [&](int cn) {
    if (issuer) {
      if (L.vis) atomicAdd(&L.vis[cn], 1u); else atomicAdd(&A.t.visits[cn], 1u);
    }
  };
  auto deposit = [&](int c, double dE) -> double {
    double E_old = 0.0;
    if (WAVE) {
      if (issuer) E_old = unsafeAtomicAdd(&A.t.E_abs[c], dE);
    } else {
      E_old = tally_add_grouped(A.t.E_abs, c, dE);
    }
    // the odd-numbered packets' share, kept apart for the noise estimate
    if (issuer && A.t.E_half && (rng.pid & 1)) unsafeAtomicAdd(&A.t.E_half[c], dE);
    if (WAVE) E_old = bcd0(E_old);
    return E_old;
  };
  auto reemit = [&](double T_old, double T_new, double xb, int nn = -1, int no = -1) -> int {
    if (WAVE) return reemit64_wave(L, T_old, T_new, xb, nn, no);
    return reemit64(L, T_old, T_new, xb, nn, no);
  };
  // bin of the reemission after a deposit dE on top of the tally E_old: the
  // temperatures before and after from the inversion, whose table segments
  // the spectrum interpolation reuses
  auto reemit_after = [&](double E_old, double dE, double xb) -> int {
    int n_old, n_new;
    double T_old;
    if (E_old == P.E_seen) {
      T_old = P.T_seen;
      n_old = P.seg_seen;
    } else {
      T_old = T_of_g_seg_near(L.tv, E_old * P.im, P.seg_seen, n_old);
    }
    const double E_new = E_old + dE;
    const double T_new = T_of_g_seg_near(L.tv, E_new * P.im, n_old, n_new);
    P.E_seen = E_new;
    P.T_seen = T_new;
    P.seg_seen = n_new;
    P.Tc = T_new;
    return reemit(T_old, T_new, xb, n_new, n_old);
  };
  int fate = 0;
  if (++P.events > A.max_events) {
    fate = 3;
  } else if (P.i < 0) {
    // central hole: free flight to the star or to the inner grid sphere
    double pd = P.p[0] * P.d[0] + P.p[1] * P.d[1] + P.p[2] * P.d[2];
    double rr = P.p[0] * P.p[0] + P.p[1] * P.p[1] + P.p[2] * P.p[2];
    double s = enter_sphere<double>(pd, rr - M.R_star * M.R_star);
    if (s >= 0.0) {
      P.p[0] += s * P.d[0]; P.p[1] += s * P.d[1]; P.p[2] += s * P.d[2];
      fate = 2;
    } else {
      s = exit_sphere<double>(pd, rr - L.r2[0]);
      P.p[0] += s * P.d[0]; P.p[1] += s * P.d[1]; P.p[2] += s * P.d[2];
      P.i = 0;
      double r2 = (P.p[0] * P.p[0] + P.p[1] * P.p[1]) + P.p[2] * P.p[2];
      P.j = mu_row(L.mu2, n_mu, r2, P.p[2] * P.p[2]);
      P.rho = M.rho[P.j];
      P.alpha = P.rho * L.chi[P.k];
      P.omega = L.omega[P.k];
      P.im = M.inv4pim[P.j];
      if (fixT) P.Tfix = fixT[P.j];
      visit(P.j);
      P.Tc = -1.0;
      P.mrw_T = -2.0;
      P.d_safe = 0.0;
      P.dm_up = INFINITY;
      P.n_int = 0;
      ++P.pc_cross;
    }
  } else {
    const int c = P.i * n_mu + P.j;
    const double alpha = P.alpha;
    int face = 1;
    double sb = 0.0, tau_b = 0.0;
    const bool inside = P.tau < alpha * P.d_safe;
    if (!inside) {
      sb = boundary64(L, n_mu, P.i, P.j, P.p, P.d, face);
      tau_b = alpha * sb;
    }
    if (!inside && tau_b <= P.tau) {
      // path-length tally of the mean intensity (when kept)
      if (issuer && A.t.path) unsafeAtomicAdd(&A.t.path[(size_t)c * M.n_lambda + P.k], A.eps * sb);
      if (issuer && P.cell_abs) atomicAdd(&A.t.n_abs[c], P.cell_abs);
      if (issuer && P.cell_mrw) atomicAdd(&A.t.n_mrw[c], P.cell_mrw);
      P.cell_abs = P.cell_mrw = 0;
      P.E_seen = -1.0;
      P.d_safe = 0.0;
      P.dm_up = INFINITY;
      P.p[0] += sb * P.d[0]; P.p[1] += sb * P.d[1]; P.p[2] += sb * P.d[2];
      P.tau -= tau_b;
      ++P.pc_cross;
      bool entered = true;
      if (face == 1) {
        if (P.i + 1 == n_r) {
          int m = (int)(fabs(P.d[2]) * M.n_inc);
          m = m < M.n_inc ? m : M.n_inc - 1;
          if (issuer) unsafeAtomicAdd(&A.t.sed[P.k * M.n_inc + m], A.eps);
          fate = 1;
          entered = false;
        } else {
          ++P.i;
        }
      } else if (face == 0) {
        --P.i;
        if (P.i < 0) entered = false;
      } else if (face == 2) {
        --P.j;
      } else {
        ++P.j;
      }
      if (entered) {
        int cn = P.i * n_mu + P.j;
        P.rho = M.rho[cn];
        P.alpha = P.rho * L.chi[P.k];
        P.im = M.inv4pim[cn];
        if (fixT) P.Tfix = fixT[cn];
        visit(cn);
      }
      P.Tc = -1.0;
      P.mrw_T = -2.0;
      P.n_int = 0;
    } else {
      // interaction in the cell
      double sint = P.tau / alpha;
      if (issuer && A.t.path) unsafeAtomicAdd(&A.t.path[(size_t)c * M.n_lambda + P.k], A.eps * sint);
      P.p[0] += sint * P.d[0]; P.p[1] += sint * P.d[1]; P.p[2] += sint * P.d[2];
      P.d_safe -= sint;
      P.dm_up += 1.000001 * sint;
      const double* fz = A.frozen_T;
      ensure_draws(rng, 6);  // albedo, bin, direction, optical depth
      if (rng.next() < P.omega) {
        ++P.pc_scat;
        if (A.g_asym != 0.0) {
          double u1, sn, cs;
          scat_draws(rng, u1, sn, cs);
          hg_turn64(A.g_asym, u1, sn, cs, P.d);
        } else {
          iso64(rng, P.d);
        }
      } else {
        ++P.pc_abs;
        ++P.cell_abs;
        // the tally update is in flight while the next draws are made
        double E_old = deposit(c, A.eps);
        double xb = rng.next();
        iso64(rng, P.d);
        P.k = fz ? reemit(-1.0, P.Tfix, xb) : reemit_after(E_old, A.eps, xb);
        P.alpha = P.rho * L.chi[P.k];
        P.omega = L.omega[P.k];
      }
      ++P.n_int;
      if (A.mrw) {
        // modified random walk while the start criterion holds
        while (P.n_int >= A.n_int_min) {
          double T_here;
          if (fixT) T_here = P.Tfix;
          else {
            if (P.Tc < 0.0) {
              // the cell's running T from its tally, kept as the last tally
              // seen so the coefficients and the next reemission reuse its
              // segment (a neighbouring cell's segment is the first guess)
              const double E_c = __hip_atomic_load(&A.t.E_abs[c], __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
              int n_c;
              P.Tc = T_of_g_seg_near(L.tv, E_c * P.im, P.seg_seen, n_c);
              P.E_seen = E_c;
              P.T_seen = P.Tc;
              P.seg_seen = n_c;
            }
            T_here = P.Tc;
          }
          if (T_here != P.mrw_T) {  // MRW coefficients of this cell at this T
            // (the segment of the running T is known from its inversion)
            const int n = T_here == P.T_seen ? P.seg_seen : t_segment(L.tv, T_here);
            const double f = (T_here - L.tv.Tn[n]) * L.tv.inv_dT[n];
            P.mrw_T = T_here;
            P.mrw_seg = n;
            P.mrw_f = f;
            P.mrw_Drho = L.tv.Drho[n] + f * (L.tv.Drho[n + 1] - L.tv.Drho[n]);
            double lam_R = 3.0 * P.mrw_Drho / P.rho;
            P.mrw_lim = A.gamma * lam_R;
          }
          const double Drho = P.mrw_Drho;
          if (P.dm_up <= P.mrw_lim) break;
          double dmin = min_boundary64(L, n_mu, P.i, P.j, P.p);
          P.d_safe = 0.999 * dmin;
          P.dm_up = 1.000001 * dmin;
          if (!(dmin > P.mrw_lim)) break;
          if (++P.events > A.max_events) break;
          ensure_draws(rng, 7);  // escape time, jump, bin, direction, optical depth
          double R0 = dmin * (1.0 - 1e-6);
          double s = mrw_escape_s(L.mrw_tab, rng.next());
          double ell = s * R0 * R0 * P.rho / Drho;  // c t = s R0^2 / D
          const int ns = P.mrw_seg;
          const double kbar = L.tv.kbar[ns] + P.mrw_f * (L.tv.kbar[ns + 1] - L.tv.kbar[ns]);
          double dE = A.eps * P.rho * kbar * ell;
          if (issuer && A.t.path) unsafeAtomicAdd(&A.t.mrw_path[c], A.eps * ell);
          double E_old = deposit(c, dE);
          double nrm[3];
          iso64(rng, nrm);
          P.p[0] += R0 * nrm[0]; P.p[1] += R0 * nrm[1]; P.p[2] += R0 * nrm[2];
          double xb = rng.next();
          iso64(rng, P.d);
          P.k = fz ? reemit(-1.0, P.Tfix, xb) : reemit_after(E_old, dE, xb);
          P.alpha = P.rho * L.chi[P.k];
          P.omega = L.omega[P.k];
          P.d_safe = 0.0;
          P.dm_up = INFINITY;
          ++P.pc_mrw;
          ++P.cell_mrw;
        }
      }
      P.tau = tau64(rng);
    }
  }
  return fate;
}

template <bool WAVE, class RNG>
__device__ __forceinline__ void finish64(Pk64& P, const RNG& rng_draws, int fate, uint64_t pid,
                                         const TraceArgs& A, uint32_t* tot, int lane) {
  const int n_mu = A.m.n_mu;
  if (!WAVE || lane == 0) {
    if (P.i >= 0 && (P.cell_abs | P.cell_mrw)) {  // the packet ended in a cell (capped)
      const int c = P.i * n_mu + P.j;
      if (P.cell_abs) atomicAdd(&A.t.n_abs[c], P.cell_abs);
      if (P.cell_mrw) atomicAdd(&A.t.n_mrw[c], P.cell_mrw);
    }
    if (fate == 1) tot[C_ESCAPED]++;
    else if (fate == 2) { tot[C_STAR]++; unsafeAtomicAdd(A.t.E_star, A.eps); }
    else tot[C_CAPPED]++;
    tot[C_CROSS] += P.pc_cross;
    tot[C_SCAT] += P.pc_scat;
    tot[C_ABS] += P.pc_abs;
    tot[C_MRW] += P.pc_mrw;
    if (A.recs) {
      int64_t r = (int64_t)(pid - A.offset);
      if (r >= 0 && r < A.n_recs) {
        mcrt_packet_rec& R = A.recs[r];
        R.fate = fate;
        R.k = P.k;
        R.n_cross = P.pc_cross;
        R.n_scat = P.pc_scat;
        R.n_abs = P.pc_abs;
        R.n_mrw = P.pc_mrw;
        R.n_draws = (int64_t)rng_draws.nd_value();
        R.x = P.p[0]; R.y = P.p[1]; R.z = P.p[2];
        R.u = P.d[0]; R.v = P.d[1]; R.w = P.d[2];
      }
    }
  }
  P.cell_abs = P.cell_mrw = 0;
  P.E_seen = -1.0;
}

// Tables of the disk into LDS (and the visit histogram, cleared).
template <int CDF_MODE>
__device__ __forceinline__ Lds64 setup_lds64(const TraceArgs& A) {
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
  return L;
}

template <int CDF_MODE>  // 2: FP64 CDF in LDS; 1: FP32 guide copy in LDS; 0: global only
__global__ void __launch_bounds__(BS64) trace_fp64_kernel(TraceArgs A) {
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda;
  const Lds64 L = setup_lds64<CDF_MODE>(A);

  const int lane = __lane_id();
  const double* fixT = A.frozen_T ? A.frozen_T : A.T_coef;
  bool alive = false, exhausted = false;
  Rng64 rng;
  Pk64 P;
  P.i = -1;
  P.events = 0;
  uint64_t pid = 0;
  bool handed = false;  // this packet tried the hand-off already
  // hand-off bookkeeping: this wavefront's packets are counted in *A.live;
  // hand-offs are allowed (both wave-uniform); the lane's packet was live
  bool counted = false, allow = false, polled = false, was_alive = false;
  uint32_t tot[N_COUNTERS] = {};

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
          P.p[0] = M.R_star * st;
          P.p[1] = 0.0;
          P.p[2] = M.R_star * ws;
          double mup = sqrt(rng.next());
          double php = 2.0 * KPI * rng.next();
          double sp = sqrt(fmax(0.0, 1.0 - mup * mup));
          double sn, cs;
          sincos(php, &sn, &cs);
          P.d[0] = mup * st + sp * cs * ws;
          P.d[1] = sp * sn;
          P.d[2] = mup * ws - sp * cs * st;
          double xs = rng.next();
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (L.star_cdf[mid] > xs) hi = mid; else lo = mid + 1;
          }
          P.k = lo;
          P.tau = -log(rng.next());
          P.i = -1;
          P.j = 0;
          P.n_int = 0;
          P.events = 0;
          P.pc_cross = P.pc_scat = P.pc_abs = P.pc_mrw = 0;
          P.rho = P.im = P.Tfix = 0.0;
          P.alpha = 0.0;
          P.omega = L.omega[P.k];
          P.Tc = -1.0;
          P.mrw_T = -2.0;
          P.mrw_Drho = P.mrw_f = P.mrw_lim = 0.0;
          P.mrw_seg = P.seg_seen = 0;
          P.d_safe = 0.0;
          P.dm_up = INFINITY;
          P.cell_abs = P.cell_mrw = 0;
          P.E_seen = -1.0;
          P.T_seen = 0.0;
          tot[C_LAUNCH]++;
          handed = false;
          alive = true;
        }
      }
    }
    if (A.live && exhausted) {
      // count this wavefront's live packets once, then the ones that leave
      const unsigned long long now = __ballot(alive);
      if (!counted) {
        if (lane == 0) {
          atomicAdd((unsigned long long*)A.live, (unsigned long long)__popcll(now));
          atomicAdd(A.waves_in, 1u);
        }
        counted = true;
      } else {
        const unsigned long long gone = __ballot(was_alive && !alive);
        if (gone && lane == 0)
          atomicAdd((unsigned long long*)A.live,
                    (unsigned long long)(-(long long)__popcll(gone)));
      }
      was_alive = alive;
    }
    const unsigned long long live = __ballot(alive);
    if (live == 0ull) {
      if (exhausted) break;
      continue;
    }
    if (!alive) continue;
    if (A.tail) {
      // a wavefront whose lanes never fall idle learns that the launch's
      // packets are all handed out from the counter itself, now and then
      if (!exhausted && __ballot((P.events & 1023) == 1023)) {
        const int leader = __ffsll((long long)__ballot(true)) - 1;
        unsigned long long nx = 0;
        if (lane == leader)
          nx = __hip_atomic_load(A.next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        nx = __shfl(nx, leader);
        if (nx >= A.n_packets) exhausted = true;
      }
      // hand-offs wait until every wavefront is counted and no more packets
      // are live than the hand-off launch has wavefronts: until then the
      // long packets run 64 to a wavefront here
      if (exhausted && !allow && (!polled || __ballot((P.events & 255) == 255))) {
        polled = true;
        const int leader = __ffsll((long long)__ballot(true)) - 1;
        long long lv = 0;
        unsigned wi = 0;
        if (lane == leader) {
          lv = __hip_atomic_load(A.live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          wi = __hip_atomic_load(A.waves_in, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        lv = __shfl(lv, leader);
        wi = __shfl(wi, leader);
        if (wi >= A.n_waves && lv <= (long long)A.live_handoff) allow = true;
      }
      // then a long packet moves to the whole-wavefront launch
      if (allow && !handed && P.events >= A.wave_events) {
        handed = true;
        const unsigned slot = atomicAdd(A.tail_count, 1u);
        if (slot < (unsigned)A.tail_cap) {
          TailState64& ts = ((TailState64*)A.tail)[slot];
          ts.P = P;
          ts.rng = rng;
          ts.pid = pid;
          tot[C_HANDED]++;
          alive = false;
          continue;
        }
      }
    }

    const int fate = event64<false>(P, rng, A, L, fixT, lane);
    if (fate != 0) {
      finish64<false>(P, rng, fate, pid, A, tot, lane);
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

// The packets handed over by trace_fp64_kernel, one wavefront each.
template <int CDF_MODE>
__global__ void __launch_bounds__(BS64) trace_fp64_tail_kernel(TraceArgs A) {
  const unsigned wpb = BS64 / 64;
  if (!A.tail) return;  // traced without hand-off (not launched then; kept safe)
  const unsigned count = min(*A.tail_count, (unsigned)A.tail_cap);
  if (blockIdx.x * wpb >= count) return;  // the whole workgroup
  const Lds64 L = setup_lds64<CDF_MODE>(A);
  const int n_r = A.m.n_r, n_mu = A.m.n_mu;
  const int lane = __lane_id();
  const double* fixT = A.frozen_T ? A.frozen_T : A.T_coef;
  uint32_t tot[N_COUNTERS] = {};
  for (;;) {
    // a wavefront takes the next state when it is done with one, so the
    // longest walks do not queue behind others
    unsigned slot = 0;
    if (lane == 0) slot = atomicAdd(A.tail_next, 1u);
    slot = (unsigned)__builtin_amdgcn_readfirstlane((int)slot);
    if (slot >= count) break;
    const TailState64& ts = ((const TailState64*)A.tail)[slot];
    Pk64 S = ts.P;
    WaveRng64 wr;
    wr.init(ts.rng);
    const uint64_t pid = ts.pid;
    int f;
    do {
      f = event64<true>(S, wr, A, L, fixT, lane);
    } while (f == 0);
    finish64<true>(S, wr, f, pid, A, tot, lane);
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
  auto tail = trace_fp64_tail_kernel<MODE>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
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
  // packets are handed off once no more are left than the hand-off launch
  // has wavefronts
  long long tb = (long long)ctx->n_cu * per_cu;
  const long long slots = ((long long)a.tail_cap + BS64 / 64 - 1) / (BS64 / 64);
  if (tb > slots) tb = slots;
  TraceArgs b = a;
  // (or the count asked for: more than it has wavefronts queue for them)
  b.live_handoff = a.live_handoff > 0 ? min((unsigned)a.live_handoff, (unsigned)a.tail_cap)
                                      : (unsigned)(tb * (BS64 / 64));
  // a launch with no more packets than that needs no count
  b.n_waves = a.n_packets <= b.live_handoff ? 0u : (unsigned)(nb * (BS64 / 64));
  hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(BS64), lds, s, b);
  if (a.tail) hipLaunchKernelGGL(tail, dim3((unsigned)tb), dim3(BS64), lds, s, b);
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
