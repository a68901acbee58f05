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
  float *re32, *mu2f;  // FP32 radial edges and squared cone cosines
  TabView tv;
  const float* cdf;
  uint32_t* vis;  // per-workgroup visit histogram [n_cells], or null
};

// Bytes of the tables; a visit histogram, when used, follows at this offset.
__host__ __device__ inline size_t lds32_bytes(int n_r, int n_mu, int n_T, int nl, bool with_cdf) {
  size_t dbl = (size_t)(n_r + 1) + (n_mu + 1) + MRW_TAB_N + 6 * (size_t)n_T;
  size_t flt = (size_t)3 * (n_mu + 1) + (size_t)(n_r + 1) + (size_t)3 * nl +
               (with_cdf ? (size_t)n_T * nl : 0);
  return dbl * 8 + N_GUIDE * 4 + ((flt * 4 + 7) & ~(size_t)7);
}

// Hardware reciprocal and square root (about 1 ulp, no range scaling: the
// operands here are normal numbers well inside the FP32 range).
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// Face distances (as exit_sphere, enter_sphere, exit_cone) with those.
// Both sides of every case are evaluated and the result selected, which
// gives the same values as branching: uniform branches cost a compare, a
// mask operation and a jump each, a select one instruction.  The discarded
// side may divide by zero; its value is never used.
__device__ __forceinline__ float exit_sphere32(float pd, float c) {
  const float disc = pd * pd - c;
  const float sq = fsqrt(fmaxf(disc, 0.0f));
  const float v = pd > 0.0f ? -fdiv(c, pd + sq) : -pd + sq;
  return (c >= 0.0f && (pd > 0.0f || disc < 0.0f)) ? 0.0f : v;
}
__device__ __forceinline__ float enter_sphere32(float pd, float c) {
  const float disc = pd * pd - c;
  float v = fdiv(c, -pd + fsqrt(fmaxf(disc, 0.0f)));
  v = (pd >= 0.0f || disc < 0.0f) ? -1.0f : v;
  return (c <= 0.0f && pd < 0.0f) ? 0.0f : v;
}
__device__ __forceinline__ float exit_cone32(float A, float B, float C, bool toward_pole) {
  const bool at_face = toward_pole ? (C >= 0.0f && B > 0.0f) : (C <= 0.0f && B < 0.0f);
  const float disc = B * B - A * C;
  const float sq = fsqrt(fmaxf(disc, 0.0f));
  // the root of the quadratic in the stable form for the sign of B
  const bool first = toward_pole ? B > 0.0f : B < 0.0f;
  const float num = first ? C : (toward_pole ? -B + sq : -B - sq);
  const float den = first ? (toward_pole ? -B - sq : -B + sq) : A;
  const float v = fdiv(num, den);
  const bool none = disc < 0.0f || !(v > 0.0f) || __builtin_isinf(v);
  return at_face ? 0.0f : none ? -1.0f : v;
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
  float best = exit_sphere32(pd, a.K_out + 2.0f * Aq + qq);
  face = 1;
  float s = enter_sphere32(pd, a.K_in + 2.0f * Aq + qq);
  if (s >= 0.0f && s < best) { best = s; face = 0; }
  float z = a.Af[2] + q[2];
  float dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  float zq = a.Af[2] * q[2];
  float qz2 = q[2] * q[2];
  // the cone below (none in the midplane row) and above (none in the polar row)
  {
    float m2 = L.mu2f[j];
    float C = a.L_lo + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    s = exit_cone32(d[2] * d[2] - m2 * dd, z * d[2] - m2 * pd, C, false);
    if (j >= 1 && s >= 0.0f && s < best) { best = s; face = 2; }
  }
  {
    float m2 = L.mu2f[j + 1];
    float C = a.L_hi + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    s = exit_cone32(d[2] * d[2] - m2 * dd, z * d[2] - m2 * pd, C, true);
    if (j + 1 < n_mu && s >= 0.0f && s < best) { best = s; face = 3; }
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
  float R = fsqrt(x * x + y * y);
  float r = fsqrt(R * R + z * z);
  float ri = L.re32[i], ro = L.re32[i + 1];
  float dmin = fminf(fdiv(a.K_in + 2.0f * Aq + qq, r + ri), -fdiv(a.K_out + 2.0f * Aq + qq, r + ro));
  float az = fabsf(z);
  float zq = a.Af[2] * q[2], qz2 = q[2] * q[2];
  {
    float m2 = L.mu2f[j];
    float f = a.L_lo + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    const float dl = fdiv(f, L.smu32[j] * az + L.mu32[j] * R);
    dmin = j >= 1 ? fminf(dmin, dl) : dmin;
  }
  {
    float m2 = L.mu2f[j + 1];
    float f = a.L_hi + 2.0f * (zq - m2 * Aq) + (qz2 - m2 * qq);
    const float dh = -fdiv(f, L.smu32[j + 1] * az + L.mu32[j + 1] * R);
    dmin = j + 1 < n_mu ? fminf(dmin, dh) : dmin;
  }
  return dmin > 0.0f ? dmin : 0.0f;
}

// Functions of one draw u used by the transport; the whole-wave generator
// evaluates them once per word, lane-parallel, so every caller gets the same
// values from either generator.
__device__ __forceinline__ float iso_mu(float u) { return 2.0f * u - 1.0f; }
__device__ __forceinline__ float iso_st(float u) {
  const float w = iso_mu(u);
  return fsqrt(fmaxf(0.0f, 1.0f - w * w));
}
__device__ __forceinline__ void iso_phi(float u, float& sn, float& cs) {
  __sincosf(2.0f * (float)KPI * u, &sn, &cs);
}
__device__ __forceinline__ float tau_of(float u) { return -__logf(u); }

// MRW escape time in FP32 (eq. probability RW): s with P(s) = P0.  The
// residual P(s) - P0 is formed from the series in P for s >= 0.1 and from
// the theta form of Q = 1 - P below, against Q0 = 1 - P0 (exact for P0 >=
// 1/2), so both long and short escapes keep their relative precision.
// Start from the table in v = ln(-ln P0), then three Newton steps.
__device__ __forceinline__ void mrw_resid32(float s, float P0, float Q0, float& r, float& dr) {
  const float pi2 = (float)(KPI * KPI);
  if (s >= 0.1f) {
    const float x = pi2 * s;
    float sum = 0.0f, dsum = 0.0f;
#pragma unroll
    for (int n = 1; n <= 7; ++n) {
      const float n2 = (float)(n * n);
      const float e = __expf(-n2 * x);
      const float sg = (n & 1) ? 1.0f : -1.0f;
      sum += sg * e;
      dsum += sg * n2 * pi2 * e;
    }
    r = 2.0f * sum - P0;
    dr = -2.0f * dsum;
  } else {
    const float inv_s = 1.0f / s;
    float sum = 0.0f, dsum = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float a = (float)((2 * k + 1) * (2 * k + 1)) * 0.25f;
      const float e = __expf(-a * inv_s);
      sum += e;
      dsum += e * a * inv_s * inv_s;
    }
    const float pre = 2.0f * rsqrtf((float)KPI * s);
    r = Q0 - pre * sum;
    dr = -(pre * dsum - 0.5f * pre * inv_s * sum);
  }
}

__device__ __forceinline__ float mrw_escape_s32(const double* tab, float P0) {
  const float Q0 = 1.0f - P0;
  const float mlnP = Q0 < 0.01f ? Q0 * (1.0f + 0.5f * Q0) : -__logf(P0);
  const float v = __logf(mlnP);
  float t = (v - (float)MRW_TAB_V0) * (float)((MRW_TAB_N - 1) / (MRW_TAB_V1 - MRW_TAB_V0));
  t = fminf(fmaxf(t, 0.0f), (float)(MRW_TAB_N - 1) - 1e-3f);
  const int q = (int)t;
  const float f = t - (float)q;
  const float s0 = (float)tab[q], s1 = (float)tab[q + 1];
  float s = s0 + f * (s1 - s0);
#pragma unroll
  for (int it = 0; it < 3; ++it) {
    float r, dr;
    mrw_resid32(s, P0, Q0, r, dr);
    const float sn = s - r / dr;
    s = sn > 0.5f * s ? sn : 0.5f * s;
  }
  return s;
}

// isotropic direction from two draws; optical depth from one
__device__ __forceinline__ void iso32(Rng32& r, float d[3]) {
  const float u1 = r.next();
  const float u2 = r.next();
  float sn, cs;
  iso_phi(u2, sn, cs);
  const float st = iso_st(u1);
  d[0] = st * cs;
  d[1] = st * sn;
  d[2] = iso_mu(u1);
}
__device__ __forceinline__ float tau32(Rng32& r) { return tau_of(r.next()); }
__device__ __forceinline__ void ensure_draws(Rng32&, int) {}
// a scattering leaves the interaction's reemission word unused, so that
// every interaction takes five words (albedo, bin, two of direction, optical
// depth) and interaction j of a run in a cell starts 5 j words on
__device__ __forceinline__ void skip_draw(Rng32& r) { (void)r.next(); }
// the two draws of a scattering: the first raw (the scattering angle), the
// second as the sine and cosine of its azimuth
__device__ __forceinline__ void scat_draws(Rng32& r, float& u1, float& sn, float& cs) {
  u1 = r.next();
  iso_phi(r.next(), sn, cs);
}

// Direction after a scattering by the Henyey-Greenstein phase function with
// asymmetry g != 0: the cosine of the scattering angle from the inverse of
// its cumulative distribution at u1, the azimuth (sine sn, cosine cs) about
// the old direction; the result is renormalised, since the rotation
// compounds over a walk in FP32.
__device__ __forceinline__ void hg_turn32(float g, float u1, float sn, float cs, float d[3]) {
  const float q = fdiv(1.0f - g * g, 1.0f - g + 2.0f * g * u1);
  const float mu = fminf(1.0f, fmaxf(-1.0f, fdiv(1.0f + g * g - q * q, 2.0f * g)));
  const float st = fsqrt(fmaxf(0.0f, 1.0f - mu * mu));
  const float x = d[0], y = d[1], z = d[2];
  const float s2 = x * x + y * y;
  float nx, ny, nz;
  if (s2 > 0.0f) {
    const float is = __builtin_amdgcn_rsqf(s2);
    const float s = s2 * is;
    nx = st * (x * z * cs - y * sn) * is + x * mu;
    ny = st * (y * z * cs + x * sn) * is + y * mu;
    nz = -st * cs * s + z * mu;
  } else {
    nx = st * cs;
    ny = st * sn;
    nz = z > 0.0f ? mu : -mu;
  }
  const float nn = __builtin_amdgcn_rsqf(nx * nx + ny * ny + nz * nz);
  d[0] = nx * nn;
  d[1] = ny * nn;
  d[2] = nz * nn;
}

// ------------------------------------------------------------------ packets
// Transport state of one packet.
struct Pk {
  Anchor an;
  float q[3], d[3], tau;
  int k, i, j, n_int;
  long long events;
  uint32_t pc_cross, pc_scat, pc_abs, pc_mrw;
  double rho;                        // density of the cell
  double im;                         // 1 / (4 pi m) of the cell
  double Tc;                         // running temperature of the cell (< 0: from its tally)
  double Tfix;                       // the cell's fixed temperature (frozen or MRW field)
  double mrw_T, mrw_Drho, mrw_f;  // MRW coefficients at mrw_T: D rho, and the
  int mrw_seg;                     // table segment and fraction of mrw_T
  float mrw_lim;
  float d_safe;   // lower bound of the distance to every face of the cell
  float dm_up;    // upper bound of it: the last computed one plus the path flown since
                  // (while it is within the MRW limit the criterion cannot hold)
  // absorptions and MRW steps in this stay in the cell, added to the tallies
  // when the packet leaves it; the cell's tally after this packet's last
  // deposit (or as last read) and its temperature (reused when nobody
  // deposited in between)
  uint32_t cell_abs, cell_mrw;
  double E_seen, T_seen;
  int seg_seen;   // table segment of T_seen
  float alpha, omega;  // extinction rho chi_k of the cell at bin k, and the albedo at k
  float lim_scale;  // 3 gamma / rho of the cell: the MRW limit is D rho times this
};

// A packet handed over to the whole-wavefront launch.
struct TailState32 {
  Pk P;
  Rng32 rng;
  uint64_t pid;
};
static_assert(sizeof(TailState32) <= TAIL_STATE_BYTES, "hand-off slot");

// ------------------------------------------------------ whole-wave mode
// Once every packet of a launch has been handed out, packets that are still
// going after wave_events events are saved and continued by a second launch
// in which a whole wavefront runs each of them: the control flow is uniform,
// the lanes generate 64 draws in one pass of the generator, and the
// reemission bin is found by a 64-wide ballot.  A lone
// lane issues about one instruction per ten cycles, so these cuts in
// instruction count are what shortens the longest random walks, which set
// the length of a launch.
__device__ __forceinline__ double wave_bcast0(double v) {
  const long long x = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, 0);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)x >> 32), 0);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The stream of one packet (the same draws as Rng32) served to a wavefront:
// the buffer is the 64 words of Philox blocks blk0 .. blk0 + 15, word p held
// by lane p (lanes 4b .. 4b + 3 generate block blk0 + b and keep one word
// each), with the functions of it that the transport takes (optical depth,
// direction cosine and sine terms).  A draw is then one read from a fixed
// register of a lane given by a uniform index, with no choice among
// registers, and the generator and transcendentals run once per 64 draws
// off the chain.
struct WaveRng {
  uint64_t pid;
  uint32_t k0, k1;
  uint32_t blk0;  // block of buffer words 0..3
  int pos;        // next word of the buffer, 0..63 (the stream's draw 4 blk0 + pos)
  float u, tau, st, sn, cs;  // this lane's word

  __device__ __forceinline__ void fill() {
    const uint32_t lane = (uint32_t)__lane_id();
    uint32_t c[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), blk0 + (lane >> 2), 0u};
    philox4x32_10(c[0], c[1], c[2], c[3], k0, k1);
    const uint32_t a = lane & 3u;
    const uint32_t w = a == 0u ? c[0] : a == 1u ? c[1] : a == 2u ? c[2] : c[3];
    u = Rng32::unit(w);
    tau = tau_of(u);
    st = iso_st(u);
    iso_phi(u, sn, cs);
  }
  __device__ __forceinline__ void init(const Rng32& r) {
    pid = r.pid;
    k0 = r.k0;
    k1 = r.k1;
    const uint64_t nd = (uint64_t)r.draws();  // index of the next word of the stream
    blk0 = (uint32_t)(nd >> 2);
    pos = (int)(nd & 3);
    fill();
  }
  // value of word p of the buffer from this lane's x
  __device__ __forceinline__ float at(float x, int p) const {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), p));
  }
  // at least n draws left in the buffer: else restart it at the block of
  // the next draw (called where a segment of at most n draws begins, so the
  // generator is inlined in two places only)
  __device__ __forceinline__ void ensure(int n) {
    if (pos + n > 64) {
      blk0 += (uint32_t)(pos >> 2);
      pos &= 3;
      fill();
    }
  }
  __device__ __forceinline__ int take() { return pos++; }
  // skip n words (a run of interactions traced lane-parallel)
  __device__ __forceinline__ void advance(int n) {
    pos += n;
    if (pos + 8 > 64) {
      blk0 += (uint32_t)(pos >> 2);
      pos &= 3;
      fill();
    }
  }
  __device__ __forceinline__ float next() { return at(u, take()); }
  __device__ __forceinline__ float next_tau() { return at(tau, take()); }
  __device__ __forceinline__ void next_iso(float d[3]) {
    const int p1 = take();
    const float w = iso_mu(at(u, p1)), s = at(st, p1);
    const int p2 = take();
    const float cs_ = at(cs, p2), sn_ = at(sn, p2);
    d[0] = s * cs_;
    d[1] = s * sn_;
    d[2] = w;
  }
  __device__ __forceinline__ void next_scat(float& u1, float& sn_, float& cs_) {
    const int p1 = take();
    u1 = at(u, p1);
    const int p2 = take();
    cs_ = at(cs, p2);
    sn_ = at(sn, p2);
  }
  __device__ __forceinline__ uint64_t draws() const { return (uint64_t)blk0 * 4u + (uint64_t)pos; }
};

__device__ __forceinline__ void iso32(WaveRng& r, float d[3]) { r.next_iso(d); }
__device__ __forceinline__ float tau32(WaveRng& r) { return r.next_tau(); }
__device__ __forceinline__ void ensure_draws(WaveRng& r, int n) { r.ensure(n); }
__device__ __forceinline__ void skip_draw(WaveRng& r) { (void)r.take(); }
__device__ __forceinline__ void scat_draws(WaveRng& r, float& u1, float& sn, float& cs) {
  r.next_scat(u1, sn, cs);
}

// Smallest k with D(k) > xi D(nl-1) (nl - 1 if none), one bin per lane.
template <typename C>
__device__ __forceinline__ int reemit_search_wave(const Reemit<C>& R, int nl, C xi) {
  const C target = xi * R.D(nl - 1);
  const int lane = __lane_id();
  for (int base = 0; base < nl; base += 64) {
    const int kk = base + lane < nl ? base + lane : nl - 1;
    const unsigned long long m = __ballot(base + lane < nl && R.D(kk) > target);
    if (m) return base + __ffsll((long long)m) - 1;
  }
  return nl - 1;
}


// One event of packet P: a flight through the central hole, a face
// crossing, or an interaction (scattering, or absorption with immediate
// reemission, Sect. 2.1) followed by MRW steps while the criterion holds
// (Sect. 2.2.2).  Returns the fate (0 going on, 1 escaped, 2 star, 3 capped).
// WAVE: the whole wavefront works on P (all lanes hold the same state) and
// lane 0 issues the memory updates.
template <bool WAVE, bool HG, class RNG>
__device__ __forceinline__ int event32(Pk& P, RNG& rng, const TraceArgs& A, const Lds32& L,
                                       const double* fixT, int lane) {
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda;
  const bool issuer = !WAVE || lane == 0;
  auto visit = [&](int cn) {
    if (issuer) {
      if (L.vis) atomicAdd(&L.vis[cn], 1u); else atomicAdd(&A.t.visits[cn], 1u);
    }
  };
  auto deposit = [&](int c, double dE) -> double {  // returns the tally before
    double E_old = 0.0;
    if (WAVE) {
      if (issuer) E_old = unsafeAtomicAdd(&A.t.E_abs[c], dE);
    } else {
      E_old = tally_add_grouped(A.t.E_abs, c, dE);
    }
    // the odd-numbered packets' share, kept apart for the noise estimate
    if (issuer && A.t.E_half && (rng.pid & 1)) unsafeAtomicAdd(&A.t.E_half[c], dE);
    if (WAVE) E_old = wave_bcast0(E_old);
    return E_old;
  };
  auto search = [&](const Reemit<float>& R, float xb) -> int {
    if (WAVE) return reemit_search_wave<float>(R, nl, xb);
    return reemit_search<float>(R, nl, xb);
  };
  // Bin of the reemission after a deposit dE on top of the cell's tally
  // E_old (immediate reemission, Sect. 2.1): the difference spectrum between
  // the temperatures after and before, from the inversion of the tally; the
  // spectrum interpolation reuses the inversion's table segments.
  auto reemit_bin = [&](double E_old, double dE, float xb) -> int {
    if (A.frozen_T) return search(reemit_setup<float>(L.tv, L.cdf, -1.0, P.Tfix), xb);
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
    return search(reemit_setup<float>(L.tv, L.cdf, T_old, T_new, n_new, n_old), xb);
  };
  auto lim_scale_of = [&](double rho) -> float { return (float)(A.gamma * 3.0 / rho); };
  int fate = 0;
  if (++P.events > A.max_events) {
    fate = 3;
  } else if (P.i < 0) {
    // central hole, FP64: the star or the inner grid sphere
    double Q[3] = {P.an.A[0] + (double)P.q[0], P.an.A[1] + (double)P.q[1],
                   P.an.A[2] + (double)P.q[2]};
    double D[3] = {(double)P.d[0], (double)P.d[1], (double)P.d[2]};
    double pd = Q[0] * D[0] + Q[1] * D[1] + Q[2] * D[2];
    double rr = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
    double s = enter_sphere<double>(pd, rr - M.R_star * M.R_star);
    P.q[0] = P.q[1] = P.q[2] = 0.0f;
    if (s >= 0.0) {
      P.an.A[0] = Q[0] + s * D[0]; P.an.A[1] = Q[1] + s * D[1]; P.an.A[2] = Q[2] + s * D[2];
      fate = 2;
    } else {
      s = exit_sphere<double>(pd, rr - L.r2[0]);
      P.an.A[0] = Q[0] + s * D[0]; P.an.A[1] = Q[1] + s * D[1]; P.an.A[2] = Q[2] + s * D[2];
      P.i = 0;
      double r2 = (P.an.A[0] * P.an.A[0] + P.an.A[1] * P.an.A[1]) + P.an.A[2] * P.an.A[2];
      P.j = mu_row(L.mu2, n_mu, r2, P.an.A[2] * P.an.A[2]);
      set_anchor(P.an, L, n_mu, P.i, P.j);
      P.rho = M.rho[P.j];
      P.alpha = (float)P.rho * L.chi[P.k];
      P.omega = L.omega[P.k];
      P.lim_scale = lim_scale_of(P.rho);
      P.im = M.inv4pim[P.j];
      if (fixT) P.Tfix = fixT[P.j];
      visit(P.j);
      P.Tc = -1.0;
      P.mrw_T = -2.0;
      P.d_safe = 0.0f;
      P.dm_up = INFINITY;
      P.n_int = 0;
      ++P.pc_cross;
    }
  } else {
    const int c = P.i * n_mu + P.j;
    const float alpha = P.alpha;
    int face = 1;
    float sb = 0.0f, tau_b = 0.0f;
    // a flight shorter than the guaranteed distance to every face stays in
    // the cell: the face distances are not needed for it.  A wavefront on
    // one packet renews that distance when it runs out (not on the face the
    // packet just came through, where it is 0): the bound costs a third of
    // the four face distances and spares them on about half of the flights
    // of a walk in optically thick cells.  Per lane, neighbouring packets
    // would take both paths.
    bool inside = P.tau < alpha * P.d_safe;
    if (WAVE && !inside && P.n_int > 0) {
      const float dm = min_boundary32(P.an, L, n_mu, P.i, P.j, P.q);
      P.d_safe = 0.999f * dm;
      P.dm_up = fminf(P.dm_up, 1.00001f * dm);
      inside = P.tau < alpha * P.d_safe;
    }
    if (!inside) {
      sb = boundary32(P.an, L, n_mu, P.i, P.j, P.q, P.d, face);
      tau_b = alpha * sb;
    }
    if (!inside && tau_b <= P.tau) {
      P.d_safe = 0.0f;
      P.dm_up = INFINITY;
      // path-length tally of the mean intensity (when kept)
      if (issuer && A.t.path) unsafeAtomicAdd(&A.t.path[(size_t)c * nl + P.k], A.eps * (double)sb);
      if (issuer && P.cell_abs) atomicAdd(&A.t.n_abs[c], P.cell_abs);
      if (issuer && P.cell_mrw) atomicAdd(&A.t.n_mrw[c], P.cell_mrw);
      P.cell_abs = P.cell_mrw = 0;
      P.E_seen = -1.0;
      P.q[0] += sb * P.d[0]; P.q[1] += sb * P.d[1]; P.q[2] += sb * P.d[2];
      P.tau -= tau_b;
      if (P.tau < 0.0f) P.tau = 0.0f;
      ++P.pc_cross;
      bool entered = true;
      if (face == 1) {
        if (P.i + 1 == n_r) {
          int m = (int)(fabsf(P.d[2]) * M.n_inc);
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
        P.alpha = (float)P.rho * L.chi[P.k];
        P.lim_scale = lim_scale_of(P.rho);
        P.im = M.inv4pim[cn];
        if (fixT) P.Tfix = fixT[cn];
        reanchor(P.an, P.q, L, n_mu, P.i, P.j);
        visit(cn);
      } else if (fate == 0) {
        // into the hole: keep the FP64 position in the anchor
        P.an.A[0] += (double)P.q[0]; P.an.A[1] += (double)P.q[1]; P.an.A[2] += (double)P.q[2];
        P.q[0] = P.q[1] = P.q[2] = 0.0f;
      }
      P.Tc = -1.0;
      P.mrw_T = -2.0;
      P.n_int = 0;
    } else {
      // the flight ends before sb (or d_safe when inside).  Where alpha is so
      // small that its reciprocal overflows, tau * rcp(alpha) is 0 * inf for
      // a packet with no optical depth left (its flight is 0) and inf
      // otherwise (bounded by the face it cannot reach)
      const float sint = P.tau > 0.0f ? fminf(fdiv(P.tau, alpha), inside ? P.d_safe : sb) : 0.0f;
      if (issuer && A.t.path) unsafeAtomicAdd(&A.t.path[(size_t)c * nl + P.k], A.eps * (double)sint);
      P.q[0] += sint * P.d[0]; P.q[1] += sint * P.d[1]; P.q[2] += sint * P.d[2];
      P.d_safe -= sint;
      P.dm_up += 1.00001f * sint;
      const double* fz = A.frozen_T;
      ensure_draws(rng, 6);  // albedo, bin, direction, optical depth
      if (rng.next() < P.omega) {
        ++P.pc_scat;
        skip_draw(rng);
        if constexpr (HG) {
          float u1, sn, cs;
          scat_draws(rng, u1, sn, cs);
          hg_turn32((float)A.g_asym, u1, sn, cs, P.d);
        } else {
          iso32(rng, P.d);
        }
      } else {
        ++P.pc_abs;
        ++P.cell_abs;
        // the tally update is in flight while the next draws are made
        double E_old = deposit(c, A.eps);
        float xb = rng.next();
        iso32(rng, P.d);
        P.k = reemit_bin(E_old, A.eps, xb);
        P.alpha = (float)P.rho * L.chi[P.k];
        P.omega = L.omega[P.k];
      }
      ++P.n_int;
      if (A.mrw) {
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
            // (the segment of the cell's running T is known from its inversion)
            const int n = T_here == P.T_seen ? P.seg_seen : t_segment(L.tv, T_here);
            const double f = (T_here - L.tv.Tn[n]) * L.tv.inv_dT[n];
            P.mrw_T = T_here;
            P.mrw_seg = n;
            P.mrw_f = f;
            P.mrw_Drho = L.tv.Drho[n] + f * (L.tv.Drho[n + 1] - L.tv.Drho[n]);
            P.mrw_lim = (float)P.mrw_Drho * P.lim_scale;
          }
          const double Drho = P.mrw_Drho;
          const float lim = P.mrw_lim;
          if (P.dm_up <= lim) break;
          {
            float dm = min_boundary32(P.an, L, n_mu, P.i, P.j, P.q);
            P.d_safe = 0.999f * dm;
            P.dm_up = 1.00001f * dm;
            if (!(dm > lim)) break;
          }
          // re-anchor so the sphere radius is exact to FP32 precision of itself
          reanchor(P.an, P.q, L, n_mu, P.i, P.j);
          float dmin = min_boundary32(P.an, L, n_mu, P.i, P.j, P.q);
          if (!(dmin > lim)) break;
          if (++P.events > A.max_events) break;
          ensure_draws(rng, 7);  // escape time, jump, bin, direction, optical depth
          double R0 = (double)dmin * (1.0 - 1e-5);
          double s = (double)mrw_escape_s32(L.mrw_tab, rng.next());
          double ell = s * R0 * R0 * P.rho / Drho;
          const int ns = P.mrw_seg;
          const double kbar = L.tv.kbar[ns] + P.mrw_f * (L.tv.kbar[ns + 1] - L.tv.kbar[ns]);
          double dE = A.eps * P.rho * kbar * ell;
          if (issuer && A.t.path) unsafeAtomicAdd(&A.t.mrw_path[c], A.eps * ell);
          double E_old = deposit(c, dE);
          float nv[3];
          iso32(rng, nv);
          P.q[0] = (float)R0 * nv[0]; P.q[1] = (float)R0 * nv[1]; P.q[2] = (float)R0 * nv[2];
          float xb = rng.next();
          iso32(rng, P.d);
          P.k = reemit_bin(E_old, dE, xb);
          P.alpha = (float)P.rho * L.chi[P.k];
          P.omega = L.omega[P.k];
          P.d_safe = 0.0f;
          P.dm_up = INFINITY;
          ++P.pc_mrw;
          ++P.cell_mrw;
        }
      }
      P.tau = tau32(rng);
    }
  }
  return fate;
}

// ------------------------------------------------------------ run-ahead
// A run of interactions inside one cell, traced lane-parallel by the
// wavefront that follows a packet (whole-wavefront mode, isotropic
// scattering).  Interaction j of the run takes the five stream words
// w0 + 5 j .. w0 + 5 j + 4 (albedo, reemission bin, direction cosine,
// azimuth, next optical depth), so lane j draws its own without knowing the
// kinds of the interactions before it.  Then:
//  * kinds and bins, in order.  From the bin of a flight, the next
//    absorption is the first later interaction whose albedo draw is not
//    below the albedo at that bin (one ballot); its bin is the reemission
//    search for the k-th deposit of the run (Sect. 2.1), between the
//    temperatures of the tallies E + k eps and E + (k + 1) eps, which the
//    lanes invert at once;
//  * positions, flight by flight in the order and with the FP32 operations
//    of one event at a time, a chunk of flights at a time;
//  * per lane, what ends a run: the flight reaches a face (tau >= alpha s_b),
//    or the MRW criterion holds after the interaction (Sect. 2.2.2, eq.
//    criterion, after n_int_min interactions in the cell); the first such
//    interaction, and everything after it, is left to event32;
//  * the deposits before it, committed by one compare-and-swap of the cell's
//    tally from the E the run started from to E + k eps (added one deposit at
//    a time, as the atomics would).  If another packet deposited in between,
//    the run is redone from the tally found.
// These are the tests event32 makes, without the conservative shortcuts it
// takes on them (the safe distance d_safe and the bound dm_up), so a packet
// follows the same events either way.  Per event, the returned atomic, the
// face distances and most of the draw handling leave the serial chain.
constexpr int RUN_KMAX = 12;  // deposits of one run
constexpr int RUN_CHUNK = 8;  // flights per chunk of the position chain

struct RunDraws {
  float a, xb, tn;   // albedo, bin, optical depth of the next flight
  float dx, dy, dz;  // direction after the interaction
};

__device__ __forceinline__ uint32_t pick4(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                          int i) {
  return i == 0 ? x0 : i == 1 ? x1 : i == 2 ? x2 : x3;
}

// The five words from stream word w (two consecutive Philox blocks), through
// the same functions of a draw as Rng32 and WaveRng.
__device__ __forceinline__ RunDraws run_draws(uint64_t pid, uint32_t k0, uint32_t k1, uint64_t w) {
  const uint32_t b = (uint32_t)(w >> 2);
  const int o = (int)(w & 3u);
  uint32_t c0 = (uint32_t)pid, c1 = (uint32_t)(pid >> 32), c2 = b, c3 = 0u;
  philox4x32_10(c0, c1, c2, c3, k0, k1);
  uint32_t e0 = (uint32_t)pid, e1 = (uint32_t)(pid >> 32), e2 = b + 1u, e3 = 0u;
  philox4x32_10(e0, e1, e2, e3, k0, k1);
  uint32_t wd[5];
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    const int i = o + t;
    wd[t] = i < 4 ? pick4(c0, c1, c2, c3, i) : pick4(e0, e1, e2, e3, i - 4);
  }
  RunDraws R;
  R.a = Rng32::unit(wd[0]);
  R.xb = Rng32::unit(wd[1]);
  const float u1 = Rng32::unit(wd[2]);
  float sn, cs;
  iso_phi(Rng32::unit(wd[3]), sn, cs);
  const float st = iso_st(u1);
  R.dx = st * cs;
  R.dy = st * sn;
  R.dz = iso_mu(u1);
  R.tn = tau_of(Rng32::unit(wd[4]));
  return R;
}

__device__ __forceinline__ float readlane_f32(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// Interactions committed (0: the next event is left to event32).  Needs
// P.i >= 0 and isotropic scattering; all lanes hold the same P.
__device__ __forceinline__ int run_ahead32(Pk& P, WaveRng& wr, const TraceArgs& A, const Lds32& L,
                                        const double* fixT, int lane) {
  const DevModel& M = A.m;
  const int n_mu = M.n_mu, nl = M.n_lambda;
  const int c = P.i * n_mu + P.j;
  const long long room = A.max_events - P.events;
  if (room <= 0) return 0;
  const int J = room < 64 ? (int)room : 64;
  const bool frozen = A.frozen_T != nullptr;
  const RunDraws R = run_draws(wr.pid, wr.k0, wr.k1, wr.draws() + 5ull * (uint64_t)lane);
  // flight `lane`: its optical depth and direction (flight 0 is the pending one)
  float tau_f = __shfl_up(R.tn, 1), fx = __shfl_up(R.dx, 1), fy = __shfl_up(R.dy, 1),
        fz = __shfl_up(R.dz, 1);
  if (lane == 0) {
    tau_f = P.tau;
    fx = P.d[0];
    fy = P.d[1];
    fz = P.d[2];
  }
  Reemit<float> Rf{};
  if (frozen) Rf = reemit_setup<float>(L.tv, L.cdf, -1.0, P.Tfix);
  // the cell's tally as this packet last saw it, else as it is now
  double Eg = P.E_seen;
  bool loaded = false;
  if (!frozen && !(Eg >= 0.0)) {
    double e = 0.0;
    if (lane == 0)
      e = __hip_atomic_load(&A.t.E_abs[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    Eg = wave_bcast0(e);
    loaded = true;
  }
  for (int attempt = 0; attempt < 3; ++attempt) {
    // lane k: the tally after k deposits of the run and its temperature
    double Ek = 0.0, Tk = 0.0;
    int nk = 0;
    if (!frozen) {
      double e = Eg;
      for (int k = 0; k <= RUN_KMAX; ++k) {
        if (lane == k) Ek = e;
        e = e + A.eps;
      }
      Tk = T_of_g_seg_near(L.tv, Ek * P.im, P.seg_seen, nk);
    }
    // kinds and bins
    int lam = P.k, pos = 0, k = 0, Jc = J, lam_after = 0;
    unsigned long long absm = 0ull;
    for (;;) {
      const float om = L.omega[lam];
      const unsigned long long m = __ballot(lane >= pos && lane < Jc && !(R.a < om));
      if (m == 0ull) break;
      const int j = __ffsll((long long)m) - 1;
      if (k == RUN_KMAX) {
        Jc = j;
        break;
      }
      const float xb = readlane_f32(R.xb, j);
      int b;
      if (frozen) {
        b = reemit_search_wave<float>(Rf, nl, xb);
      } else {
        const double To = readlane_f64(Tk, k), Tn = readlane_f64(Tk, k + 1);
        const int no = __builtin_amdgcn_readlane(nk, k), nn = __builtin_amdgcn_readlane(nk, k + 1);
        b = reemit_search_wave<float>(reemit_setup<float>(L.tv, L.cdf, To, Tn, nn, no), nl, xb);
      }
      if (lane == k) lam_after = b;
      absm |= 1ull << j;
      ++k;
      lam = b;
      pos = j + 1;
    }
    // flight `lane`: bin, extinction, length, and the MRW limit after its interaction
    const int kj = __popcll(absm & ((1ull << lane) - 1ull));
    const int lam_src = __shfl(lam_after, kj > 0 ? kj - 1 : 0);
    const int lam_j = kj > 0 ? lam_src : P.k;
    const float alpha_j = (float)P.rho * L.chi[lam_j];
    const float sint_j = tau_f > 0.0f ? fdiv(tau_f, alpha_j) : 0.0f;
    float lim_j = 0.0f;
    if (A.mrw) {
      const int kk = kj + (int)((absm >> lane) & 1ull);
      const double T_kk = __shfl(Tk, kk);
      const int n_kk = __shfl(nk, kk);
      double T_here;
      int n_here;
      if (fixT) {
        // the segment as event32 finds it: the one of the tally's inversion
        // when the fixed T happens to equal the T last seen
        T_here = P.Tfix;
        const double Ts = (!frozen && kk > 0) ? T_kk : P.T_seen;
        const int ns = (!frozen && kk > 0) ? n_kk : P.seg_seen;
        n_here = T_here == Ts ? ns : t_segment(L.tv, T_here);
      } else {
        T_here = T_kk;
        n_here = n_kk;
      }
      const double f = (T_here - L.tv.Tn[n_here]) * L.tv.inv_dT[n_here];
      const double Drho = L.tv.Drho[n_here] + f * (L.tv.Drho[n_here + 1] - L.tv.Drho[n_here]);
      lim_j = (float)Drho * P.lim_scale;
    }
    // positions in chunks, then the tests of the chunk's flights
    float q0 = P.q[0], q1 = P.q[1], q2 = P.q[2];
    float qa[3] = {0.0f, 0.0f, 0.0f}, qb[3] = {0.0f, 0.0f, 0.0f};
    int n = Jc;
    for (int j0 = 0; j0 < Jc; j0 += RUN_CHUNK) {
      const int j1 = j0 + RUN_CHUNK < Jc ? j0 + RUN_CHUNK : Jc;
      for (int j = j0; j < j1; ++j) {
        const float s = readlane_f32(sint_j, j);
        const float ex = readlane_f32(fx, j), ey = readlane_f32(fy, j), ez = readlane_f32(fz, j);
        if (lane == j) {
          qa[0] = q0;
          qa[1] = q1;
          qa[2] = q2;
        }
        q0 += s * ex;
        q1 += s * ey;
        q2 += s * ez;
        if (lane == j) {
          qb[0] = q0;
          qb[1] = q1;
          qb[2] = q2;
        }
      }
      const bool mine = lane >= j0 && lane < j1;
      const float dd[3] = {fx, fy, fz};
      int face;
      const float sb = boundary32(P.an, L, n_mu, P.i, P.j, qa, dd, face);
      const bool cross = alpha_j * sb <= tau_f;
      const bool clip = !cross && sint_j > sb;
      bool mrw = false;
      if (A.mrw && P.n_int + lane + 1 >= A.n_int_min)
        mrw = min_boundary32(P.an, L, n_mu, P.i, P.j, qb) > lim_j;
      const unsigned long long bm = __ballot(mine && (cross || clip || mrw));
      if (bm) {
        n = __ffsll((long long)bm) - 1;
        break;
      }
    }
    if (n == 0) return 0;
    const unsigned long long cm = n >= 64 ? ~0ull : ((1ull << n) - 1ull);
    const int kst = __popcll(absm & cm);
    if (kst > 0) {
      if (frozen) {
        if (lane == 0)
          for (int t = 0; t < kst; ++t) unsafeAtomicAdd(&A.t.E_abs[c], A.eps);
      } else {
        const double En = readlane_f64(Ek, kst);
        unsigned long long old = 0ull;
        const unsigned long long want = (unsigned long long)__double_as_longlong(Eg);
        if (lane == 0)
          old = atomicCAS((unsigned long long*)&A.t.E_abs[c], want,
                          (unsigned long long)__double_as_longlong(En));
        old = (unsigned long long)__double_as_longlong(
            wave_bcast0(__longlong_as_double((long long)old)));
        if (old != want) {  // another packet deposited: redo from its tally
          Eg = __longlong_as_double((long long)old);
          loaded = true;
          continue;
        }
      }
      // the odd-numbered packets' share, one deposit at a time
      if (lane == 0 && A.t.E_half && (wr.pid & 1))
        for (int t = 0; t < kst; ++t) unsafeAtomicAdd(&A.t.E_half[c], A.eps);
    }
    // the state after interaction n - 1
    const int last = n - 1;
    P.q[0] = readlane_f32(qb[0], last);
    P.q[1] = readlane_f32(qb[1], last);
    P.q[2] = readlane_f32(qb[2], last);
    P.d[0] = readlane_f32(R.dx, last);
    P.d[1] = readlane_f32(R.dy, last);
    P.d[2] = readlane_f32(R.dz, last);
    P.tau = readlane_f32(R.tn, last);
    if (kst > 0) P.k = __builtin_amdgcn_readlane(lam_after, kst - 1);
    P.alpha = (float)P.rho * L.chi[P.k];
    P.omega = L.omega[P.k];
    P.n_int += n;
    P.events += n;
    P.pc_scat += (uint32_t)(n - kst);
    P.pc_abs += (uint32_t)kst;
    P.cell_abs += (uint32_t)kst;
    if (!frozen && (kst > 0 || loaded)) {
      P.E_seen = readlane_f64(Ek, kst);
      P.T_seen = readlane_f64(Tk, kst);
      P.seg_seen = __builtin_amdgcn_readlane(nk, kst);
      P.Tc = P.T_seen;
    }
    P.d_safe = 0.0f;
    P.dm_up = INFINITY;
    wr.advance(5 * n);
    return n;
  }
  return 0;  // the tally kept changing under the run: one event at a time
}

// End of a packet: remaining per-cell counts, counters, the star's tally and
// the optional record.
template <bool WAVE, class RNG>
__device__ __forceinline__ void finish32(Pk& P, const RNG& rng, int fate, uint64_t pid,
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
        mcrt_packet_rec& Rr = A.recs[r];
        Rr.fate = fate;
        Rr.k = P.k;
        Rr.n_cross = P.pc_cross;
        Rr.n_scat = P.pc_scat;
        Rr.n_abs = P.pc_abs;
        Rr.n_mrw = P.pc_mrw;
        Rr.n_draws = (int64_t)rng.draws();
        Rr.x = P.an.A[0] + P.q[0]; Rr.y = P.an.A[1] + P.q[1]; Rr.z = P.an.A[2] + P.q[2];
        Rr.u = P.d[0]; Rr.v = P.d[1]; Rr.w = P.d[2];
      }
    }
  }
  P.cell_abs = P.cell_mrw = 0;
  P.E_seen = -1.0;
}

// Tables of the workgroup's disk into LDS (and the visit histogram, cleared).
template <bool CDF_LDS>
__device__ __forceinline__ Lds32 setup_lds32(const TraceArgs& A) {
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
    takef(L.re32, n_r + 1, [&](int a) { return (float)M.r_edges[a]; });
    takef(L.mu2f, n_mu + 1, [&](int a) { return (float)M.mu2[a]; });
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
  return L;
}

template <bool CDF_LDS, bool HG>
__device__ __forceinline__ void trace_fp32_body(const TraceArgs& A) {
  const DevModel& M = A.m;
  const int n_r = M.n_r, n_mu = M.n_mu, nl = M.n_lambda;
  const Lds32 L = setup_lds32<CDF_LDS>(A);

  const int lane = __lane_id();
  const double* fixT = A.frozen_T ? A.frozen_T : A.T_coef;
  bool alive = false, exhausted = false;
  Rng32 rng;
  Pk P;
  P.i = -1;
  P.events = 0;
  uint64_t pid = 0;
  bool handed = false;  // this packet tried the hand-off already
  // hand-off bookkeeping: this wavefront's packets are counted in *A.live;
  // hand-offs are allowed (both wave-uniform); the lane's packet was live
  bool counted = false, allow = false, polled = false, was_alive = false;
  uint32_t tot[N_COUNTERS] = {};

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
          P.an.A[0] = M.R_star * (double)st;
          P.an.A[1] = 0.0;
          P.an.A[2] = M.R_star * (double)ws;
          float mup = sqrtf(rng.next());
          float php = 2.0f * (float)KPI * rng.next();
          float sp = sqrtf(fmaxf(0.0f, 1.0f - mup * mup));
          float sn, cs;
          __sincosf(php, &sn, &cs);
          P.d[0] = mup * st + sp * cs * ws;
          P.d[1] = sp * sn;
          P.d[2] = mup * ws - sp * cs * st;
          float nrm = rsqrtf(P.d[0] * P.d[0] + P.d[1] * P.d[1] + P.d[2] * P.d[2]);
          P.d[0] *= nrm; P.d[1] *= nrm; P.d[2] *= nrm;
          float xs = rng.next();
          int lo = 0, hi = nl - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (L.star_cdf[mid] > xs) hi = mid; else lo = mid + 1;
          }
          P.k = lo;
          P.tau = -__logf(rng.next());
          P.q[0] = P.q[1] = P.q[2] = 0.0f;
          P.i = -1;
          P.j = 0;
          P.n_int = 0;
          P.events = 0;
          P.pc_cross = P.pc_scat = P.pc_abs = P.pc_mrw = 0;
          P.rho = P.im = P.Tfix = 0.0;
          P.alpha = 0.0f;
          P.omega = L.omega[P.k];
          P.lim_scale = 0.0f;
          P.seg_seen = 0;
          P.Tc = -1.0;
          P.mrw_T = -2.0;
          P.mrw_Drho = P.mrw_f = 0.0;
          P.mrw_seg = 0;
          P.mrw_lim = 0.0f;
          P.d_safe = 0.0f;
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
          TailState32& ts = ((TailState32*)A.tail)[slot];
          ts.P = P;
          ts.rng = rng;
          ts.pid = pid;
          tot[C_HANDED]++;
          alive = false;
          continue;
        }
      }
    }

    const int fate = event32<false, HG>(P, rng, A, L, fixT, lane);
    if (fate != 0) {
      finish32<false>(P, rng, fate, pid, A, tot, lane);
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

template <bool CDF_LDS, bool HG, int BS>
__global__ void __launch_bounds__(BS) trace_fp32_kernel(TraceArgs A) {
  trace_fp32_body<CDF_LDS, HG>(A);
}

// The packets handed over by the trace launch, one wavefront each; this
// workgroup (of BS threads) is number `rank` of those serving the disk.
template <bool CDF_LDS, bool HG, int BS = BS32>
__device__ __forceinline__ void trace_fp32_tail_body(const TraceArgs& A, unsigned rank) {
  const unsigned wpb = BS / 64;
  if (!A.tail) return;  // traced without hand-off
  const unsigned count = min(*A.tail_count, (unsigned)A.tail_cap);
  if (rank * wpb >= count) return;  // the whole workgroup
  const Lds32 L = setup_lds32<CDF_LDS>(A);
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
    const TailState32& ts = ((const TailState32*)A.tail)[slot];
    Pk S = ts.P;
    WaveRng wr;
    wr.init(ts.rng);
    const uint64_t pid = ts.pid;
    int f;
    do {
      if constexpr (!HG) {
        if (A.runahead && S.i >= 0 && S.alpha > 0.0f) {
          const int n = run_ahead32(S, wr, A, L, fixT, lane);
          if (lane == 0) tot[C_RUN] += (uint32_t)n;
        }
      }
      f = event32<true, HG>(S, wr, A, L, fixT, lane);
    } while (f == 0);
    finish32<true>(S, wr, f, pid, A, tot, lane);
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

template <bool CDF_LDS, bool HG, int BS>
__global__ void __launch_bounds__(BS) trace_fp32_tail_kernel(TraceArgs A) {
  trace_fp32_tail_body<CDF_LDS, HG, BS>(A, blockIdx.x);
}

// Many disks in one launch: workgroup b works on disk block_disk[b] for the
// whole launch (its tables stay in LDS), taking packets from that disk's
// counter; workgroups are shared out in proportion to the disks' packets.
template <bool CDF_LDS>
__global__ void __launch_bounds__(BS32) trace_fp32_batch_kernel(const TraceArgs* __restrict__ As,
                                                                const int* __restrict__ block_disk) {
  trace_fp32_body<CDF_LDS, false>(As[block_disk[blockIdx.x]]);
}

// Hand-offs of a batched launch.  The workgroups are shared out by the
// packets each disk handed off (one wavefront per packet, BS32 / 64 per
// workgroup): every disk with hand-offs gets one workgroup, and the rest go
// in proportion to what each disk wants beyond that.  Every workgroup reads
// the same counts and computes the same split.  The launch has at least one
// workgroup per disk.
template <bool CDF_LDS>
__global__ void __launch_bounds__(BS32)
    trace_fp32_batch_tail_kernel(const TraceArgs* __restrict__ As, int n_disks) {
  const unsigned wpb = BS32 / 64;
  long long n_nz = 0, extra = 0;
  // disks traced without hand-off (wave_events = 0) have no hand-off buffer
  auto handed = [&](int d) -> unsigned {
    return As[d].tail ? min(*As[d].tail_count, (unsigned)As[d].tail_cap) : 0u;
  };
  for (int d = 0; d < n_disks; ++d) {
    const unsigned c = handed(d);
    if (c) {
      ++n_nz;
      extra += (long long)((c + wpb - 1) / wpb) - 1;
    }
  }
  const long long spare = (long long)gridDim.x - n_nz;
  long long first = 0;
  for (int d = 0; d < n_disks; ++d) {
    const unsigned c = handed(d);
    if (!c) continue;
    const long long want = (long long)((c + wpb - 1) / wpb) - 1;
    const long long got = 1 + (extra <= spare ? want : (want * spare) / extra);
    if ((long long)blockIdx.x < first + got) {
      trace_fp32_tail_body<CDF_LDS, false>(As[d], (unsigned)(blockIdx.x - first));
      return;
    }
    first += got;
  }
}

template <bool CDF_LDS, bool HG, int BS>
int launch32(mcrt_ctx* ctx, const TraceArgs& a, size_t lds, hipStream_t s) {
  auto kern = trace_fp32_kernel<CDF_LDS, HG, BS>;
  auto tail = trace_fp32_tail_kernel<CDF_LDS, HG, BS>;
  if (lds > 64 * 1024) {
    (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    (void)hipFuncSetAttribute((const void*)tail, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  }
  int occ = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, BS, lds) != hipSuccess || occ < 1)
    occ = 1;
  int per_cu = ctx->opt.blocks_per_cu > 0 ? ctx->opt.blocks_per_cu : occ;
  long long nb = (long long)ctx->n_cu * per_cu;
  long long need = ((long long)a.n_packets + BS - 1) / BS;
  if (nb > need) nb = need < 1 ? 1 : need;
  // the hand-off launch: enough workgroups for every slot, one workgroup
  // per compute unit at a time; packets are handed off once no more are
  // left than it has wavefronts
  long long tb = (long long)ctx->n_cu * per_cu;
  const long long slots = ((long long)a.tail_cap + BS / 64 - 1) / (BS / 64);
  if (tb > slots) tb = slots;
  TraceArgs b = a;
  // (or the count asked for: more than it has wavefronts queue for them)
  b.live_handoff = a.live_handoff > 0 ? min((unsigned)a.live_handoff, (unsigned)a.tail_cap)
                                      : (unsigned)(tb * (BS / 64));
  // a launch with no more packets than that needs no count
  b.n_waves = a.n_packets <= b.live_handoff ? 0u : (unsigned)(nb * (BS / 64));
  hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(BS), lds, s, b);
  if (a.tail) hipLaunchKernelGGL(tail, dim3((unsigned)tb), dim3(BS), lds, s, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

}  // namespace

template <int BS>
int launch_trace_fp32_bs(mcrt_ctx* ctx, const TraceArgs& a, size_t cap, hipStream_t s) {
  const DevModel& M = ctx->m;
  const size_t vis = (size_t)4 * M.n_r * M.n_mu;
  TraceArgs b = a;
  size_t with = lds32_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda, true);
  if (with <= cap) {
    b.vis_lds = with + vis <= cap;
    const size_t lds = b.vis_lds ? with + vis : with;
    return a.g_asym != 0.0 ? launch32<true, true, BS>(ctx, b, lds, s)
                           : launch32<true, false, BS>(ctx, b, lds, s);
  }
  size_t without = lds32_bytes(M.n_r, M.n_mu, M.n_T, M.n_lambda, false);
  b.vis_lds = without + vis <= cap;
  const size_t lds = b.vis_lds ? without + vis : without;
  return a.g_asym != 0.0 ? launch32<false, true, BS>(ctx, b, lds, s)
                         : launch32<false, false, BS>(ctx, b, lds, s);
}

// LDS: the tables (with the emission CDF when it fits), then the visit
// histogram when that fits too.  512-thread workgroups (the default) take up
// to 155 KB, one per compute unit: 8 wavefronts, the ~215 registers of the
// kernel allowing 2 per SIMD.  768-thread ones share the same LDS among 12
// wavefronts, 3 per SIMD, which caps the registers at 168 (the compiler
// spills ~130 bytes per lane).  256-thread ones take up to half of the LDS,
// so that two share a compute unit (the CDF then usually stays in L2).
int launch_trace_fp32(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s) {
  const int bs = ctx->opt.block_size;
  if (bs == 256) return launch_trace_fp32_bs<256>(ctx, a, (size_t)155 * 1024 / 2, s);
  if (bs == 768) return launch_trace_fp32_bs<768>(ctx, a, (size_t)155 * 1024, s);
  return launch_trace_fp32_bs<512>(ctx, a, (size_t)155 * 1024, s);
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
  e = cdf_lds ? hipFuncSetAttribute((const void*)trace_fp32_batch_tail_kernel<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)
              : hipFuncSetAttribute((const void*)trace_fp32_batch_tail_kernel<false>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  (void)e;
  (void)hipGetLastError();
  return MCRT_OK;
}

int launch_trace_fp32_batch(const TraceArgs* d_args, const int* d_block_disk, int n_disks,
                            int n_blocks, size_t lds, bool cdf_lds, hipStream_t s) {
  if (cdf_lds) {
    hipLaunchKernelGGL(trace_fp32_batch_kernel<true>, dim3(n_blocks), dim3(BS32), lds, s, d_args,
                       d_block_disk);
    hipLaunchKernelGGL(trace_fp32_batch_tail_kernel<true>, dim3(n_blocks), dim3(BS32), lds, s,
                       d_args, n_disks);
  } else {
    hipLaunchKernelGGL(trace_fp32_batch_kernel<false>, dim3(n_blocks), dim3(BS32), lds, s, d_args,
                       d_block_disk);
    hipLaunchKernelGGL(trace_fp32_batch_tail_kernel<false>, dim3(n_blocks), dim3(BS32), lds, s,
                       d_args, n_disks);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(nullptr, std::string("batched trace launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

}  // namespace mcrt
