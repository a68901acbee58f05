// Device helpers shared by the FP64 and FP32 transport kernels: table
// lookups (temperature segment, inversion of the emission G(T), reemission
// bin), the MRW escape-time law, face distances and the LDS layout.
//
// Table lookups replace binary searches by one arithmetic guess plus short
// fix-up scans, and return exactly what a binary search over the same nodes
// returns (largest node index with value <= argument), so the FP64 path makes
// the same choices as a reference that searches.
#pragma once
#include <hip/hip_runtime.h>

#include "mcrt_internal.h"

namespace mcrt {

constexpr double KPI = 3.14159265358979323846;

// ---------------------------------------------------------------- tables
struct TabView {
  int n_T, nl;
  double lnT_lo, inv_dlnT;   // T nodes 1..n_T-1 are T_lo exp((n-1) dlnT)
  double lnG0, inv_du;       // guide over u = ln g from ln G[1]
  int n_guide;
  const double* Tn;          // [n_T]
  const double* G;           // [n_T]
  const double* Drho;        // [n_T]
  const double* kbar;        // [n_T]
  const int* guide;          // [n_guide]: largest n with G[n] <= g at the bin's lower edge
  const double* inv_dT;      // [n_T] 1 / (Tn[n+1] - Tn[n])
  const double* g_slope;     // [n_T] (Tn[n+1] - Tn[n]) / (G[n+1] - G[n])
};

// largest n in [0, n_T-2] with Tn[n] <= T
__device__ __forceinline__ int t_segment(const TabView& t, double T) {
  const int top = t.n_T - 2;
  if (!(T >= t.Tn[1])) return 0;
  if (T >= t.Tn[t.n_T - 1]) return top;
  int n = 1 + (int)((__logf((float)T) - (float)t.lnT_lo) * (float)t.inv_dlnT);
  n = n < 1 ? 1 : (n > top ? top : n);
  while (n > 1 && T < t.Tn[n]) --n;
  while (n < top && T >= t.Tn[n + 1]) ++n;
  return n;
}

// largest n in [0, n_T-2] with G[n] <= g  (g >= 0)
__device__ __forceinline__ int g_segment(const TabView& t, double g) {
  const int top = t.n_T - 2;
  if (!(g >= t.G[1])) return 0;
  if (g >= t.G[t.n_T - 1]) return top;
  int b = (int)((__logf((float)g) - (float)t.lnG0) * (float)t.inv_du);
  b = b < 0 ? 0 : (b >= t.n_guide ? t.n_guide - 1 : b);
  int n = t.guide[b];
  while (n > 1 && g < t.G[n]) --n;
  while (n < top && g >= t.G[n + 1]) ++n;
  return n;
}

__device__ __forceinline__ double T_of_g(const TabView& t, double g) {
  if (g <= 0.0) return 0.0;
  int n = g_segment(t, g);
  return t.Tn[n] + (g - t.G[n]) * t.g_slope[n];
}

// T_of_g that also returns the segment n the temperature lies in (up to
// rounding at the nodes), so a reemission can skip locating it again.
__device__ __forceinline__ double T_of_g_seg(const TabView& t, double g, int& n) {
  if (g <= 0.0) {
    n = 0;
    return 0.0;
  }
  n = g_segment(t, g);
  return t.Tn[n] + (g - t.G[n]) * t.g_slope[n];
}

// T_of_g_seg with a guess of the segment (the one of a nearby g): when
// G[h] <= g < G[h+1] the segment is h, read in one round of table loads;
// otherwise the guide search.  The same n and T as T_of_g_seg.
__device__ __forceinline__ double T_of_g_seg_near(const TabView& t, double g, int h, int& n) {
  if (g > 0.0 && h >= 0 && h <= t.n_T - 2) {
    const double Gh = t.G[h], Gh1 = t.G[h + 1], Th = t.Tn[h], Sh = t.g_slope[h];
    if (Gh <= g && g < Gh1) {
      n = h;
      return Th + (g - Gh) * Sh;
    }
  }
  return T_of_g_seg(t, g, n);
}
// Reemission bin from the difference of the cumulative emission spectra at
// T_new and T_old (linear in T between nodes); T_old < 0: the full spectrum
// at T_new.  Smallest k with D(k) > xi * D(n_lambda - 1).
template <typename C>
struct Reemit {
  const C* an;
  const C* bn;
  const C* ao;
  const C* bo;
  C fn, fo, df;
  bool diff, same;

  __device__ __forceinline__ C D(int k) const {
    if (same) return df * (bn[k] - an[k]);
    C cn = an[k] + fn * (bn[k] - an[k]);
    if (!diff) return cn;
    return cn - (ao[k] + fo * (bo[k] - ao[k]));
  }
};

// With nn_in / no_in >= 0 the segments of T_new / T_old are taken as given
// (from the inversion that produced them) instead of located again.
template <typename C>
__device__ __forceinline__ Reemit<C> reemit_setup(const TabView& t, const C* cdf, double T_old,
                                                  double T_new, int nn_in = -1, int no_in = -1) {
  Reemit<C> R;
  const int nl = t.nl;
  int nn = nn_in >= 0 ? nn_in : t_segment(t, T_new);
  R.fn = (C)((T_new - t.Tn[nn]) * t.inv_dT[nn]);
  R.diff = (T_old >= 0.0) && (T_new > T_old);
  int no = 0;
  R.fo = (C)0;
  if (R.diff) {
    no = no_in >= 0 ? no_in : t_segment(t, T_old);
    R.fo = (C)((T_old - t.Tn[no]) * t.inv_dT[no]);
  }
  R.an = cdf + (size_t)nn * nl;
  R.bn = R.an + nl;
  R.ao = cdf + (size_t)no * nl;
  R.bo = R.ao + nl;
  R.same = R.diff && (no == nn);
  R.df = R.fn - R.fo;
  if (!(R.D(nl - 1) > (C)0)) {
    R.diff = false;
    R.same = false;
  }
  return R;
}

// Smallest k with D(k) > xi * D(nl-1); D is non-decreasing in k.  Eight-way
// search: seven independent probes per level, so a lane waits for three
// rounds of LDS loads instead of seven.
template <typename C>
__device__ __forceinline__ int reemit_search(const Reemit<C>& R, int nl, C xi) {
  C target = xi * R.D(nl - 1);
  int lo = 0, hi = nl - 1;  // answer in [lo, hi]
  while (hi - lo > 7) {
    int w = hi - lo;
    int cnt = 0;
#pragma unroll
    for (int q = 1; q < 8; ++q) cnt += (R.D(lo + (w * q) / 8) > target) ? 0 : 1;
    int nlo = lo + (w * cnt) / 8 + (cnt ? 1 : 0);
    int nhi = cnt < 7 ? lo + (w * (cnt + 1)) / 8 : hi;
    lo = nlo;
    hi = nhi;
  }
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (R.D(mid) > target) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// ------------------------------------------------------------- MRW law
// Survival P(s) in a sphere with an absorbing edge, s = D c t / R0^2, and dP/ds
// (eq. probability RW); the theta-function form below s = 0.1.
__device__ __forceinline__ void mrw_survival(double s, double& P, double& dP) {
  if (s >= 0.1) {
    double x = KPI * KPI * s, sum = 0.0, dsum = 0.0;
    for (int n = 1; n <= 7; ++n) {
      double n2 = (double)(n * n);
      double e = exp(-n2 * x);
      double sg = (n & 1) ? 1.0 : -1.0;
      sum += sg * e;
      dsum -= sg * n2 * KPI * KPI * e;
    }
    P = 2.0 * sum;
    dP = 2.0 * dsum;
  } else {
    double sum = 0.0, dsum = 0.0;
    for (int k = 0; k < 3; ++k) {
      double a = (double)((2 * k + 1) * (2 * k + 1)) * 0.25;
      double e = exp(-a / s);
      sum += e;
      dsum += e * a / (s * s);
    }
    double pre = 2.0 / (sqrt(KPI) * sqrt(s));
    P = 1.0 - pre * sum;
    dP = -(pre * dsum - 0.5 * pre / s * sum);
  }
}

// P(s) = P0: table start in v = ln(-ln P0), three Newton steps
__device__ __forceinline__ double mrw_escape_s(const double* tab, double P0) {
  double v = log(-log(P0));
  double t = (v - MRW_TAB_V0) / (MRW_TAB_V1 - MRW_TAB_V0) * (MRW_TAB_N - 1);
  t = fmin(fmax(t, 0.0), (double)(MRW_TAB_N - 1) - 1e-9);
  int q = (int)t;
  double f = t - q;
  double s = tab[q] + f * (tab[q + 1] - tab[q]);
  for (int it = 0; it < 3; ++it) {
    double P, dP;
    mrw_survival(s, P, dP);
    double sn = s - (P - P0) / dP;
    s = sn > 0.5 * s ? sn : 0.5 * s;
  }
  return s;
}

// ---------------------------------------------------------- face distances
// Leave a sphere from inside: c = r^2 - R^2, pd = p.d.
template <typename R>
__device__ __forceinline__ R exit_sphere(R pd, R c) {
  R disc = pd * pd - c;
  if (c >= (R)0 && (pd > (R)0 || disc < (R)0)) return (R)0;
  disc = disc < (R)0 ? (R)0 : disc;
  R sq = sqrt(disc);
  return pd > (R)0 ? -c / (pd + sq) : -pd + sq;
}

// Reach a sphere from outside; negative if missed.
template <typename R>
__device__ __forceinline__ R enter_sphere(R pd, R c) {
  if (c <= (R)0 && pd < (R)0) return (R)0;
  if (pd >= (R)0) return (R)-1;
  R disc = pd * pd - c;
  if (disc < (R)0) return (R)-1;
  return c / (-pd + sqrt(disc));
}

// Leave across the cone pair |z| = mu r, f(s) = A s^2 + 2 B s + C.  toward_pole:
// the cell is on the wedge side (f < 0), left when f turns positive; else on
// the pole side, left when f turns negative.  Negative: never.
template <typename R>
__device__ __forceinline__ R exit_cone(R A, R B, R C, bool toward_pole) {
  if (toward_pole) {
    if (C >= (R)0 && B > (R)0) return (R)0;
  } else {
    if (C <= (R)0 && B < (R)0) return (R)0;
  }
  R disc = B * B - A * C;
  if (disc < (R)0) return (R)-1;
  R sq = sqrt(disc);
  // the root in the stable form for the sign of B, one division either way
  const bool first = toward_pole ? B > (R)0 : B < (R)0;
  const R num = first ? C : (toward_pole ? -B + sq : -B - sq);
  const R den = first ? (toward_pole ? -B - sq : -B + sq) : A;
  const R v = num / den;
  if (!(v > (R)0) || __builtin_isinf(v)) return (R)-1;
  return v;
}

// Row of mu of a point: largest e with mu2[e] * r2 <= z2 (mu2[0] = 0).
__device__ __forceinline__ int mu_row(const double* mu2, int n_mu, double r2, double z2) {
  int lo = 0, hi = n_mu;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (mu2[mid] * r2 <= z2) lo = mid; else hi = mid;
  }
  return lo;
}

// Value of lane l (a wave-uniform index) of a per-lane double.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long x = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((unsigned long long)x >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Tally add returning the value before it, aggregated over the wavefront:
// the active lanes whose cell is the first active lane's cell (packets that
// absorb in one cell at the same step -- the hot cells of the inner rim) make
// one atomic for their sum, and each takes the interval after its
// predecessors' in lane order, as if they had added one after another; the
// other lanes add on their own.  Call with the lanes that deposit active.
__device__ __forceinline__ double tally_add_grouped(double* tally, int c, double v) {
  const unsigned long long act = __ballot(true);
  const int first = __ffsll((long long)act) - 1;
  const int c0 = __builtin_amdgcn_readlane(c, first);
  const unsigned long long grp = __ballot(c == c0);
  if (__popcll(grp) == 1) return unsafeAtomicAdd(&tally[c], v);
  const int lane = __lane_id();
  double pre = 0.0, tot = 0.0;
  for (unsigned long long m = grp; m; m &= m - 1) {
    const int l = __ffsll((long long)m) - 1;
    const double x = readlane_f64(v, l);
    pre += l < lane ? x : 0.0;
    tot += x;
  }
  double old;
  if (c == c0) {
    double b = 0.0;
    if (lane == first) b = unsafeAtomicAdd(&tally[c0], tot);
    old = readlane_f64(b, first) + pre;
  } else {
    old = unsafeAtomicAdd(&tally[c], v);
  }
  return old;
}

// Wavefront sums of per-lane counters, one atomic per counter per wavefront.
__device__ __forceinline__ void flush_counters(unsigned long long* dst, const uint32_t* v, int n) {
  for (int q = 0; q < n; ++q) {
    unsigned long long x = v[q];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (__lane_id() == 0 && x) atomicAdd(&dst[q], x);
  }
}

}  // namespace mcrt
