// Temperature update and the partial diffusion approximation on gfx950.
//
// update_T: one thread per cell inverts 4 pi m G(T) = E (G linear in T
// between table nodes), FP64.
//
// PDA (Sect. 2.2.1, eq. T diffusion): div(D grad u) = 0, u = T^4, on the
// low-photon region with Dirichlet u from the Monte Carlo T of neighbouring
// cells.  Finite volumes on the (r, mu) cells: the conductance of a face is
// A_f D_f / dist_f with the harmonic mean D_f of the two cells' D = D*rho(T)/rho
// (the diffusion coefficient of Sect. 2.2.3); faces toward the grid edges,
// the pole, the folded midplane and dust-free cells carry no flux.  The
// symmetric 5-point operator is stored as diag + east (i+1) + north (j+1)
// conductances over the whole grid (zero outside the region).  Jacobi-
// preconditioned CG runs two fused streaming kernels per iteration with all
// scalars on the device:
//   K1: p <- z + beta p (z = r/diag, recomputed at the neighbours as well),
//       q = A p, partial p.q
//   K2: alpha = rz/pq, x += alpha p, r -= alpha q, partial r.z; the last
//       workgroup forms beta and the convergence flag.
// Algorithmic traffic per unknown and iteration: K1 reads diag, east, north,
// r, p (neighbour values come from cache) and writes p, q; K2 reads diag,
// x, p, q, r and writes x, r: 15 doubles = 120 bytes.
// Picard sweeps on D(T) wrap the solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mcrt_internal.h"

namespace mcrt {
namespace {

constexpr double PI = 3.14159265358979323846;
constexpr int BS = 256;

__device__ inline int seg_of_g(const double* x, int n, double v) {
  if (v >= x[n - 1]) return n - 2;
  int lo = 0, hi = n - 1;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (x[mid] <= v) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ inline double T_from_g(const double* G, const double* Tn, int n_T, double g) {
  if (g <= 0.0) return 0.0;
  int n = seg_of_g(G, n_T, g);
  return Tn[n] + (g - G[n]) / (G[n + 1] - G[n]) * (Tn[n + 1] - Tn[n]);
}

__device__ inline double table_at(const double* Tn, int n_T, const double* tab, double T) {
  int n = seg_of_g(Tn, n_T, T);
  double f = (T - Tn[n]) / (Tn[n + 1] - Tn[n]);
  return tab[n] + f * (tab[n + 1] - tab[n]);
}

__global__ void update_T_kernel(DevModel M, const double* E, double* T, int nc) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  T[c] = T_from_g(M.G, M.Tn, M.n_T, E[c] * M.inv4pim[c]);
}

// Convergence statistic of the vertical-structure loop (Sect. 2.5): per
// dusty cell entered by >= n_min packets, T from its tally and the relative
// variance of T from the spread of the odd and even packets' halves,
//   s2 = (dlnT/dlnE)^2 ((2 E_half - E) / E)^2,
// the slope a central difference of the inversion over E (1 +- 1e-4); the
// squared relative change against the stored pass and the two variances are
// summed over the cells eligible in both.  The stored T and s2 are replaced.
// sums: [0] sum x^2, [1] sum (s2 + s2_prev), [2] cells (cleared before).
__global__ void conv_kernel(DevModel M, const double* __restrict__ E,
                            const double* __restrict__ E_half, const uint32_t* __restrict__ vis,
                            int n_min, int first, double* T_prev, double* s2_prev, double* sums,
                            int nc) {
  __shared__ double red[3][BS];
  double sx = 0.0, ss = 0.0, n = 0.0;
  for (int c = blockIdx.x * BS + threadIdx.x; c < nc; c += gridDim.x * BS) {
    const double im = M.inv4pim[c];
    const double e = E[c];
    const double g = e * im;
    const double T = T_from_g(M.G, M.Tn, M.n_T, g);
    double s2 = -1.0;
    if (vis[c] >= (uint32_t)n_min && im > 0.0 && e > 0.0 && T > 0.0) {
      const double h = 1e-4;
      const double Tp = T_from_g(M.G, M.Tn, M.n_T, g * (1.0 + h));
      const double Tm = T_from_g(M.G, M.Tn, M.n_T, g * (1.0 - h));
      const double slope = log(Tp / Tm) / (2.0 * h);
      const double rel = (2.0 * E_half[c] - e) / e;
      s2 = slope * slope * rel * rel;
      const double sp = s2_prev[c], Tq = T_prev[c];
      if (!first && sp >= 0.0 && Tq > 0.0) {
        const double x = (T - Tq) / T;
        sx += x * x;
        ss += s2 + sp;
        n += 1.0;
      }
    }
    T_prev[c] = T;
    s2_prev[c] = s2;
  }
  red[0][threadIdx.x] = sx;
  red[1][threadIdx.x] = ss;
  red[2][threadIdx.x] = n;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q)
      if (red[q][0] != 0.0) unsafeAtomicAdd(&sums[q], red[q][0]);
}

// out: R = sqrt(sum x^2 / sum noise^2) (0 when nothing was compared), the
// RMS change, the RMS noise, the cells.
__global__ void conv_finish_kernel(const double* sums, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double n = sums[2];
  out[0] = sums[1] > 0.0 ? sqrt(sums[0] / sums[1]) : 0.0;
  out[1] = n > 0.0 ? sqrt(sums[0] / n) : 0.0;
  out[2] = n > 0.0 ? sqrt(sums[1] / n) : 0.0;
  out[3] = n;
}

// Vertical hydrostatic equilibrium (Sect. 2.5, eq. balance), one thread per
// radial shell at its mid radius r, through the cell centres (z = r mu,
// R = r sqrt(1 - mu^2)): ln(rho T) falls by A times the trapezoidal integral
// of z / (R^3 T) between consecutive centres, A = mu_mol m_p G M / k, T
// floored at T_floor.  The shell keeps its mass; the cell masses'
// 1 / (4 pi m) follow.  A shell with an optically thick dust cell (width >= 1
// at its most opaque wavelength) at T <= 0 (no absorption there, so no
// temperature) is left as it is and counted in *cold: a zero temperature
// would collapse its scale height.  Cold cells transparent at every
// wavelength hold next to no mass and are floored like any other.
__global__ void hydro_kernel(DevModel M, const double* T, double* rho, double* inv4pim, double A,
                             double T_floor, unsigned int* cold) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.n_r) return;
  const int n_mu = M.n_mu;
  for (int j = 0; j < n_mu; ++j) {
    const int c = i * n_mu + j;
    if (rho[c] > 0.0 && !(T[c] > 0.0) && rho[c] * M.chi_max * M.cell_len[c] >= 1.0) {
      atomicAdd(cold, 1u);
      return;
    }
  }
  const double PI_ = 3.14159265358979323846;
  const double a = M.r_edges[i], b = M.r_edges[i + 1];
  const double dr3 = b * b * b - a * a * a;
  const double r = 0.5 * (a + b);
  double mass = 0.0;
  for (int j = 0; j < n_mu; ++j) {
    const double V = 4.0 * PI_ / 3.0 * dr3 * (M.mu_edges[j + 1] - M.mu_edges[j]);
    mass += rho[i * n_mu + j] * V;
  }
  double z_prev = 0.0, h_prev = 0.0, T0 = 0.0, acc = 0.0, s = 0.0;
  for (int j = 0; j < n_mu; ++j) {
    const double mc = 0.5 * (M.mu_edges[j] + M.mu_edges[j + 1]);
    const double z = r * mc;
    const double R = r * sqrt(1.0 - mc * mc);
    const double Tj = fmax(T[i * n_mu + j], T_floor);
    const double h = z / (R * R * R * Tj);
    if (j == 0) T0 = Tj; else acc += 0.5 * (h_prev + h) * (z - z_prev);
    const double f = exp(log(T0 / Tj) - A * acc);
    const double V = 4.0 * PI_ / 3.0 * dr3 * (M.mu_edges[j + 1] - M.mu_edges[j]);
    s += f * V;
    rho[i * n_mu + j] = f;  // the profile, scaled below
    z_prev = z;
    h_prev = h;
  }
  for (int j = 0; j < n_mu; ++j) {
    const int c = i * n_mu + j;
    const double V = 4.0 * PI_ / 3.0 * dr3 * (M.mu_edges[j + 1] - M.mu_edges[j]);
    const double rn = s > 0.0 ? mass * rho[c] / s : 0.0;
    rho[c] = rn;
    const double mc_ = rn * V;
    inv4pim[c] = mc_ > 0.0 ? 1.0 / (4.0 * PI_ * mc_) : 0.0;
  }
}

__global__ void fill_kernel(uint32_t* p, size_t n_words) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; t < n_words; t += stride) p[t] = 0u;
}

// ------------------------------------------------------------------ PDA
struct PdaScalars {
  double rz, rz_new, pq, rz_ref;
  double beta;
  unsigned int ticket;
  int done;
  int iter;
  int pad;
  unsigned long long floor_bits;   // min Dirichlet T (bits of a non-negative double)
  unsigned long long change_bits;  // max |dT/T| of a Picard sweep
  int n_region, n_isolated;
  int changed;                     // component propagation
  int pad2;
};

struct PdaArrays {
  uint8_t* region;
  uint8_t* touch;
  double *Tw, *Tbc, *diag, *aE, *aN, *b, *x, *r, *p0, *p1, *q;
  double *z, *lm;  // preconditioned residual; pivots of the theta-line factorisation
  PdaScalars* sc;
};

__device__ inline bool in_grid(int i, int j, int n_r, int n_mu) {
  return i >= 0 && i < n_r && j >= 0 && j < n_mu;
}

// A neighbour outside the region gives the Monte Carlo solve its boundary
// value (Sect. 2.2.1) when it holds dust and a temperature: a cell in which no
// packet was absorbed has none, and its face carries no flux.
__device__ inline bool gives_bc(const DevModel& M, const uint8_t* region, const double* T_mc,
                                int cb) {
  return M.rho[cb] > 0.0 && region[cb] != 1 && T_mc[cb] > 0.0;
}

// Optical width of cell c at its most opaque wavelength.
__device__ inline double optical_width(const DevModel& M, int c) {
  return M.rho[c] * M.chi_max * M.cell_len[c];
}

// The cells whose Monte Carlo temperature is not trusted (Sect. 3.1): a
// caller mask, else fewer than thr packet entries, or (sigma > 0) a photon
// noise 1 / (4 sqrt(N)) of the temperature above sigma, N the cell's
// absorptions plus MRW deposits (no event: no temperature), in a cell of
// optical width >= 1 (diffusion holds only in opaque matter; a nearly empty
// cell absorbs few packets because it is transparent, not shielded).
// Dust-free cells never join.
struct RegionRule {
  const uint8_t* mask;
  const uint32_t* visits;
  const uint32_t* n_abs;
  const uint32_t* n_mrw;
  int thr;
  double sigma;
};

__device__ inline bool in_region(const DevModel& M, const RegionRule& R, int c) {
  if (!(M.rho[c] > 0.0)) return false;
  if (R.mask) return R.mask[c] != 0;
  if (R.thr > 0 && R.visits[c] < (uint32_t)R.thr) return true;
  if (R.sigma > 0.0 && optical_width(M, c) >= 1.0) {
    const double N = (double)R.n_abs[c] + (double)R.n_mrw[c];
    if (N == 0.0 || 1.0 / (4.0 * sqrt(N)) > R.sigma) return true;
  }
  return false;
}

__global__ void pda_region_kernel(DevModel M, RegionRule R, PdaArrays P) {
  int nc = M.n_r * M.n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  P.region[c] = in_region(M, R, c) ? 1 : 0;
}

// The rule alone, into a caller mask (mcrt_region_mask).
__global__ void region_mask_kernel(DevModel M, RegionRule R, uint8_t* out, int nc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < nc) out[c] = in_region(M, R, c) ? 1 : 0;
}

// touch = region cell with a neighbour that gives a boundary value
__global__ void pda_touch_kernel(DevModel M, const double* T_mc, PdaArrays P) {
  int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  uint8_t t = 0;
  if (P.region[c] == 1) {
    int i = c / n_mu, j = c - i * n_mu;
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    for (int q = 0; q < 4; ++q) {
      int ib = i + di[q], jb = j + dj[q];
      if (!in_grid(ib, jb, n_r, n_mu)) continue;
      int cb = ib * n_mu + jb;
      if (gives_bc(M, P.region, T_mc, cb)) t = 1;
    }
    atomicAdd(&P.sc->n_region, 1);
  }
  P.touch[c] = t;
}

// Spread "touches Dirichlet" through connected region cells by alternating
// row and column scans (each thread one line, forward and backward), in one
// workgroup, until nothing changes; unreached region cells become 2.
__global__ void pda_components_kernel(DevModel M, PdaArrays P) {
  const int n_r = M.n_r, n_mu = M.n_mu;
  __shared__ int changed;
  for (int round = 0; round < 100000; ++round) {
    if (threadIdx.x == 0) changed = 0;
    __syncthreads();
    int local = 0;
    for (int i = threadIdx.x; i < n_r; i += blockDim.x) {  // rows: fixed i, along j
      uint8_t carry = 0;
      for (int j = 0; j < n_mu; ++j) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
      carry = 0;
      for (int j = n_mu - 1; j >= 0; --j) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_mu; j += blockDim.x) {  // columns: fixed j, along i
      uint8_t carry = 0;
      for (int i = 0; i < n_r; ++i) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
      carry = 0;
      for (int i = n_r - 1; i >= 0; --i) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
    }
    if (local) atomicOr(&changed, 1);
    __syncthreads();
    int ch = changed;
    __syncthreads();
    if (!ch) break;
  }
  int n_iso = 0;
  for (int c = threadIdx.x; c < n_r * n_mu; c += blockDim.x) {
    if (P.region[c] == 1 && !P.touch[c]) {
      P.region[c] = 2;
      ++n_iso;
    }
  }
  if (n_iso) atomicAdd(&P.sc->n_isolated, n_iso);
}

__global__ void pda_floor_kernel(DevModel M, const double* T_mc, PdaArrays P) {
  int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc || P.region[c] != 1) return;
  int i = c / n_mu, j = c - i * n_mu;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  double m = INFINITY;
  for (int q = 0; q < 4; ++q) {
    int ib = i + di[q], jb = j + dj[q];
    if (!in_grid(ib, jb, n_r, n_mu)) continue;
    int cb = ib * n_mu + jb;
    if (gives_bc(M, P.region, T_mc, cb)) m = fmin(m, T_mc[cb]);
  }
  if (m < INFINITY) atomicMin(&P.sc->floor_bits, (unsigned long long)__double_as_longlong(m));
}

// full = 1: everything (region counts, floor = +inf); 0: the CG and Picard scalars only
__global__ void pda_reset_scalars_kernel(PdaScalars* S, int full) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  S->rz = S->rz_new = S->pq = S->rz_ref = S->beta = 0.0;
  S->ticket = 0;
  S->done = 0;
  S->iter = 0;
  S->change_bits = 0ull;
  if (full) {
    S->floor_bits = 0x7FF0000000000000ull;
    S->n_region = S->n_isolated = 0;
    S->changed = 0;
  }
}

__global__ void pda_init_T_kernel(DevModel M, const double* T_mc, PdaArrays P) {
  int nc = M.n_r * M.n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double fl = __longlong_as_double((long long)P.sc->floor_bits);
  if (!(fl < INFINITY)) fl = 0.0;
  double t = T_mc[c];
  P.Tbc[c] = t;
  P.Tw[c] = (P.region[c] == 1) ? fmax(t, fl) : t;
}

// face conductance A_f D_f / dist_f between cell a=(i,j) and its neighbour b
struct PdaGeom {
  const double* rc;   // [n_r] (r_i + r_i+1)/2
  const double* thc;  // [n_mu] (acos mu_j + acos mu_j+1)/2
  const double* Ar;   // [n_r][n_mu] area of sphere r_{i+1} over the cell's mu range
  const double* Amu;  // [n_r][n_mu] area of cone mu_{j+1} over the cell's r range
  const double* kscale;  // nullable per-cell extinction scale
};

// resistance R = 1/D = rho s / (D rho)(T) of a dusty cell: the face mean
// 2 / (R_a + R_b) is the harmonic mean of D and stays finite where D itself
// would overflow (densities in the subnormal range)
__device__ inline double Rcell(const DevModel& M, const PdaGeom& g, const double* Tw, int c) {
  double ks = g.kscale ? g.kscale[c] : 1.0;
  return M.rho[c] * ks / table_at(M.Tn, M.n_T, M.Drho, Tw[c]);
}

__global__ void pda_assemble_kernel(DevModel M, PdaGeom g, PdaArrays P) {
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  if (P.region[c] != 1) {
    P.diag[c] = 1.0;
    P.aE[c] = 0.0;
    P.aN[c] = 0.0;
    P.b[c] = 0.0;
    return;
  }
  const int i = c / n_mu, j = c - i * n_mu;
  const double Ra = Rcell(M, g, P.Tw, c);
  double diag = 0.0, rhs = 0.0, aE = 0.0, aN = 0.0;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (int q = 0; q < 4; ++q) {
    int ib = i + di[q], jb = j + dj[q];
    if (!in_grid(ib, jb, n_r, n_mu)) continue;
    int cb = ib * n_mu + jb;
    if (!(M.rho[cb] > 0.0)) continue;
    if (P.region[cb] != 1 && !(P.Tbc[cb] > 0.0)) continue;  // no boundary value
    double Rb = Rcell(M, g, P.Tw, cb);
    double A, dist;
    if (q < 2) {
      int ilo = i < ib ? i : ib;
      A = g.Ar[ilo * n_mu + j];
      dist = fabs(g.rc[ib] - g.rc[i]);
    } else {
      int jlo = j < jb ? j : jb;
      A = g.Amu[i * n_mu + jlo];
      dist = g.rc[i] * fabs(g.thc[jb] - g.thc[j]);
    }
    double a = A * (2.0 / (Ra + Rb)) / dist;
    diag += a;
    if (P.region[cb] == 1) {
      if (q == 1) aE = a;
      if (q == 3) aN = a;
    } else {
      double t = P.Tbc[cb];
      double t2 = t * t;
      rhs += a * (t2 * t2);
    }
  }
  P.diag[c] = diag;
  P.aE[c] = aE;
  P.aN[c] = aN;
  P.b[c] = rhs;
}

__device__ inline double block_sum(double v) {
  __shared__ double red[BS / 64];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  return s;  // valid in thread 0
}

// (A v)_c for region cells (v zero outside the region)
__device__ inline double apply_A(const PdaArrays& P, const double* v, int c, int i, int j, int n_r,
                                 int n_mu) {
  double y = P.diag[c] * v[c];
  if (i + 1 < n_r) y -= P.aE[c] * v[c + n_mu];
  if (i > 0) y -= P.aE[c - n_mu] * v[c - n_mu];
  if (j + 1 < n_mu) y -= P.aN[c] * v[c + 1];
  if (j > 0) y -= P.aN[c - 1] * v[c - 1];
  return y;
}

// r = b - A x, z = r / diag, p = z; partial r.z and b.(b/diag)
__global__ void pcg_start_kernel(int n_r, int n_mu, PdaArrays P) {
  int nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, bb = 0.0;
  if (c < nc) {
    if (P.region[c] == 1) {
      int i = c / n_mu, j = c - i * n_mu;
      double r = P.b[c] - apply_A(P, P.x, c, i, j, n_r, n_mu);
      P.r[c] = r;
      rz = r * r / P.diag[c];
      bb = P.b[c] * P.b[c] / P.diag[c];
    } else {
      P.r[c] = 0.0;
    }
    P.p0[c] = 0.0;
    P.p1[c] = 0.0;
  }
  double s1 = block_sum(rz);
  __syncthreads();
  double s2 = block_sum(bb);
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&P.sc->rz, s1);
    unsafeAtomicAdd(&P.sc->rz_ref, s2);
  }
}

__device__ inline double p_new_at(const PdaArrays& P, const double* pold, double beta, int c) {
  return P.region[c] == 1 ? P.r[c] / P.diag[c] + beta * pold[c] : 0.0;
}

__global__ void pcg_k1(int n_r, int n_mu, PdaArrays P, const double* pold, double* pnew) {
  if (P.sc->done) return;
  const int nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  const double beta = P.sc->iter == 0 ? 0.0 : P.sc->beta;
  double pq = 0.0;
  if (c < nc) {
    if (P.region[c] == 1) {
      int i = c / n_mu, j = c - i * n_mu;
      double pc = p_new_at(P, pold, beta, c);
      double y = P.diag[c] * pc;
      if (i + 1 < n_r) y -= P.aE[c] * p_new_at(P, pold, beta, c + n_mu);
      if (i > 0) y -= P.aE[c - n_mu] * p_new_at(P, pold, beta, c - n_mu);
      if (j + 1 < n_mu) y -= P.aN[c] * p_new_at(P, pold, beta, c + 1);
      if (j > 0) y -= P.aN[c - 1] * p_new_at(P, pold, beta, c - 1);
      pnew[c] = pc;
      P.q[c] = y;
      pq = pc * y;
    } else {
      pnew[c] = 0.0;
      P.q[c] = 0.0;
    }
  }
  double s = block_sum(pq);
  if (threadIdx.x == 0) unsafeAtomicAdd(&P.sc->pq, s);
}

__global__ void pcg_k2(int n_r, int n_mu, PdaArrays P, const double* p, double tol2,
                       int max_iter) {
  if (P.sc->done) return;
  const int nc = n_r * n_mu;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  const double pq = P.sc->pq;
  const double alpha = pq != 0.0 ? P.sc->rz / pq : 0.0;
  double rz = 0.0;
  if (c < nc && P.region[c] == 1) {
    P.x[c] += alpha * p[c];
    double r = P.r[c] - alpha * P.q[c];
    P.r[c] = r;
    rz = r * r / P.diag[c];
  }
  double s = block_sum(rz);
  __shared__ bool last;
  if (threadIdx.x == 0) {
    unsafeAtomicAdd(&P.sc->rz_new, s);
    __threadfence();
    unsigned t = atomicAdd(&P.sc->ticket, 1u);
    last = (t == gridDim.x - 1);
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    PdaScalars* S = P.sc;
    double rzn = __hip_atomic_load(&S->rz_new, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double rzo = S->rz;
    S->beta = rzo != 0.0 ? rzn / rzo : 0.0;
    S->rz = rzn;
    S->rz_new = 0.0;
    S->pq = 0.0;
    S->ticket = 0;
    S->iter += 1;
    if (!(rzn > tol2 * S->rz_ref) || S->iter >= max_iter) S->done = 1;
  }
}

// T <- u^(1/4) on the region, max |dT/T|
__global__ void pda_update_kernel(int nc, PdaArrays P) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc || P.region[c] != 1) return;
  double u = P.x[c] > 0.0 ? P.x[c] : 0.0;
  double Tn = sqrt(sqrt(u));
  double ch = fabs(Tn - P.Tw[c]) / fmax(Tn, 1e-300);
  P.Tw[c] = Tn;
  atomicMax(&P.sc->change_bits, (unsigned long long)__double_as_longlong(ch));
}

__global__ void pda_x_from_T_kernel(int nc, PdaArrays P) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double t = P.Tw[c];
  double t2 = t * t;
  P.x[c] = P.region[c] == 1 ? t2 * t2 : 0.0;
}

__global__ void pda_writeback_kernel(int nc, PdaArrays P, double* T_out, uint8_t* reg_out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  if (P.region[c] == 1) T_out[c] = P.Tw[c];
  reg_out[c] = P.region[c];
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ------------------------------------------------------------------------
// The whole PDA of one disk in one workgroup: region, components, floor,
// Picard sweeps with assembly and Jacobi-PCG, write-back.  No host round
// trips, so it can be captured in a graph; in a batch each workgroup solves
// one disk.  Reductions use wavefront shuffles and LDS.
// ------------------------------------------------------------------------
constexpr int WG = 1024;

struct PdaWgArgs {
  DevModel M;
  PdaArrays P;
  PdaGeom g;
  RegionRule rule;
  const double* T_mc;       // Monte Carlo temperature (Dirichlet data, initial guess)
  double* T_out;            // region cells overwritten
  uint8_t* reg_out;
  int max_sweeps;
  double tol;
  int cg_max_iter;
  double cg_tol2;
  int precond;              // 0 diagonal, 1 theta lines
  mcrt_pda_stats* stats;    // device, nullable
  unsigned int* fails;      // nullable: counts solves that hit a cap (batched passes)
};

template <bool MAX>
__device__ double wg_reduce(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_xor(v, off);
    v = MAX ? fmax(v, o) : v + o;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = MAX ? fmax(r, red[q]) : r + red[q];
  return r;
}

__device__ double apply_A_at(const PdaArrays& P, const double* v, int c, int n_r, int n_mu) {
  int i = c / n_mu, j = c - i * n_mu;
  return apply_A(P, v, c, i, j, n_r, n_mu);
}

__device__ void components_wg(const DevModel& M, const PdaArrays& P, int* changed) {
  const int n_r = M.n_r, n_mu = M.n_mu;
  for (int round = 0; round < 100000; ++round) {
    if (threadIdx.x == 0) *changed = 0;
    __syncthreads();
    int local = 0;
    for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
      uint8_t carry = 0;
      for (int j = 0; j < n_mu; ++j) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
      carry = 0;
      for (int j = n_mu - 1; j >= 0; --j) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n_mu; j += blockDim.x) {
      uint8_t carry = 0;
      for (int i = 0; i < n_r; ++i) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
      carry = 0;
      for (int i = n_r - 1; i >= 0; --i) {
        int c = i * n_mu + j;
        if (P.region[c] != 1) { carry = 0; continue; }
        if (carry && !P.touch[c]) { P.touch[c] = 1; local = 1; }
        carry = P.touch[c];
      }
    }
    if (local) atomicOr(changed, 1);
    __syncthreads();
    int ch = *changed;
    __syncthreads();
    if (!ch) break;
  }
}

// Preconditioner of the workgroup CG.  Diagonal (Jacobi), or block Jacobi
// with one block per radius: the region cells of the theta line i couple to
// their theta neighbours through aN, a tridiagonal system solved exactly
// (Thomas algorithm, one thread per line).  The blocks are diagonally
// dominant (diag sums every face), so the pivots lm stay positive.  lm = 0
// outside the region.
__device__ void line_factor(const PdaArrays& P, int n_r, int n_mu) {
  __syncthreads();
  for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
    const int c0 = i * n_mu;
    double mprev = 0.0;
    for (int j = 0; j < n_mu; ++j) {
      const int c = c0 + j;
      double m = 0.0;
      if (P.region[c] == 1) {
        const double a = j > 0 ? P.aN[c - 1] : 0.0;
        m = 1.0 / (P.diag[c] - a * a * mprev);
      }
      P.lm[c] = m;
      mprev = m;
    }
  }
  __syncthreads();
}

// z = M^-1 v on the region (z = 0 elsewhere).  Ends with a barrier.
__device__ void wg_precond(const PdaArrays& P, int n_r, int n_mu, int precond, const double* v,
                           double* z) {
  const int nc = n_r * n_mu;
  if (!precond) {
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
      z[c] = P.region[c] == 1 ? v[c] / P.diag[c] : 0.0;
    __syncthreads();
    return;
  }
  __syncthreads();  // v written by other threads
  for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
    const int c0 = i * n_mu;
    double y = 0.0;
#pragma unroll 4
    for (int j = 0; j < n_mu; ++j) {
      const int c = c0 + j;
      const double m = P.lm[c];
      const double a = j > 0 ? P.aN[c - 1] : 0.0;
      y = m != 0.0 ? (v[c] + a * y) * m : 0.0;
      z[c] = y;
    }
    double zn = 0.0;
#pragma unroll 4
    for (int j = n_mu - 1; j >= 0; --j) {
      const int c = c0 + j;
      zn = z[c] + P.aN[c] * P.lm[c] * zn;
      z[c] = zn;
    }
  }
  __syncthreads();
}

// Preconditioned CG on the assembled operator: solves A x = b over region ==
// 1 from the given x; stops when r.z <= tol2 * b.(M^-1 b).
__device__ int wg_cg(const PdaArrays& P, int n_r, int n_mu, int precond, const double* b,
                     double* x, int max_iter, double tol2, double* red, double* resid) {
  const int nc = n_r * n_mu;
  if (precond) line_factor(P, n_r, n_mu);
  wg_precond(P, n_r, n_mu, precond, b, P.z);
  double bb = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x)
    if (P.region[c] == 1) bb += b[c] * P.z[c];
  const double ref = wg_reduce<false>(bb, red);
  for (int c = threadIdx.x; c < nc; c += blockDim.x)
    if (P.region[c] == 1) P.r[c] = b[c] - apply_A_at(P, x, c, n_r, n_mu);
  wg_precond(P, n_r, n_mu, precond, P.r, P.z);
  double rz = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    if (P.region[c] != 1) continue;
    P.p0[c] = P.z[c];
    rz += P.r[c] * P.z[c];
  }
  rz = wg_reduce<false>(rz, red);
  int it = 0;
  while (rz > tol2 * ref && it < max_iter) {
    double pq = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      double y = apply_A_at(P, P.p0, c, n_r, n_mu);
      P.q[c] = y;
      pq += P.p0[c] * y;
    }
    pq = wg_reduce<false>(pq, red);
    const double alpha = pq != 0.0 ? rz / pq : 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      x[c] += alpha * P.p0[c];
      P.r[c] -= alpha * P.q[c];
    }
    wg_precond(P, n_r, n_mu, precond, P.r, P.z);
    double rzn = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
      if (P.region[c] == 1) rzn += P.r[c] * P.z[c];
    rzn = wg_reduce<false>(rzn, red);
    const double beta = rz != 0.0 ? rzn / rz : 0.0;
    rz = rzn;
    ++it;
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
      if (P.region[c] == 1) P.p0[c] = P.z[c] + beta * P.p0[c];
    __syncthreads();
  }
  *resid = ref > 0.0 ? sqrt(rz / ref) : 0.0;
  return it;
}

__device__ void pda_wg_body(const PdaWgArgs& a) {
  const DevModel& M = a.M;
  const PdaArrays& P = a.P;
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  __shared__ double red[WG / 64];
  __shared__ int changed;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  // region and Dirichlet contact
  for (int c = threadIdx.x; c < nc; c += blockDim.x) P.region[c] = in_region(M, a.rule, c) ? 1 : 0;
  __syncthreads();
  double n_reg = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    uint8_t t = 0;
    if (P.region[c] == 1) {
      int i = c / n_mu, j = c - i * n_mu;
      for (int q = 0; q < 4; ++q) {
        int ib = i + di[q], jb = j + dj[q];
        if (!in_grid(ib, jb, n_r, n_mu)) continue;
        int cb = ib * n_mu + jb;
        if (gives_bc(M, P.region, a.T_mc, cb)) t = 1;
      }
      n_reg += 1.0;
    }
    P.touch[c] = t;
  }
  n_reg = wg_reduce<false>(n_reg, red);
  components_wg(M, P, &changed);
  double n_iso = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x)
    if (P.region[c] == 1 && !P.touch[c]) {
      P.region[c] = 2;
      n_iso += 1.0;
    }
  n_iso = wg_reduce<false>(n_iso, red);
  // floor: smallest Dirichlet temperature next to the region
  double mflo = -INFINITY;  // max of -T
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    if (P.region[c] != 1) continue;
    int i = c / n_mu, j = c - i * n_mu;
    for (int q = 0; q < 4; ++q) {
      int ib = i + di[q], jb = j + dj[q];
      if (!in_grid(ib, jb, n_r, n_mu)) continue;
      int cb = ib * n_mu + jb;
      if (gives_bc(M, P.region, a.T_mc, cb)) mflo = fmax(mflo, -a.T_mc[cb]);
    }
  }
  double fl = -wg_reduce<true>(mflo, red);
  if (!(fl < INFINITY)) fl = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double t = a.T_mc[c];
    P.Tbc[c] = t;
    P.Tw[c] = (P.region[c] == 1) ? fmax(t, fl) : t;
  }
  __syncthreads();
  const int n_solve = (int)(n_reg - n_iso + 0.5);
  int sweeps = 0, iters_total = 0, iters_last = 0, conv = 0;
  double change = 0.0, resid = 0.0, prev = INFINITY;
  if (n_solve > 0) {
    // Picard sweeps stop when the largest relative change falls below tol, or
    // stalls below sqrt(tol) (the rounding floor of the linear solve)
    const double stall = sqrt(a.tol);
    for (sweeps = 1; sweeps <= a.max_sweeps; ++sweeps) {
      // assemble with D from the current temperature
      for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        if (P.region[c] != 1) {
          P.diag[c] = 1.0; P.aE[c] = 0.0; P.aN[c] = 0.0; P.b[c] = 0.0;
          P.x[c] = 0.0; P.r[c] = 0.0; P.p0[c] = 0.0; P.q[c] = 0.0;
          continue;
        }
        const int i = c / n_mu, j = c - i * n_mu;
        const double Ra = Rcell(M, a.g, P.Tw, c);
        double diag = 0.0, rhs = 0.0, aE = 0.0, aN = 0.0;
        for (int q = 0; q < 4; ++q) {
          int ib = i + di[q], jb = j + dj[q];
          if (!in_grid(ib, jb, n_r, n_mu)) continue;
          int cb = ib * n_mu + jb;
          if (!(M.rho[cb] > 0.0)) continue;
          if (P.region[cb] != 1 && !(P.Tbc[cb] > 0.0)) continue;  // no boundary value
          double Rb = Rcell(M, a.g, P.Tw, cb);
          double A, dist;
          if (q < 2) {
            int ilo = i < ib ? i : ib;
            A = a.g.Ar[ilo * n_mu + j];
            dist = fabs(a.g.rc[ib] - a.g.rc[i]);
          } else {
            int jlo = j < jb ? j : jb;
            A = a.g.Amu[i * n_mu + jlo];
            dist = a.g.rc[i] * fabs(a.g.thc[jb] - a.g.thc[j]);
          }
          double cond = A * (2.0 / (Ra + Rb)) / dist;
          diag += cond;
          if (P.region[cb] == 1) {
            if (q == 1) aE = cond;
            if (q == 3) aN = cond;
          } else {
            double t = P.Tbc[cb], t2 = t * t;
            rhs += cond * (t2 * t2);
          }
        }
        P.diag[c] = diag; P.aE[c] = aE; P.aN[c] = aN; P.b[c] = rhs;
        double t = P.Tw[c], t2 = t * t;
        P.x[c] = t2 * t2;
      }
      __syncthreads();
      // PCG from the current T^4
      int it = wg_cg(P, n_r, n_mu, a.precond, P.b, P.x, a.cg_max_iter, a.cg_tol2, red, &resid);
      iters_total += it;
      iters_last = it;
      double ch = 0.0;
      for (int c = threadIdx.x; c < nc; c += blockDim.x) {
        if (P.region[c] != 1) continue;
        double u = P.x[c] > 0.0 ? P.x[c] : 0.0;
        double Tn = sqrt(sqrt(u));
        ch = fmax(ch, fabs(Tn - P.Tw[c]) / fmax(Tn, 1e-300));
        P.Tw[c] = Tn;
      }
      change = wg_reduce<true>(ch, red);
      if (change < a.tol || (change < stall && change >= prev)) {
        conv = 1;
        break;
      }
      prev = change;
    }
    if (sweeps > a.max_sweeps) sweeps = a.max_sweeps;
  } else {
    conv = 1;
  }
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    if (P.region[c] == 1) a.T_out[c] = P.Tw[c];
    a.reg_out[c] = P.region[c];
  }
  if (threadIdx.x == 0 && a.fails && (iters_last >= a.cg_max_iter || !conv))
    atomicAdd(a.fails, 1u);
  if (threadIdx.x == 0 && a.stats) {
    mcrt_pda_stats s;
    s.sweeps = sweeps;
    s.cg_iters_total = iters_total;
    s.cg_iters_last = iters_last;
    s.n_region = n_solve;
    s.n_isolated = (int)(n_iso + 0.5);
    s.last_change = change;
    s.last_residual = resid;
    s.converged = conv;
    *a.stats = s;
  }
}

// One workgroup per disk, arguments in device memory (batched passes and
// graph capture); or one disk with its arguments passed by value.
__global__ void __launch_bounds__(WG) pda_wg_kernel(const PdaWgArgs* args) {
  pda_wg_body(args[blockIdx.x]);
}

__global__ void __launch_bounds__(WG) pda_wg_kernel_val(PdaWgArgs a) { pda_wg_body(a); }

}  // namespace

int launch_update_T(mcrt_ctx* ctx, hipStream_t s) {
  int nc = ctx->n_cells;
  hipLaunchKernelGGL(update_T_kernel, dim3((nc + BS - 1) / BS), dim3(BS), 0, s, ctx->m,
                     ctx->t.E_abs, ctx->d_T, nc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("update_T launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

int launch_hydrostatic(mcrt_ctx* ctx, double A, double T_floor, hipStream_t s) {
  const int n_r = ctx->n_r;
  if (launch_zero(&ctx->d_health->hydro_cold, 4, s) != MCRT_OK) {
    set_error(ctx, "hydrostatic: clearing the cold-shell count failed");
    return MCRT_E_HIP;
  }
  hipLaunchKernelGGL(hydro_kernel, dim3((n_r + 63) / 64), dim3(64), 0, s, ctx->m, ctx->d_T,
                     (double*)ctx->m.rho, (double*)ctx->m.inv4pim, A, T_floor,
                     &ctx->d_health->hydro_cold);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(ctx, std::string("hydrostatic launch: ") + hipGetErrorString(e));
    return MCRT_E_HIP;
  }
  return MCRT_OK;
}

// The convergence state of a context: T [n_cells], s2 [n_cells], then the
// sums [4] and the result [4].
int launch_convergence(mcrt_ctx* ctx, int n_min, int first, hipStream_t s) {
  const int nc = ctx->n_cells;
  double* T_prev = ctx->d_conv;
  double* s2_prev = T_prev + nc;
  double* sums = s2_prev + nc;
  int r = launch_zero(sums, 4 * sizeof(double), s);
  if (r) return r;
  unsigned nb = (unsigned)((nc + BS - 1) / BS);
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(conv_kernel, dim3(nb), dim3(BS), 0, s, ctx->m, ctx->t.E_abs, ctx->d_E_half,
                     ctx->t.visits, n_min, first, T_prev, s2_prev, sums, nc);
  hipLaunchKernelGGL(conv_finish_kernel, dim3(1), dim3(64), 0, s, sums, sums + 4);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

const double* conv_result(const mcrt_ctx* ctx) { return ctx->d_conv + 2 * (size_t)ctx->n_cells + 4; }

int launch_zero(void* p, size_t bytes, hipStream_t s) {
  size_t words = bytes / 4;
  if (!words) return MCRT_OK;
  unsigned nb = (unsigned)((words + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(fill_kernel, dim3(nb), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

namespace {
// Geometry of the finite volumes: cell-centre radii and angles, and the areas
// of the faces r_{i+1} (over the cell's mu range) and mu_{j+1} (over its r
// range), both hemispheres.  Every PDA solve takes it from this kernel, so
// all solvers see the same numbers.
__global__ void pda_geom_kernel(DevModel M, double* rc, double* thc, double* Ar, double* Amu) {
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    const int i = c / n_mu, j = c - i * n_mu;
    const double a = M.r_edges[i], b = M.r_edges[i + 1];
    const double m0 = M.mu_edges[j], m1 = M.mu_edges[j + 1];
    if (j == 0) rc[i] = 0.5 * (a + b);
    if (i == 0) thc[j] = 0.5 * (acos(m0) + acos(m1));
    Ar[c] = 2.0 * PI * b * b * 2.0 * (m1 - m0);
    Amu[c] = PI * (b * b - a * a) * 2.0 * sqrt(fmax(0.0, 1.0 - m1 * m1));
  }
}
}  // namespace

// Geometry arrays of the PDA live at the start of the PDA scratch blob.
static int pda_alloc(mcrt_ctx* ctx, PdaArrays& P, PdaGeom& g) {
  const int nc = ctx->n_cells, n_r = ctx->n_r, n_mu = ctx->n_mu;
  size_t nd = (size_t)nc * sizeof(double);
  size_t bytes = align256(sizeof(PdaScalars)) + 2 * align256(nc) + 13 * align256(nd) +
                 align256(n_r * sizeof(double)) + align256(n_mu * sizeof(double)) +
                 2 * align256(nd) + align256(sizeof(PdaWgArgs)) + align256(sizeof(mcrt_pda_stats));
  if (ctx->d_pda_blob == nullptr) {
    if (hipMalloc(&ctx->d_pda_blob, bytes) != hipSuccess) {
      set_error(ctx, "PDA scratch allocation failed");
      return MCRT_E_OOM;
    }
    ctx->pda_bytes = bytes;
    // geometry, once per context (before any stream work that reads it)
    char* q = (char*)ctx->d_pda_blob;
    q += align256(sizeof(PdaScalars)) + 2 * align256(nc) + 13 * align256(nd);
    double* rc = (double*)q;
    q += align256(n_r * sizeof(double));
    double* thc = (double*)q;
    q += align256(n_mu * sizeof(double));
    double* Ar = (double*)q;
    q += align256(nd);
    double* Amu = (double*)q;
    const unsigned nb = (unsigned)std::min<size_t>(((size_t)nc + 255) / 256, 1024);
    hipLaunchKernelGGL(pda_geom_kernel, dim3(nb), dim3(256), 0, 0, ctx->m, rc, thc, Ar, Amu);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
      set_error(ctx, "PDA geometry failed");
      return MCRT_E_HIP;
    }
  }
  char* q = (char*)ctx->d_pda_blob;
  P.sc = (PdaScalars*)q;
  q += align256(sizeof(PdaScalars));
  P.region = (uint8_t*)q;
  q += align256(nc);
  P.touch = (uint8_t*)q;
  q += align256(nc);
  double** arr[13] = {&P.Tw, &P.Tbc, &P.diag, &P.aE, &P.aN, &P.b, &P.x, &P.r, &P.p0, &P.p1, &P.q,
                      &P.z, &P.lm};
  for (auto a : arr) {
    *a = (double*)q;
    q += align256(nd);
  }
  g.rc = (const double*)q;
  q += align256(n_r * sizeof(double));
  g.thc = (const double*)q;
  q += align256(n_mu * sizeof(double));
  g.Ar = (const double*)q;
  q += align256(nd);
  g.Amu = (const double*)q;
  g.kscale = nullptr;
  return MCRT_OK;
}

// device slots for one single-workgroup solve: arguments and statistics
static void pda_wg_slots(mcrt_ctx* ctx, PdaWgArgs** args, mcrt_pda_stats** stats) {
  const int nc = ctx->n_cells;
  size_t nd = (size_t)nc * sizeof(double);
  char* q = (char*)ctx->d_pda_blob + ctx->pda_bytes - align256(sizeof(PdaWgArgs)) -
            align256(sizeof(mcrt_pda_stats));
  (void)nd;
  *args = (PdaWgArgs*)q;
  *stats = (mcrt_pda_stats*)(q + align256(sizeof(PdaWgArgs)));
}

static RegionRule region_rule(const mcrt_ctx* ctx, const uint8_t* mask) {
  RegionRule R;
  R.mask = mask;
  R.visits = ctx->t.visits;
  R.n_abs = ctx->t.n_abs;
  R.n_mrw = ctx->t.n_mrw;
  R.thr = ctx->opt.pda_visits;
  R.sigma = ctx->opt.pda_sigma;
  return R;
}

int launch_region_mask(mcrt_ctx* ctx, int visits_min, double sigma, uint8_t* out, hipStream_t s) {
  RegionRule R = region_rule(ctx, nullptr);
  R.thr = visits_min;
  R.sigma = sigma;
  const int nc = ctx->n_cells;
  hipLaunchKernelGGL(region_mask_kernel, dim3((nc + BS - 1) / BS), dim3(BS), 0, s, ctx->m, R, out,
                     nc);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

static int pda_solve_wg(mcrt_ctx* ctx, const uint8_t* mask, mcrt_pda_stats* st, hipStream_t s,
                        const PdaArrays& P, const PdaGeom& g) {
  PdaWgArgs h;
  h.M = ctx->m;
  h.P = P;
  h.g = g;
  h.rule = region_rule(ctx, mask);
  h.fails = nullptr;
  h.T_mc = ctx->d_T;
  h.T_out = ctx->d_T;
  h.reg_out = ctx->d_region;
  h.max_sweeps = ctx->opt.pda_max_sweeps;
  h.tol = ctx->opt.pda_tol;
  h.cg_max_iter = ctx->opt.cg_max_iter;
  h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
  h.precond = ctx->opt.pda_precond;
  PdaWgArgs* d_args;
  mcrt_pda_stats* d_stats;
  pda_wg_slots(ctx, &d_args, &d_stats);
  h.stats = d_stats;
  // the previous solve on this context may still read the argument slot
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(d_args, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) {
    set_error(ctx, "PDA argument upload failed");
    return MCRT_E_HIP;
  }
  hipLaunchKernelGGL(pda_wg_kernel, dim3(1), dim3(WG), 0, s, (const PdaWgArgs*)d_args);
  if (hipGetLastError() != hipSuccess) {
    set_error(ctx, "PDA launch failed");
    return MCRT_E_HIP;
  }
  mcrt_pda_stats out{};
  if (hipMemcpyAsync(&out, d_stats, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error(ctx, "PDA failed");
    return MCRT_E_HIP;
  }
  if (st) *st = out;
  if (out.cg_iters_last >= ctx->opt.cg_max_iter || !out.converged) return MCRT_E_NOT_CONVERGED;
  return out.n_isolated > 0 ? MCRT_E_SINGULAR_REGION : MCRT_OK;
}

int pda_solve(mcrt_ctx* ctx, const uint8_t* mask, mcrt_pda_stats* st, hipStream_t s) {
  PdaArrays P;
  PdaGeom g;
  ctx->lin_ready = false;  // the scratch of a linear solve is overwritten
  int rc = pda_alloc(ctx, P, g);
  if (rc) return rc;
  const int nc = ctx->n_cells, n_r = ctx->n_r, n_mu = ctx->n_mu;
  if (ctx->opt.pda_solver == 2 || (ctx->opt.pda_solver == 0 && nc <= 65536))
    return pda_solve_wg(ctx, mask, st, s, P, g);
  const dim3 grid((nc + BS - 1) / BS), blk(BS);
  const DevModel& M = ctx->m;
  hipLaunchKernelGGL(pda_reset_scalars_kernel, dim3(1), dim3(64), 0, s, P.sc, 1);
  hipLaunchKernelGGL(pda_region_kernel, grid, blk, 0, s, M, region_rule(ctx, mask), P);
  hipLaunchKernelGGL(pda_touch_kernel, grid, blk, 0, s, M, ctx->d_T, P);
  hipLaunchKernelGGL(pda_components_kernel, dim3(1), dim3(256), 0, s, M, P);
  hipLaunchKernelGGL(pda_floor_kernel, grid, blk, 0, s, M, ctx->d_T, P);
  hipLaunchKernelGGL(pda_init_T_kernel, grid, blk, 0, s, M, ctx->d_T, P);
  PdaScalars h{};
  hipMemcpyAsync(&h, P.sc, sizeof(h), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    set_error(ctx, "PDA setup failed");
    return MCRT_E_HIP;
  }
  mcrt_pda_stats out{};
  out.n_region = h.n_region - h.n_isolated;
  out.n_isolated = h.n_isolated;
  out.converged = 1;
  int status = MCRT_OK;
  if (out.n_region > 0) {
    const double tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
    const int chunk = 16;
    int sweep;
    double prev = INFINITY;
    out.converged = 0;
    for (sweep = 1; sweep <= ctx->opt.pda_max_sweeps; ++sweep) {
      hipLaunchKernelGGL(pda_assemble_kernel, grid, blk, 0, s, M, g, P);
      hipLaunchKernelGGL(pda_x_from_T_kernel, grid, blk, 0, s, nc, P);
      hipLaunchKernelGGL(pda_reset_scalars_kernel, dim3(1), dim3(64), 0, s, P.sc, 0);
      hipLaunchKernelGGL(pcg_start_kernel, grid, blk, 0, s, n_r, n_mu, P);
      int it = 0;
      for (;;) {
        for (int q = 0; q < chunk; ++q, ++it) {
          const double* pold = (it & 1) ? P.p1 : P.p0;
          double* pnew = (it & 1) ? P.p0 : P.p1;
          hipLaunchKernelGGL(pcg_k1, grid, blk, 0, s, n_r, n_mu, P, pold, pnew);
          hipLaunchKernelGGL(pcg_k2, grid, blk, 0, s, n_r, n_mu, P, (const double*)pnew, tol2,
                             ctx->opt.cg_max_iter);
        }
        hipMemcpyAsync(&h, P.sc, sizeof(h), hipMemcpyDeviceToHost, s);
        if (hipStreamSynchronize(s) != hipSuccess) {
          set_error(ctx, "PDA CG failed");
          return MCRT_E_HIP;
        }
        if (h.done) break;
      }
      out.cg_iters_total += h.iter;
      out.cg_iters_last = h.iter;
      out.last_residual = h.rz_ref > 0.0 ? std::sqrt(h.rz / h.rz_ref) : 0.0;
      if (h.iter >= ctx->opt.cg_max_iter) status = MCRT_E_NOT_CONVERGED;
      hipLaunchKernelGGL(pda_update_kernel, grid, blk, 0, s, nc, P);
      hipMemcpyAsync(&h, P.sc, sizeof(h), hipMemcpyDeviceToHost, s);
      if (hipStreamSynchronize(s) != hipSuccess) {
        set_error(ctx, "PDA update failed");
        return MCRT_E_HIP;
      }
      double change;
      unsigned long long bits = h.change_bits;
      std::memcpy(&change, &bits, sizeof(change));
      out.last_change = change;
      out.sweeps = sweep;
      if (change < ctx->opt.pda_tol || (change < std::sqrt(ctx->opt.pda_tol) && change >= prev)) {
        out.converged = 1;
        break;
      }
      prev = change;
    }
    if (!out.converged && status == MCRT_OK) status = MCRT_E_NOT_CONVERGED;
  }
  hipLaunchKernelGGL(pda_writeback_kernel, grid, blk, 0, s, nc, P, ctx->d_T, ctx->d_region);
  if (hipGetLastError() != hipSuccess) {
    set_error(ctx, "PDA launch failed");
    return MCRT_E_HIP;
  }
  if (st) *st = out;
  if (status == MCRT_OK && out.n_isolated > 0) status = MCRT_E_SINGULAR_REGION;
  return status;
}

// ------------------------------------------------------------------------
// Differentiation of the PDA with respect to the density and an extinction
// scale per cell.  The forward is one linear solve with the diffusion
// coefficient frozen at a given temperature field T_D:
//   D_c = (D rho)(T_D,c) / (rho_c s_c),  A(D) u = b(D),  T = u^(1/4) on the region,
// Dirichlet T_bc elsewhere.  For an objective J(T) the adjoint solves
// A lambda = dJ/du (A is symmetric) and, with the residual r = A u - b,
//   dJ/dp = - lambda . dr/dp,   dr/dp = sum_faces (dr/da_f)(da_f/dD_c)(dD_c/dp),
// a_f = A_f 2 D_a D_b / ((D_a + D_b) dist_f), dD_c/dlog rho_c = -D_c,
// dD_c/ds_c = -D_c / s_c.  The face term lambda . dr/da_f is
// (lambda_a - lambda_b)(u_a - u_b) between two region cells and
// lambda_a (u_a - u_b) between a region cell a and a Dirichlet cell b.
// ------------------------------------------------------------------------
namespace {

struct PdaLinArgs {
  DevModel M;
  PdaArrays P;
  PdaGeom g;
  const uint8_t* mask;
  const double* rho;       // per-cell density (defaults to the model's)
  const double* kscale;    // nullable
  const double* T_D;
  const double* T_bc;
  double* T_out;
  uint8_t* reg_out;
  int cg_max_iter;
  double cg_tol2;
  int precond;
  mcrt_pda_stats* stats;
  // adjoint
  const double* dJdT;
  double* g_logrho;
  double* g_kscale;
  double* nl;              // nonlinear adjoint: NL_ARRAYS work arrays of n_cells doubles
};

// face conductance from the two resistances, and its derivative by R_a
__device__ inline double lin_cond(const PdaLinArgs& a, int i, int j, int ib, int jb, double Ra,
                                  double Rb, double* dA_dRa) {
  double A, dist;
  const int n_mu = a.M.n_mu;
  if (ib != i) {
    int ilo = i < ib ? i : ib;
    A = a.g.Ar[ilo * n_mu + j];
    dist = fabs(a.g.rc[ib] - a.g.rc[i]);
  } else {
    int jlo = j < jb ? j : jb;
    A = a.g.Amu[i * n_mu + jlo];
    dist = a.g.rc[i] * fabs(a.g.thc[jb] - a.g.thc[j]);
  }
  double s = Ra + Rb;
  if (dA_dRa) *dA_dRa = -A / dist * 2.0 / (s * s);
  return A * (2.0 / s) / dist;
}

// Forward: region from the mask (components without Dirichlet contact -> 2),
// R = 1/D from T_D, one linear solve.  Keeps u (x), R (p1), s (b), T_bc (Tbc)
// and the operator for the adjoint.
__global__ void __launch_bounds__(WG) pda_linear_kernel(const PdaLinArgs* args) {
  const PdaLinArgs& a = *args;
  const DevModel& M = a.M;
  const PdaArrays& P = a.P;
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  __shared__ double red[WG / 64];
  __shared__ int changed;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    P.region[c] = (a.rho[c] > 0.0 && a.mask[c] != 0) ? 1 : 0;
    double s = a.kscale ? a.kscale[c] : 1.0;
    P.p1[c] = a.rho[c] > 0.0 ? a.rho[c] * s / table_at(M.Tn, M.n_T, M.Drho, a.T_D[c]) : 0.0;
    P.Tbc[c] = a.T_bc[c];
  }
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    uint8_t t = 0;
    if (P.region[c] == 1) {
      int i = c / n_mu, j = c - i * n_mu;
      for (int q = 0; q < 4; ++q) {
        int ib = i + di[q], jb = j + dj[q];
        if (!in_grid(ib, jb, n_r, n_mu)) continue;
        int cb = ib * n_mu + jb;
        if (a.rho[cb] > 0.0 && P.region[cb] != 1) t = 1;
      }
    }
    P.touch[c] = t;
  }
  __syncthreads();
  components_wg(M, P, &changed);
  for (int c = threadIdx.x; c < nc; c += blockDim.x)
    if (P.region[c] == 1 && !P.touch[c]) P.region[c] = 2;
  __syncthreads();
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    P.x[c] = 0.0; P.r[c] = 0.0; P.p0[c] = 0.0; P.q[c] = 0.0;
    if (P.region[c] != 1) {
      P.diag[c] = 1.0; P.aE[c] = 0.0; P.aN[c] = 0.0; P.Tw[c] = 0.0;
      continue;
    }
    const int i = c / n_mu, j = c - i * n_mu;
    double diag = 0.0, rhs = 0.0, aE = 0.0, aN = 0.0;
    for (int q = 0; q < 4; ++q) {
      int ib = i + di[q], jb = j + dj[q];
      if (!in_grid(ib, jb, n_r, n_mu)) continue;
      int cb = ib * n_mu + jb;
      if (!(a.rho[cb] > 0.0)) continue;
      double cond = lin_cond(a, i, j, ib, jb, P.p1[c], P.p1[cb], nullptr);
      diag += cond;
      if (P.region[cb] == 1) {
        if (q == 1) aE = cond;
        if (q == 3) aN = cond;
      } else {
        double t = P.Tbc[cb], t2 = t * t;
        rhs += cond * (t2 * t2);
      }
    }
    P.diag[c] = diag; P.aE[c] = aE; P.aN[c] = aN;
    P.Tw[c] = rhs;  // right-hand side
    double t = a.T_D[c], t2 = t * t;
    P.x[c] = t2 * t2;
  }
  __syncthreads();
  double resid;
  int it = wg_cg(P, n_r, n_mu, a.precond, P.Tw, P.x, a.cg_max_iter, a.cg_tol2, red, &resid);
  double n1 = 0.0, n2 = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    n1 += P.region[c] == 1 ? 1.0 : 0.0;
    n2 += P.region[c] == 2 ? 1.0 : 0.0;
    P.b[c] = a.kscale ? a.kscale[c] : 1.0;
    double u = P.x[c] > 0.0 ? P.x[c] : 0.0;
    a.T_out[c] = P.region[c] == 1 ? sqrt(sqrt(u)) : P.Tbc[c];
    a.reg_out[c] = P.region[c];
  }
  n1 = wg_reduce<false>(n1, red);
  n2 = wg_reduce<false>(n2, red);
  if (threadIdx.x == 0 && a.stats) {
    mcrt_pda_stats s{};
    s.sweeps = 1;
    s.cg_iters_total = it;
    s.cg_iters_last = it;
    s.n_region = (int)n1;
    s.n_isolated = (int)n2;
    s.last_residual = resid;
    s.converged = 1;  // one linear solve, no Picard sweeps
    *a.stats = s;
  }
}

// dJ/d(log rho_c) and dJ/ds_c from the adjoint lambda: -lambda . dr/dp
// through the resistances R = rho s / (D rho)(T) of the kept solve.
__device__ void grad_from_lambda(const PdaLinArgs& a, const PdaArrays& P, const double* lam) {
  const DevModel& M = a.M;
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double dJdR = 0.0;
    if (a.rho[c] > 0.0) {
      const int i = c / n_mu, j = c - i * n_mu;
      const bool rc_ = P.region[c] == 1;
      double uc = rc_ ? P.x[c] : P.Tbc[c] * P.Tbc[c] * P.Tbc[c] * P.Tbc[c];
      for (int q = 0; q < 4; ++q) {
        int ib = i + di[q], jb = j + dj[q];
        if (!in_grid(ib, jb, n_r, n_mu)) continue;
        int cb = ib * n_mu + jb;
        if (!(a.rho[cb] > 0.0)) continue;
        const bool rb = P.region[cb] == 1;
        if (!rc_ && !rb) continue;
        double ub = rb ? P.x[cb] : P.Tbc[cb] * P.Tbc[cb] * P.Tbc[cb] * P.Tbc[cb];
        double lam_dr;  // lambda . dr/da_f
        if (rc_ && rb) lam_dr = (lam[c] - lam[cb]) * (uc - ub);
        else if (rc_) lam_dr = lam[c] * (uc - ub);
        else lam_dr = lam[cb] * (ub - uc);
        double dA;
        (void)lin_cond(a, i, j, ib, jb, P.p1[c], P.p1[cb], &dA);
        dJdR -= lam_dr * dA;
      }
    }
    // dR/dlog rho = R, dR/ds = R/s
    const double R = P.p1[c];
    a.g_logrho[c] = R * dJdR;
    if (a.g_kscale) a.g_kscale[c] = R / P.b[c] * dJdR;
  }
}

// Adjoint of the linear solve above (same workgroup arrays).
__global__ void __launch_bounds__(WG) pda_adjoint_kernel(const PdaLinArgs* args) {
  const PdaLinArgs& a = *args;
  const DevModel& M = a.M;
  const PdaArrays& P = a.P;
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  __shared__ double red[WG / 64];
  // right-hand side dJ/du = dJ/dT * T / (4 u) on the region, staged in the
  // g_logrho output (overwritten by the gradient at the end); lambda in Tw
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double g = 0.0;
    if (P.region[c] == 1) {
      double u = P.x[c];
      g = u > 0.0 ? a.dJdT[c] * sqrt(sqrt(u)) / (4.0 * u) : 0.0;
    }
    P.Tw[c] = 0.0;
    a.g_logrho[c] = g;
  }
  __syncthreads();
  double resid;
  int it = wg_cg(P, n_r, n_mu, a.precond, a.g_logrho, P.Tw, a.cg_max_iter, a.cg_tol2, red, &resid);
  __syncthreads();
  grad_from_lambda(a, P, P.Tw);
  if (threadIdx.x == 0 && a.stats) {
    mcrt_pda_stats s{};
    s.sweeps = 1;
    s.cg_iters_total = it;
    s.cg_iters_last = it;
    s.last_residual = resid;
    s.converged = 1;  // one linear solve, no Picard sweeps
    *a.stats = s;
  }
}

// Adjoint of the nonlinear PDA (Picard to its fixed point, D = D(T)).  At the
// fixed point the residual r_c = sum_f a_f (u_c - u_b) of every region cell
// vanishes; its Jacobian J = dr/du holds, beside the conductances, their
// dependence on u through R(T(u)):
//   J_cc = sum_f [a_f + da_f/dR_c dR_c/du_c (u_c - u_b)],
//   J_cb = -a_f + da_f/dR_b dR_b/du_b (u_c - u_b)       (b in the region),
// da_f/dR = -a_f / (R_c + R_b), dR/du = -R (D rho)'(T) / (D rho)(T) T / (4 u),
// (D rho)' the slope of the table segment.  J is not symmetric: the adjoint
// J^T lambda = dJ/du is solved by BiCGSTAB with the diagonal as
// preconditioner, then the gradient is that of the linear adjoint with this
// lambda.  Work arrays (of the nl scratch): lambda, r, rh, p, v, s, t, y, z,
// the diagonal, per cell b the four couplings J_cb from its neighbours, and
// the factors of the theta-line preconditioner.  That preconditioner
// (pda_precond = 1; else the diagonal) solves the tridiagonal block of J^T
// along each radius exactly, as the linear solve's does for A: the couplings
// across theta dominate where the cells are thin in theta.
constexpr int NL_ARRAYS = 16;

__global__ void __launch_bounds__(WG) pda_nl_adjoint_kernel(const PdaLinArgs* args) {
  const PdaLinArgs& a = *args;
  const DevModel& M = a.M;
  const PdaArrays& P = a.P;
  const int n_r = M.n_r, n_mu = M.n_mu, nc = n_r * n_mu;
  __shared__ double red[WG / 64];
  double* const lam = a.nl;
  double* const r = lam + nc;
  double* const rh = r + nc;
  double* const p = rh + nc;
  double* const v = p + nc;
  double* const sv = v + nc;
  double* const t = sv + nc;
  double* const y = t + nc;
  double* const z = y + nc;
  double* const jd = z + nc;
  double* const in0 = jd + nc;  // in0 .. in3: J_cb from the neighbour in direction q
  double* const cp = in0 + 4 * (size_t)nc;  // line factors: modified super-diagonal
  double* const dinv = cp + nc;             // and reciprocal pivots
  const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
  auto u_of = [&](int c) -> double {
    if (P.region[c] == 1) return P.x[c];
    const double tb = P.Tbc[c], t2 = tb * tb;
    return t2 * t2;
  };
  auto dRdu_of = [&](int c) -> double {  // region cells
    const double u = P.x[c];
    if (!(u > 0.0) || !(a.rho[c] > 0.0)) return 0.0;
    const double T = sqrt(sqrt(u));
    const int n = seg_of_g(M.Tn, M.n_T, T);
    const double f = (T - M.Tn[n]) / (M.Tn[n + 1] - M.Tn[n]);
    const double Drho = M.Drho[n] + f * (M.Drho[n + 1] - M.Drho[n]);
    const double slope = (M.Drho[n + 1] - M.Drho[n]) / (M.Tn[n + 1] - M.Tn[n]);
    return -P.p1[c] * slope / Drho * T / (4.0 * u);
  };
  // the transposed operator's coefficients
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double d = 1.0, cq[4] = {0.0, 0.0, 0.0, 0.0};
    if (P.region[c] == 1) {
      const int i = c / n_mu, j = c - i * n_mu;
      const double uc = P.x[c], dRc = dRdu_of(c);
      d = 0.0;
      for (int q = 0; q < 4; ++q) {
        const int ib = i + di[q], jb = j + dj[q];
        if (!in_grid(ib, jb, n_r, n_mu)) continue;
        const int cb = ib * n_mu + jb;
        if (!(a.rho[cb] > 0.0)) continue;
        const double af = lin_cond(a, i, j, ib, jb, P.p1[c], P.p1[cb], nullptr);
        const double dadR = -af / (P.p1[c] + P.p1[cb]);
        const double ub = u_of(cb);
        d += af + dadR * dRc * (uc - ub);
        // row cb's coupling to column c, J_{cb,c} (cb in the region)
        if (P.region[cb] == 1) cq[q] = -af + dadR * dRc * (ub - uc);
      }
    }
    jd[c] = d;
    for (int q = 0; q < 4; ++q) in0[(size_t)q * nc + c] = cq[q];
  }
  __syncthreads();
  // theta-line factors (Thomas algorithm, no pivoting: the blocks are
  // diagonally dominant); cells outside the region are identity rows
  const bool lines = a.precond == 1;
  if (lines) {
    for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
      double cprev = 0.0;
      for (int j = 0; j < n_mu; ++j) {
        const int c = i * n_mu + j;
        if (P.region[c] != 1) {
          cp[c] = 0.0;
          dinv[c] = 1.0;
          cprev = 0.0;
          continue;
        }
        const double sub = j > 0 ? in0[2 * (size_t)nc + c] : 0.0;
        const double sup = j + 1 < n_mu ? in0[3 * (size_t)nc + c] : 0.0;
        const double den = jd[c] - sub * cprev;
        dinv[c] = 1.0 / den;
        cp[c] = sup * dinv[c];
        cprev = cp[c];
      }
    }
    __syncthreads();
  }
  // M^-1 x into out (all region cells; a barrier follows in the caller)
  auto precond = [&](const double* x, double* out) {
    if (!lines) {
      for (int c = threadIdx.x; c < nc; c += blockDim.x)
        if (P.region[c] == 1) out[c] = x[c] / jd[c];
      return;
    }
    for (int i = threadIdx.x; i < n_r; i += blockDim.x) {
      double prev = 0.0;
      for (int j = 0; j < n_mu; ++j) {
        const int c = i * n_mu + j;
        if (P.region[c] != 1) {
          out[c] = 0.0;
          prev = 0.0;
          continue;
        }
        const double sub = j > 0 ? in0[2 * (size_t)nc + c] : 0.0;
        prev = (x[c] - sub * prev) * dinv[c];
        out[c] = prev;
      }
      for (int j = n_mu - 2; j >= 0; --j) {
        const int c = i * n_mu + j;
        if (P.region[c] == 1) out[c] -= cp[c] * out[c + 1];
      }
    }
  };
  auto applyT = [&](const double* x, int c) -> double {  // (J^T x)_c, c in the region
    const int i = c / n_mu, j = c - i * n_mu;
    double acc = jd[c] * x[c];
    for (int q = 0; q < 4; ++q) {
      const int ib = i + di[q], jb = j + dj[q];
      if (!in_grid(ib, jb, n_r, n_mu)) continue;
      const int cb = ib * n_mu + jb;
      if (P.region[cb] == 1) acc += in0[(size_t)q * nc + c] * x[cb];
    }
    return acc;
  };
  // right-hand side dJ/du, and BiCGSTAB from lambda = 0
  double bb = 0.0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) {
    double g = 0.0;
    if (P.region[c] == 1) {
      const double u = P.x[c];
      g = u > 0.0 ? a.dJdT[c] * sqrt(sqrt(u)) / (4.0 * u) : 0.0;
    }
    lam[c] = 0.0;
    r[c] = g;
    rh[c] = g;
    p[c] = 0.0;
    v[c] = 0.0;
    bb += g * g;
  }
  bb = wg_reduce<false>(bb, red);
  double rho_old = 1.0, alpha = 1.0, omega = 1.0, rr = bb;
  int it = 0;
  while (bb > 0.0 && rr > a.cg_tol2 * bb && it < a.cg_max_iter) {
    double rho = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
      if (P.region[c] == 1) rho += rh[c] * r[c];
    rho = wg_reduce<false>(rho, red);
    if (rho == 0.0) break;  // breakdown: stop with the iterate reached
    const double beta = (rho / rho_old) * (alpha / omega);
    for (int c = threadIdx.x; c < nc; c += blockDim.x)
      if (P.region[c] == 1) p[c] = r[c] + beta * (p[c] - omega * v[c]);
    __syncthreads();
    precond(p, y);
    __syncthreads();
    double rv = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      v[c] = applyT(y, c);
      rv += rh[c] * v[c];
    }
    rv = wg_reduce<false>(rv, red);
    alpha = rv != 0.0 ? rho / rv : 0.0;
    double ss = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      sv[c] = r[c] - alpha * v[c];
      ss += sv[c] * sv[c];
    }
    ss = wg_reduce<false>(ss, red);   // (its barrier also orders sv for the sweep)
    precond(sv, z);
    __syncthreads();
    ++it;
    if (ss <= a.cg_tol2 * bb) {
      for (int c = threadIdx.x; c < nc; c += blockDim.x)
        if (P.region[c] == 1) lam[c] += alpha * y[c];
      rr = ss;
      break;
    }
    double ts = 0.0, tt = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      t[c] = applyT(z, c);
      ts += t[c] * sv[c];
      tt += t[c] * t[c];
    }
    ts = wg_reduce<false>(ts, red);
    tt = wg_reduce<false>(tt, red);
    omega = tt > 0.0 ? ts / tt : 0.0;
    double rn = 0.0;
    for (int c = threadIdx.x; c < nc; c += blockDim.x) {
      if (P.region[c] != 1) continue;
      lam[c] += alpha * y[c] + omega * z[c];
      r[c] = sv[c] - omega * t[c];
      rn += r[c] * r[c];
    }
    rr = wg_reduce<false>(rn, red);
    rho_old = rho;
    if (omega == 0.0) break;
  }
  __syncthreads();
  grad_from_lambda(a, P, lam);
  if (threadIdx.x == 0 && a.stats) {
    mcrt_pda_stats s{};
    s.sweeps = 1;
    s.cg_iters_total = it;
    s.cg_iters_last = it;
    s.last_residual = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    s.converged = (bb == 0.0 || rr <= a.cg_tol2 * bb) ? 1 : 0;
    *a.stats = s;
  }
}

// Largest relative change of T over the region cells, into *out (as the
// bits of a non-negative double, so an integer maximum orders them).
__global__ void nl_change_kernel(const double* T_new, const double* T_old, const uint8_t* region,
                                 int nc, unsigned long long* out) {
  double m = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += gridDim.x * blockDim.x) {
    if (region[c] != 1) continue;
    const double ch = fabs(T_new[c] - T_old[c]) / fmax(T_new[c], 1e-300);
    m = fmax(m, ch);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

__global__ void nl_zero_kernel(unsigned long long* out) {
  if (threadIdx.x == 0) *out = 0ull;
}

}  // namespace

// The argument slot of the single-workgroup solve doubles as the slot of the
// linear/adjoint pair (both are synchronous).
// kind: 0 the linear solve, 1 its adjoint, 2 the adjoint of the nonlinear solve
static int pda_lin_call(mcrt_ctx* ctx, const PdaLinArgs& h, int kind, mcrt_pda_stats* st,
                        hipStream_t s) {
  static_assert(sizeof(PdaLinArgs) <= 4096, "argument slot");
  PdaWgArgs* d_args;
  mcrt_pda_stats* d_stats;
  pda_wg_slots(ctx, &d_args, &d_stats);
  PdaLinArgs hh = h;
  hh.stats = d_stats;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(ctx->d_lin_args, &hh, sizeof(hh), hipMemcpyHostToDevice) != hipSuccess) {
    set_error(ctx, "PDA argument upload failed");
    return MCRT_E_HIP;
  }
  if (kind == 2)
    hipLaunchKernelGGL(pda_nl_adjoint_kernel, dim3(1), dim3(WG), 0, s,
                       (const PdaLinArgs*)ctx->d_lin_args);
  else if (kind == 1)
    hipLaunchKernelGGL(pda_adjoint_kernel, dim3(1), dim3(WG), 0, s,
                       (const PdaLinArgs*)ctx->d_lin_args);
  else
    hipLaunchKernelGGL(pda_linear_kernel, dim3(1), dim3(WG), 0, s,
                       (const PdaLinArgs*)ctx->d_lin_args);
  mcrt_pda_stats out{};
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&out, d_stats, sizeof(out), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    set_error(ctx, "PDA linear/adjoint launch failed");
    return MCRT_E_HIP;
  }
  if (st) *st = out;
  return out.cg_iters_last >= ctx->opt.cg_max_iter ? MCRT_E_NOT_CONVERGED : MCRT_OK;
}

int pda_linear(mcrt_ctx* ctx, const uint8_t* mask, const double* rho, const double* kscale,
               const double* T_D, const double* T_bc, double* T_out, mcrt_pda_stats* st,
               hipStream_t s) {
  PdaArrays P;
  PdaGeom g;
  int rc = pda_alloc(ctx, P, g);
  if (rc) return rc;
  if (!ctx->d_lin_args && hipMalloc(&ctx->d_lin_args, sizeof(PdaLinArgs)) != hipSuccess) {
    set_error(ctx, "PDA argument slot");
    return MCRT_E_OOM;
  }
  PdaLinArgs h{};
  h.M = ctx->m;
  h.P = P;
  h.g = g;
  h.mask = mask;
  h.rho = rho ? rho : ctx->m.rho;
  h.kscale = kscale;
  h.T_D = T_D;
  h.T_bc = T_bc;
  h.T_out = T_out;
  h.reg_out = ctx->d_region;
  h.cg_max_iter = ctx->opt.cg_max_iter;
  h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
  h.precond = ctx->opt.pda_precond;
  ctx->lin_rho = h.rho;
  ctx->lin_ready = true;
  ctx->nl_ready = false;
  return pda_lin_call(ctx, h, 0, st, s);
}

int pda_adjoint(mcrt_ctx* ctx, const double* dJdT, double* g_logrho, double* g_kscale,
                mcrt_pda_stats* st, hipStream_t s) {
  if (!ctx->lin_ready) {
    set_error(ctx, "mcrt_pda_adjoint needs a preceding mcrt_pda_linear");
    return MCRT_E_ARG;
  }
  PdaArrays P;
  PdaGeom g;
  int rc = pda_alloc(ctx, P, g);
  if (rc) return rc;
  PdaLinArgs h{};
  h.M = ctx->m;
  h.P = P;
  h.g = g;
  h.rho = ctx->lin_rho;
  h.dJdT = dJdT;
  h.g_logrho = g_logrho;
  h.g_kscale = g_kscale;
  h.cg_max_iter = ctx->opt.cg_max_iter;
  h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
  h.precond = ctx->opt.pda_precond;
  return pda_lin_call(ctx, h, 1, st, s);
}

// The nonlinear PDA for differentiation: Picard sweeps of the linear solve,
// D from the T of the previous sweep (the first from T_bc), until the
// largest relative change of T falls below pda_tol or stalls below its
// square root (the rule of mcrt_pda_solve).  The last sweep's linear solve
// stays for the adjoint.
static int nl_scratch(mcrt_ctx* ctx) {
  if (ctx->d_nl) return MCRT_OK;
  const size_t bytes = (size_t)(NL_ARRAYS + 1) * ctx->n_cells * sizeof(double) + 256;
  if (hipMalloc(&ctx->d_nl, bytes) != hipSuccess) {
    ctx->d_nl = nullptr;
    set_error(ctx, "nonlinear PDA scratch allocation failed");
    return MCRT_E_OOM;
  }
  return MCRT_OK;
}

int pda_nonlinear(mcrt_ctx* ctx, const uint8_t* mask, const double* rho, const double* kscale,
                  const double* T_bc, double* T_out, mcrt_pda_stats* st, hipStream_t s) {
  int rc = nl_scratch(ctx);
  if (rc) return rc;
  const int nc = ctx->n_cells;
  double* T_cur = (double*)ctx->d_nl + (size_t)NL_ARRAYS * nc;
  unsigned long long* d_change = (unsigned long long*)(T_cur + nc);
  if (hipMemcpyAsync(T_cur, T_bc, (size_t)nc * sizeof(double), hipMemcpyDeviceToDevice, s) !=
      hipSuccess) {
    set_error(ctx, "nonlinear PDA: copy failed");
    return MCRT_E_HIP;
  }
  mcrt_pda_stats out{}, lst{};
  int status = MCRT_OK;
  double prev = INFINITY;
  const unsigned nb = (unsigned)std::min<size_t>(((size_t)nc + 255) / 256, 1024);
  for (int sweep = 1; sweep <= ctx->opt.pda_max_sweeps; ++sweep) {
    rc = pda_linear(ctx, mask, rho, kscale, T_cur, T_bc, T_out, &lst, s);
    if (rc != MCRT_OK && rc != MCRT_E_NOT_CONVERGED) return rc;
    if (rc == MCRT_E_NOT_CONVERGED) status = rc;
    out.cg_iters_total += lst.cg_iters_total;
    out.cg_iters_last = lst.cg_iters_last;
    out.last_residual = lst.last_residual;
    out.n_region = lst.n_region;
    out.n_isolated = lst.n_isolated;
    out.sweeps = sweep;
    hipLaunchKernelGGL(nl_zero_kernel, dim3(1), dim3(64), 0, s, d_change);
    hipLaunchKernelGGL(nl_change_kernel, dim3(nb), dim3(256), 0, s, (const double*)T_out,
                       (const double*)T_cur, (const uint8_t*)ctx->d_region, nc, d_change);
    unsigned long long bits = 0;
    if (hipMemcpyAsync(&bits, d_change, sizeof(bits), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(T_cur, T_out, (size_t)nc * sizeof(double), hipMemcpyDeviceToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      set_error(ctx, "nonlinear PDA sweep failed");
      return MCRT_E_HIP;
    }
    double change;
    std::memcpy(&change, &bits, sizeof(change));
    out.last_change = change;
    if (change < ctx->opt.pda_tol || (change < std::sqrt(ctx->opt.pda_tol) && change >= prev)) {
      out.converged = 1;
      break;
    }
    prev = change;
  }
  if (!out.converged && status == MCRT_OK) status = MCRT_E_NOT_CONVERGED;
  ctx->nl_ready = true;  // after pda_linear, which clears it
  if (st) *st = out;
  return status;
}

int pda_nl_adjoint(mcrt_ctx* ctx, const double* dJdT, double* g_logrho, double* g_kscale,
                   mcrt_pda_stats* st, hipStream_t s) {
  if (!ctx->lin_ready || !ctx->nl_ready || !ctx->d_nl) {
    set_error(ctx, "mcrt_pda_nonlinear_adjoint needs a preceding mcrt_pda_nonlinear");
    return MCRT_E_ARG;
  }
  PdaArrays P;
  PdaGeom g;
  int rc = pda_alloc(ctx, P, g);
  if (rc) return rc;
  PdaLinArgs h{};
  h.M = ctx->m;
  h.P = P;
  h.g = g;
  h.rho = ctx->lin_rho;
  h.dJdT = dJdT;
  h.g_logrho = g_logrho;
  h.g_kscale = g_kscale;
  h.nl = (double*)ctx->d_nl;
  h.cg_max_iter = ctx->opt.cg_max_iter;
  h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
  h.precond = ctx->opt.pda_precond;
  return pda_lin_call(ctx, h, 2, st, s);
}

// ---------------------------------------------------------------- batches
size_t pda_wg_args_size() { return sizeof(PdaWgArgs); }

// Host-side arguments of the single-workgroup PDA of each context (visits
// rule, in place on the context's T and region), statistics into each
// context's slot.
int pda_batch_fill(mcrt_ctx** ctxs, int n, void* host) {
  PdaWgArgs* out = (PdaWgArgs*)host;
  for (int d = 0; d < n; ++d) {
    mcrt_ctx* ctx = ctxs[d];
    PdaArrays P;
    PdaGeom g;
    int rc = pda_alloc(ctx, P, g);
    if (rc) return rc;
    PdaWgArgs& h = out[d];
    h.M = ctx->m;
    h.P = P;
    h.g = g;
    h.rule = region_rule(ctx, nullptr);
    h.fails = &ctx->d_health->pda_fails;
    h.T_mc = ctx->d_T;
    h.T_out = ctx->d_T;
    h.reg_out = ctx->d_region;
    h.max_sweeps = ctx->opt.pda_max_sweeps;
    h.tol = ctx->opt.pda_tol;
    h.cg_max_iter = ctx->opt.cg_max_iter;
    h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
    h.precond = ctx->opt.pda_precond;
    PdaWgArgs* da;
    mcrt_pda_stats* ds;
    pda_wg_slots(ctx, &da, &ds);
    h.stats = ds;
  }
  return MCRT_OK;
}

int pda_batch_launch(const void* d_args, int n, hipStream_t s) {
  hipLaunchKernelGGL(pda_wg_kernel, dim3(n), dim3(WG), 0, s, (const PdaWgArgs*)d_args);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

mcrt_pda_stats* pda_stats_slot(mcrt_ctx* ctx) {
  PdaWgArgs* da;
  mcrt_pda_stats* ds;
  pda_wg_slots(ctx, &da, &ds);
  return ds;
}

namespace {
__global__ void copy_kernel(double* dst, const double* src, size_t n) {
  size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; t < n; t += stride) dst[t] = src[t];
}
}  // namespace

int launch_copy(double* dst, const double* src, size_t n, hipStream_t s) {
  if (!n) return MCRT_OK;
  unsigned nb = (unsigned)((n + 255) / 256);
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(copy_kernel, dim3(nb), dim3(256), 0, s, dst, src, n);
  return hipGetLastError() == hipSuccess ? MCRT_OK : MCRT_E_HIP;
}

}  // namespace mcrt

// ------------------------------------------------------------------------
// The PDA solve without allocation, for callers that cannot allocate device
// memory.  Its work arrays live in one file-scope device array: the region
// and contact flags, the thirteen FP64 work vectors of the single-workgroup
// solver, the cell-centre geometry and the statistics slot, for up to
// MCRT_NOALLOC_MAX_CELLS cells.  Each device holds its own copy; its address
// is looked up once per device.  Calls on one device share it, so calls that
// overlap in time on one device race.
// ------------------------------------------------------------------------
namespace {
constexpr size_t NA_CELLS = MCRT_NOALLOC_MAX_CELLS;
constexpr size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }
// flags 2 x u8, 13 work vectors, geometry (rc [n_r], thc [n_mu], Ar, Amu: each
// at most NA_CELLS doubles), statistics
constexpr size_t NA_BYTES = 2 * al256(NA_CELLS) + 13 * al256(NA_CELLS * 8) +
                            4 * al256(NA_CELLS * 8) + al256(sizeof(mcrt_pda_stats));

__device__ __align__(256) unsigned char scratch[NA_BYTES];

std::mutex na_mutex;
void* na_ptr[64] = {};

// address of this device's scratch array (looked up once per device, with the
// device current)
int na_scratch(int device, void** out) {
  if (device < 0 || device >= 64) return MCRT_E_ARG;
  std::lock_guard<std::mutex> lk(na_mutex);
  if (!na_ptr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MCRT_E_HIP;
    na_ptr[device] = p;
  }
  *out = na_ptr[device];
  return MCRT_OK;
}

}  // namespace

extern "C" int mcrt_pda_solve_noalloc(mcrt_ctx* ctx, const uint8_t* mask_dev,
                                      mcrt_pda_stats* stats, hipStream_t stream) {
  using namespace mcrt;
  if (!ctx) {
    set_error(nullptr, "null context");
    return MCRT_E_ARG;
  }
  if ((size_t)ctx->n_cells > NA_CELLS) {
    set_error(ctx, "mcrt_pda_solve_noalloc: " + std::to_string(ctx->n_cells) +
                       " cells exceed its fixed scratch of " + std::to_string(NA_CELLS));
    return MCRT_E_ARG;
  }
  if (!mask_dev && ctx->opt.pda_visits <= 0 && !(ctx->opt.pda_sigma > 0.0)) {
    set_error(ctx, "no PDA mask, pda_visits <= 0 and pda_sigma = 0");
    return MCRT_E_ARG;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
    set_error(ctx, "mcrt_pda_solve_noalloc: the context's device is not the current device");
    return MCRT_E_ARG;
  }
  void* base = nullptr;
  int rc = na_scratch(ctx->device, &base);
  if (rc) {
    set_error(ctx, "mcrt_pda_solve_noalloc: scratch address lookup failed");
    return rc;
  }
  const size_t nc = (size_t)ctx->n_cells;
  char* q = (char*)base;
  PdaWgArgs h;
  h.M = ctx->m;
  PdaArrays& P = h.P;
  P.sc = nullptr;  // scalars of the grid-wide solver: unused here
  P.region = (uint8_t*)q;
  q += al256(nc);
  P.touch = (uint8_t*)q;
  q += al256(nc);
  double** arr[13] = {&P.Tw, &P.Tbc, &P.diag, &P.aE, &P.aN, &P.b, &P.x, &P.r, &P.p0, &P.p1, &P.q,
                      &P.z, &P.lm};
  for (auto a : arr) {
    *a = (double*)q;
    q += al256(nc * 8);
  }
  double* rc_ = (double*)q;
  q += al256(nc * 8);
  double* thc = (double*)q;
  q += al256(nc * 8);
  double* Ar = (double*)q;
  q += al256(nc * 8);
  double* Amu = (double*)q;
  q += al256(nc * 8);
  mcrt_pda_stats* d_stats = (mcrt_pda_stats*)q;
  h.g.rc = rc_;
  h.g.thc = thc;
  h.g.Ar = Ar;
  h.g.Amu = Amu;
  h.g.kscale = nullptr;
  h.rule = region_rule(ctx, mask_dev);
  h.T_mc = ctx->d_T;
  h.T_out = ctx->d_T;
  h.reg_out = ctx->d_region;
  h.max_sweeps = ctx->opt.pda_max_sweeps;
  h.tol = ctx->opt.pda_tol;
  h.cg_max_iter = ctx->opt.cg_max_iter;
  h.cg_tol2 = ctx->opt.cg_tol * ctx->opt.cg_tol;
  h.precond = ctx->opt.pda_precond;
  h.stats = d_stats;
  h.fails = nullptr;
  const unsigned nb = (unsigned)std::min<size_t>((nc + 255) / 256, 1024);
  hipLaunchKernelGGL(pda_geom_kernel, dim3(nb), dim3(256), 0, stream, ctx->m, rc_, thc, Ar, Amu);
  hipLaunchKernelGGL(pda_wg_kernel_val, dim3(1), dim3(WG), 0, stream, h);
  if (hipGetLastError() != hipSuccess) {
    set_error(ctx, "mcrt_pda_solve_noalloc: launch failed");
    return MCRT_E_HIP;
  }
  mcrt_pda_stats out{};
  if (hipMemcpyAsync(&out, d_stats, sizeof(out), hipMemcpyDeviceToHost, stream) != hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess) {
    set_error(ctx, "mcrt_pda_solve_noalloc: solve failed");
    return MCRT_E_HIP;
  }
  if (stats) *stats = out;
  if (out.cg_iters_last >= ctx->opt.cg_max_iter || !out.converged) return MCRT_E_NOT_CONVERGED;
  return out.n_isolated > 0 ? MCRT_E_SINGULAR_REGION : MCRT_OK;
}
