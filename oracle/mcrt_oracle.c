/*
 * CPU oracle: Monte Carlo radiative transfer with immediate reemission, the
 * modified random walk and the partial diffusion approximation, after
 * Min et al. (2009).  Plain, single-threaded FP64.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU-baseline timing).  It
 * shares no code with the HIP library.
 *
 * Where the paper is silent the readings used are stated at each step; the
 * same readings bind the GPU path, which implements them independently.
 */
#include "mcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018, cgs */
static const double H_PLANCK = 6.62607015e-27;
static const double K_BOLTZ = 1.380649e-16;
static const double C_LIGHT = 2.99792458e10;
static const double SIGMA_SB = 5.670374419e-5;
static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, Salmon, Moraes, Dror & Shaw (SC'11): ten rounds of two      */
/* 32x32->64 multiplies with a Weyl-sequence key schedule.                    */
/* ------------------------------------------------------------------------ */
void ora_philox4x32_10(uint32_t ctr[4], const uint32_t key_in[2]) {
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)ctr[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)ctr[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ ctr[1] ^ k0;
    uint32_t n2 = hi0 ^ ctr[3] ^ k1;
    ctr[0] = n0;
    ctr[1] = lo1;
    ctr[2] = n2;
    ctr[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

/* One packet's stream: draw d uses counter (pid_lo, pid_hi, d/2, 0) and the
 * 64-bit word (out[2h] << 32 | out[2h+1]) with h = d % 2; its top 52 bits x
 * give (x + 1/2) / 2^52, a double strictly inside (0, 1). */
typedef struct {
  uint32_t key[2];
  uint64_t pid;
  uint64_t d;
  uint32_t buf[4];
} rng_t;

static double u64_to_unit(uint32_t a, uint32_t b) {
  uint64_t x = ((uint64_t)a << 32) | (uint64_t)b;
  return ((double)(x >> 12) + 0.5) * (1.0 / 4503599627370496.0);
}

static double rng_next(rng_t* r) {
  uint64_t h = r->d & 1u;
  if (h == 0) {
    uint64_t blk = r->d >> 1;
    r->buf[0] = (uint32_t)r->pid;
    r->buf[1] = (uint32_t)(r->pid >> 32);
    r->buf[2] = (uint32_t)blk;
    r->buf[3] = (uint32_t)(blk >> 32);
    ora_philox4x32_10(r->buf, r->key);
  }
  r->d++;
  return u64_to_unit(r->buf[2 * h], r->buf[2 * h + 1]);
}

static void rng_init(rng_t* r, uint64_t seed, uint64_t pid) {
  r->key[0] = (uint32_t)seed;
  r->key[1] = (uint32_t)(seed >> 32);
  r->pid = pid;
  r->d = 0;
}

void ora_uniforms(uint64_t seed, uint64_t pid, uint64_t d0, int64_t n, double* out) {
  rng_t r;
  rng_init(&r, seed, pid);
  for (uint64_t i = 0; i < d0; ++i) rng_next(&r);
  for (int64_t i = 0; i < n; ++i) out[i] = rng_next(&r);
}

/* ------------------------------------------------------------------------ */
/* Planck bin integrals by composite Simpson in u = ln(nu)                    */
/* ------------------------------------------------------------------------ */
static void planck_point(double nu, double T, double* B, double* dB) {
  double pre = 2.0 * H_PLANCK * nu * nu * nu / (C_LIGHT * C_LIGHT);
  if (T <= 0.0) {
    *B = 0.0;
    *dB = 0.0;
    return;
  }
  double x = H_PLANCK * nu / (K_BOLTZ * T);
  double ex = exp(-x);
  double om = -expm1(-x); /* 1 - e^-x */
  *B = pre * ex / om;
  *dB = pre * (x / T) * ex / (om * om);
}

void ora_planck_bins(const double* lambda_edges, int n_lambda, double T, double* Bbar,
                     double* dBbar) {
  const int M = 256; /* Simpson sub-intervals per bin */
  for (int k = 0; k < n_lambda; ++k) {
    double nu_lo = C_LIGHT / lambda_edges[k + 1];
    double nu_hi = C_LIGHT / lambda_edges[k];
    double ua = log(nu_lo), ub = log(nu_hi), hstep = (ub - ua) / M;
    double sB = 0.0, sdB = 0.0;
    for (int q = 0; q <= M; ++q) {
      double u = ua + q * hstep;
      double nu = exp(u), B, dB;
      planck_point(nu, T, &B, &dB);
      double w = (q == 0 || q == M) ? 1.0 : ((q & 1) ? 4.0 : 2.0);
      sB += w * B * nu; /* dnu = nu du */
      sdB += w * dB * nu;
    }
    Bbar[k] = sB * hstep / 3.0;
    dBbar[k] = sdB * hstep / 3.0;
  }
}

/* ------------------------------------------------------------------------ */
/* Tables (Sect. 2.2.3).  Temperature-dependent quantities are tabulated at   */
/* n_T nodes: node 0 is T = 0, nodes 1..n_T-1 are log-spaced T_lo..T_hi, and  */
/* values are interpolated linearly in T between nodes (reading).  Frequency  */
/* integrals are sums over the wavelength bins (reading).                     */
/* ------------------------------------------------------------------------ */
/* eq:eta nu iter at one temperature, from eta = kappa dB/dT: eta_k <-
 * kappa_k dB_k (sum eta kappa/chi)/(sum eta) + (sigma_k/chi_k) eta_k until the
 * largest relative change is below 1e-13.  Anisotropic scattering enters the
 * diffusion quantities through the isotropic equivalent sigma' = (1 - g) sigma
 * (Sect. 2.2.3).  dBb [n_lambda] the bin integrals of dB/dT; eta_new scratch.
 * Returns the iterations taken. */
static int eta_iterate(const ora_model* m, const double* dBb, double* eta, double* eta_new) {
  const int nl = m->n_lambda;
  const double sim = 1.0 - m->g_asym;
  for (int k = 0; k < nl; ++k) eta[k] = m->kappa_abs[k] * dBb[k];
  int it;
  for (it = 0; it < 20000; ++it) {
    double num = 0.0, den = 0.0;
    for (int k = 0; k < nl; ++k) {
      double chi = m->kappa_abs[k] + m->kappa_sca[k] * sim;
      num += eta[k] * m->kappa_abs[k] / chi;
      den += eta[k];
    }
    double ratio = num / den, change = 0.0;
    for (int k = 0; k < nl; ++k) {
      double sca = m->kappa_sca[k] * sim;
      double chi = m->kappa_abs[k] + sca;
      eta_new[k] = m->kappa_abs[k] * dBb[k] * ratio + (sca / chi) * eta[k];
      double rel = fabs(eta_new[k] - eta[k]) / (fabs(eta_new[k]) + 1e-300);
      if (eta_new[k] != 0.0 && rel > change) change = rel;
    }
    memcpy(eta, eta_new, sizeof(double) * nl);
    if (change < 1e-13) break;
  }
  return it + 1;
}

int ora_build_tables(const ora_model* m, ora_tables* t) {
  const int nl = m->n_lambda, nT = t->n_T;
  if (nT < 3 || nl < 1) return -1;
  double* Bb = (double*)malloc(sizeof(double) * nl);
  double* dBb = (double*)malloc(sizeof(double) * nl);
  double* eta = (double*)malloc(sizeof(double) * nl);
  double* eta_new = (double*)malloc(sizeof(double) * nl);
  t->eta_iters_max = 0;
  double lr = log(t->T_hi / t->T_lo);
  for (int n = 0; n < nT; ++n) {
    double T = (n == 0) ? 0.0 : t->T_lo * exp(lr * (double)(n - 1) / (double)(nT - 2));
    if (n == nT - 1) T = t->T_hi;
    if (n == 1) T = t->T_lo;
    t->T[n] = T;
    ora_planck_bins(m->lambda_edges, nl, T, Bb, dBb);
    double c = 0.0;
    for (int k = 0; k < nl; ++k) {
      c += m->kappa_abs[k] * Bb[k];
      t->cdf[(size_t)n * nl + k] = c;
    }
    if (n == 0) continue;
    const double sim = 1.0 - m->g_asym;
    int its = eta_iterate(m, dBb, eta, eta_new);
    if (its > t->eta_iters_max) t->eta_iters_max = its;
    /* eq:avd, eq:avd2 (per unit rho), eq:diffusion coeff, kappa-bar */
    double s_eta = 0.0, s_d = 0.0, s_d2 = 0.0, s_kc = 0.0, s_ic = 0.0;
    for (int k = 0; k < nl; ++k) {
      double chi = m->kappa_abs[k] + m->kappa_sca[k] * sim;
      s_eta += eta[k];
      s_d += eta[k] / chi;
      s_d2 += eta[k] / (chi * chi);
      s_kc += eta[k] * m->kappa_abs[k] / chi;
      s_ic += eta[k] / chi;
    }
    double d1 = s_d / s_eta;        /* <d> * rho */
    double d2 = 2.0 * s_d2 / s_eta; /* <d^2> * rho^2 */
    t->Drho[n] = d2 / (6.0 * d1);
    t->kbar[n] = s_kc / s_ic;
  }
  /* below T_lo: the T_lo values (the limit T -> 0 is not needed) */
  t->Drho[0] = t->Drho[1];
  t->kbar[0] = t->kbar[1];
  /* star: L = 4 pi R^2 sigma T^4; spectrum restricted to the bins, renormalised */
  ora_planck_bins(m->lambda_edges, nl, m->T_star, Bb, dBb);
  double tot = 0.0;
  for (int k = 0; k < nl; ++k) tot += Bb[k];
  double c = 0.0;
  for (int k = 0; k < nl; ++k) {
    c += Bb[k];
    t->star_cdf[k] = c / tot;
  }
  t->star_cdf[nl - 1] = 1.0;
  t->L_star = 4.0 * PI * m->R_star * m->R_star * SIGMA_SB * pow(m->T_star, 4.0);
  free(Bb);
  free(dBb);
  free(eta);
  free(eta_new);
  return 0;
}

/* linear-in-T position of T among the nodes: segment n and weight f */
static void t_segment(const ora_tables* t, double T, int* n, double* f) {
  int lo = 0, hi = t->n_T - 1; /* invariant T[lo] <= T < T[hi] unless beyond */
  if (T >= t->T[t->n_T - 1]) {
    *n = t->n_T - 2;
  } else {
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (t->T[mid] <= T) lo = mid; else hi = mid;
    }
    *n = lo;
  }
  *f = (T - t->T[*n]) / (t->T[*n + 1] - t->T[*n]);
}

static double t_interp(const ora_tables* t, const double* tab, double T) {
  int n;
  double f;
  t_segment(t, T, &n, &f);
  return tab[n] + f * (tab[n + 1] - tab[n]);
}

/* G(T) = cdf at the last bin; the cell emits 4 pi m G(T) */
static double G_node(const ora_tables* t, int nl, int n) { return t->cdf[(size_t)n * nl + nl - 1]; }

/* radiative equilibrium: 4 pi m G(T) = E, G piecewise linear in T */
static double T_of_g(const ora_tables* t, int nl, double g) {
  if (g <= 0.0) return 0.0;
  int lo = 0, hi = t->n_T - 1, n;
  if (g >= G_node(t, nl, hi)) {
    n = t->n_T - 2;
  } else {
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (G_node(t, nl, mid) <= g) lo = mid; else hi = mid;
    }
    n = lo;
  }
  double Ga = G_node(t, nl, n), Gb = G_node(t, nl, n + 1);
  return t->T[n] + (g - Ga) / (Gb - Ga) * (t->T[n + 1] - t->T[n]);
}

double ora_T_of_E(const ora_model* m, const ora_tables* t, double E, double mass) {
  if (mass <= 0.0) return 0.0;
  return T_of_g(t, m->n_lambda, E / (4.0 * PI * mass));
}

/* Cumulative emission at T of bins 0..k, linear in T between nodes */
static double cdf_at(const ora_tables* t, int nl, int n, double f, int k) {
  double a = t->cdf[(size_t)n * nl + k], b = t->cdf[(size_t)(n + 1) * nl + k];
  return a + f * (b - a);
}

/* Reemission bin (immediate reemission): from the difference spectrum
 * kappa_k [Bbar_k(T_new) - Bbar_k(T_old)], or the full spectrum at T_new when
 * there is no old temperature (T_old < 0) or no difference. */
static int reemit_bin(const ora_tables* t, int nl, double T_old, double T_new, double xi) {
  int nn, no = 0;
  double fn, fo = 0.0;
  t_segment(t, T_new, &nn, &fn);
  int use_diff = (T_old >= 0.0 && T_new > T_old);
  if (use_diff) t_segment(t, T_old, &no, &fo);
  /* D(k): difference of the cumulative spectra; same-segment case factored */
  double tot;
  int same = use_diff && (no == nn);
  if (same) {
    tot = (fn - fo) * (t->cdf[(size_t)(nn + 1) * nl + nl - 1] - t->cdf[(size_t)nn * nl + nl - 1]);
  } else if (use_diff) {
    tot = cdf_at(t, nl, nn, fn, nl - 1) - cdf_at(t, nl, no, fo, nl - 1);
  } else {
    tot = cdf_at(t, nl, nn, fn, nl - 1);
  }
  if (!(tot > 0.0)) { /* degenerate difference: full spectrum at T_new */
    use_diff = 0;
    same = 0;
    tot = cdf_at(t, nl, nn, fn, nl - 1);
  }
  double target = xi * tot;
  int lo = 0, hi = nl - 1; /* smallest k with D(k) > target */
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    double Dk;
    if (same)
      Dk = (fn - fo) * (t->cdf[(size_t)(nn + 1) * nl + mid] - t->cdf[(size_t)nn * nl + mid]);
    else if (use_diff)
      Dk = cdf_at(t, nl, nn, fn, mid) - cdf_at(t, nl, no, fo, mid);
    else
      Dk = cdf_at(t, nl, nn, fn, mid);
    if (Dk > target) hi = mid; else lo = mid + 1;
  }
  return lo;
}

int ora_reemit_sample(const ora_model* m, const ora_tables* t, double T_old, double T_new,
                      double xi) {
  return reemit_bin(t, m->n_lambda, T_old, T_new, xi);
}

double ora_table_interp(const ora_tables* t, int which, double T) {
  return t_interp(t, which == 0 ? t->Drho : t->kbar, T);
}

/* ------------------------------------------------------------------------ */
/* MRW escape-time law (eq:probability RW).  With s = D c t / R0^2,           */
/* P(s) = 2 sum_{n>=1} (-1)^{n+1} exp(-n^2 pi^2 s); for small s the           */
/* equivalent theta-function form 1 - 2 sqrt(pi/x) sum_k exp(-pi^2 (2k+1)^2   */
/* / (4x)), x = pi^2 s, converges fast.  P decreases from 1 to 0.             */
/* ------------------------------------------------------------------------ */
double ora_mrw_survival(double s) {
  if (s <= 0.0) return 1.0;
  double x = PI * PI * s;
  if (s >= 0.1) {
    double sum = 0.0;
    for (int n = 1; n < 200; ++n) {
      double term = exp(-(double)n * n * x);
      sum += (n & 1) ? term : -term;
      if (term < 1e-300 || term < 1e-18 * fabs(sum)) break;
    }
    return 2.0 * sum;
  }
  double sum = 0.0;
  for (int k = 0; k < 200; ++k) {
    double a = (double)(2 * k + 1);
    double term = exp(-PI * PI * a * a / (4.0 * x));
    sum += term;
    if (term < 1e-300 || term < 1e-18 * sum) break;
  }
  return 1.0 - 2.0 * sqrt(PI / x) * sum;
}

/* P(s) = P0 by bisection on log s (P is strictly decreasing) */
double ora_mrw_escape_s(double P0) {
  double lo = 1e-6, hi = 10.0;
  while (ora_mrw_survival(lo) < P0) lo *= 0.5;
  while (ora_mrw_survival(hi) > P0) hi *= 2.0;
  for (int it = 0; it < 200; ++it) {
    double mid = sqrt(lo * hi);
    if (ora_mrw_survival(mid) > P0) lo = mid; else hi = mid;
    if (hi - lo <= 1e-16 * hi) break;
  }
  return 0.5 * (lo + hi);
}

/* Energy one MRW step deposits in cell c, per unit packet energy: the
 * packet travels c t = s R0^2 / D inside the sphere (s from eq. probability
 * RW, D = 1/(rho chi_R) / 3 from the table at Tc, Sect. 2.2.3) and is absorbed
 * along that path at the rate rho kappa-bar(Tc) per unit length. */
double ora_mrw_deposit(const ora_model* m, const ora_tables* t, int64_t c, double Tc, double R0,
                       double s) {
  double D = t_interp(t, t->Drho, Tc) / m->rho[c];
  double ell = s * R0 * R0 / D; /* c t */
  return m->rho[c] * t_interp(t, t->kbar, Tc) * ell;
}

/* ------------------------------------------------------------------------ */
/* Geometry: folded spherical grid.  Cell (i, j) is r_i <= r < r_{i+1} and    */
/* mu_j <= |z|/r < mu_{j+1}; both mirror halves belong to the cell.  Faces:   */
/* spheres r_i, r_{i+1}; cones mu_j (j >= 1) and mu_{j+1} (j+1 < n_mu).  The   */
/* midplane and the pole are not faces.                                       */
/* ------------------------------------------------------------------------ */
int64_t ora_locate(const ora_model* m, double x, double y, double z) {
  double r2 = (x * x + y * y) + z * z;
  double z2 = z * z;
  if (!(r2 >= m->r_edges[0] * m->r_edges[0])) return -1;
  if (!(r2 < m->r_edges[m->n_r] * m->r_edges[m->n_r])) return -1;
  int i = 0;
  for (int e = 1; e < m->n_r; ++e)
    if (m->r_edges[e] * m->r_edges[e] <= r2) i = e;
  int j = 0;
  for (int e = 1; e < m->n_mu; ++e)
    if ((m->mu_edges[e] * m->mu_edges[e]) * r2 <= z2) j = e;
  return (int64_t)i * m->n_mu + j;
}

/* path length to a sphere of squared radius R2, leaving it from inside */
static int sphere_out(double pd, double c, double* s) {
  double disc = pd * pd - c;
  if (c >= 0.0 && (pd > 0.0 || disc < 0.0)) { *s = 0.0; return 1; }
  if (disc < 0.0) disc = 0.0;
  double sq = sqrt(disc);
  *s = (pd > 0.0) ? -c / (pd + sq) : -pd + sq;
  return 1;
}

/* path length to a sphere of squared radius R2, reached from outside */
static int sphere_in(double pd, double c, double* s) {
  if (c <= 0.0 && pd < 0.0) { *s = 0.0; return 1; }
  if (pd >= 0.0) return 0;
  double disc = pd * pd - c;
  if (disc < 0.0) return 0;
  *s = c / (-pd + sqrt(disc));
  return 1;
}

/* path length to leave the cone pair |z| = mu r.  f(s) = A s^2 + 2 B s + C
 * with f < 0 inside the midplane-side wedge.  upper = 1: the cell lies on the
 * wedge side (f < 0) and leaves when f turns positive; upper = 0: the cell
 * lies on the pole side and leaves when f turns negative. */
static int cone_exit(double A, double B, double C, int upper, double* s) {
  if (upper) {
    if (C >= 0.0 && B > 0.0) { *s = 0.0; return 1; }
  } else {
    if (C <= 0.0 && B < 0.0) { *s = 0.0; return 1; }
  }
  double disc = B * B - A * C;
  if (disc < 0.0) return 0;
  double sq = sqrt(disc);
  double v;
  if (upper)
    v = (B > 0.0) ? C / (-B - sq) : (-B + sq) / A;
  else
    v = (B < 0.0) ? C / (-B + sq) : (-B - sq) / A;
  if (!(v > 0.0) || isinf(v)) return 0;
  *s = v;
  return 1;
}

/* face ids: 0 inner sphere, 1 outer sphere, 2 lower cone, 3 upper cone */
static double face_distance(const ora_model* m, int i, int j, const double p[3],
                            const double d[3], int* face) {
  double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
  double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
  double best = INFINITY, s;
  *face = -1;
  double ro = m->r_edges[i + 1];
  if (sphere_out(pd, rr - ro * ro, &s) && s < best) { best = s; *face = 1; }
  double ri = m->r_edges[i];
  if (sphere_in(pd, rr - ri * ri, &s) && s < best) { best = s; *face = 0; }
  if (j >= 1) {
    double mu = m->mu_edges[j], m2 = mu * mu;
    double A = d[2] * d[2] - m2 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double B = p[2] * d[2] - m2 * pd;
    double C = p[2] * p[2] - m2 * rr;
    if (cone_exit(A, B, C, 0, &s) && s < best) { best = s; *face = 2; }
  }
  if (j + 1 < m->n_mu) {
    double mu = m->mu_edges[j + 1], m2 = mu * mu;
    double A = d[2] * d[2] - m2 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double B = p[2] * d[2] - m2 * pd;
    double C = p[2] * p[2] - m2 * rr;
    if (cone_exit(A, B, C, 1, &s) && s < best) { best = s; *face = 3; }
  }
  return best;
}

/* distance from p to the nearest of the cell's bounding surfaces (spheres
 * and full cones; a lower bound of the distance to the cell boundary) */
static double min_face_distance(const ora_model* m, int i, int j, const double p[3]) {
  double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  double d = r - m->r_edges[i];
  double d2 = m->r_edges[i + 1] - r;
  if (d2 < d) d = d2;
  double mu = fabs(p[2]) / r;
  double smu = sqrt(fmax(0.0, 1.0 - mu * mu));
  if (j >= 1) { /* r sin(theta_j - theta) */
    double me = m->mu_edges[j];
    double v = r * (sqrt(1.0 - me * me) * mu - me * smu);
    if (v < d) d = v;
  }
  if (j + 1 < m->n_mu) { /* r sin(theta - theta_{j+1}) */
    double me = m->mu_edges[j + 1];
    double v = r * (me * smu - sqrt(1.0 - me * me) * mu);
    if (v < d) d = v;
  }
  return d > 0.0 ? d : 0.0;
}

static void iso_dir(rng_t* r, double d[3]) {
  double w = 2.0 * rng_next(r) - 1.0;
  double ph = 2.0 * PI * rng_next(r);
  double st = sqrt(fmax(0.0, 1.0 - w * w));
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = w;
}

/* New direction after a scattering with asymmetry parameter g, from two
 * draws.  g = 0: isotropic, as iso_dir.  Otherwise the cosine of the
 * scattering angle follows the Henyey-Greenstein phase function, from the
 * inverse of its cumulative distribution, and the azimuth is uniform; the
 * new direction is that rotation of d. */
static void scatter_dir_u(double g, double u1, double u2, double d[3]) {
  double ph = 2.0 * PI * u2;
  if (g == 0.0) {
    double w = 2.0 * u1 - 1.0, st = sqrt(fmax(0.0, 1.0 - w * w));
    d[0] = st * cos(ph);
    d[1] = st * sin(ph);
    d[2] = w;
    return;
  }
  double q = (1.0 - g * g) / (1.0 - g + 2.0 * g * u1);
  double mu = (1.0 + g * g - q * q) / (2.0 * g);
  mu = fmin(1.0, fmax(-1.0, mu));
  double st = sqrt(fmax(0.0, 1.0 - mu * mu));
  double cp = cos(ph), sp = sin(ph);
  double x = d[0], y = d[1], z = d[2];
  double s = sqrt(x * x + y * y); /* sin of the polar angle of d */
  if (s == 0.0) {
    d[0] = st * cp;
    d[1] = st * sp;
    d[2] = z > 0.0 ? mu : -mu;
  } else {
    d[0] = st * (x * z * cp - y * sp) / s + x * mu;
    d[1] = st * (y * z * cp + x * sp) / s + y * mu;
    d[2] = -st * cp * s + z * mu;
  }
}

static void scatter_dir(rng_t* r, double g, double d[3]) {
  double u1 = rng_next(r);
  double u2 = rng_next(r);
  scatter_dir_u(g, u1, u2, d);
}

void ora_scatter_dirs(double g, const double* u, const double* din, double* dout, int n) {
  for (int a = 0; a < n; ++a) {
    double d[3] = {din[3 * a], din[3 * a + 1], din[3 * a + 2]};
    scatter_dir_u(g, u[2 * a], u[2 * a + 1], d);
    dout[3 * a] = d[0];
    dout[3 * a + 1] = d[1];
    dout[3 * a + 2] = d[2];
  }
}

void ora_cell_volumes(const ora_model* m, double* V) {
  for (int i = 0; i < m->n_r; ++i) {
    double a = m->r_edges[i], b = m->r_edges[i + 1];
    double dr3 = b * b * b - a * a * a;
    for (int j = 0; j < m->n_mu; ++j)
      V[(size_t)i * m->n_mu + j] = 4.0 * PI / 3.0 * dr3 * (m->mu_edges[j + 1] - m->mu_edges[j]);
  }
}

/* Optical width of cell c at its most opaque wavelength: rho chi_max l with
 * l the cell's largest width -- radial r_{i+1} - r_i, or polar r_c times its
 * angular width (the midplane row spans both hemispheres: twice its half
 * width).  Below 1 the cell is transparent at every wavelength along every
 * direction.  (The thin midplane row is opaque along its radial width while
 * its height is a sliver, so the largest width, not the smallest, says
 * whether it is diffusive.) */
static double cell_optical_width(const ora_model* m, int c) {
  int i = c / m->n_mu, j = c % m->n_mu;
  double chi = 0.0;
  for (int k = 0; k < m->n_lambda; ++k) {
    double x = m->kappa_abs[k] + m->kappa_sca[k];
    if (x > chi) chi = x;
  }
  double rc = 0.5 * (m->r_edges[i] + m->r_edges[i + 1]);
  double wr = m->r_edges[i + 1] - m->r_edges[i];
  double wt = rc * (acos(m->mu_edges[j]) - acos(m->mu_edges[j + 1])) * (j == 0 ? 2.0 : 1.0);
  return m->rho[c] * chi * (wr > wt ? wr : wt);
}

/* Vertical hydrostatic equilibrium (Sect. 2.5, eq. balance): dP/dz =
 * -rho G M z / R^3 with P = k rho T / (mu_mol m_p), along each radial shell
 * of the grid at its mid radius r (z = r mu, R = r sqrt(1 - mu^2)) through
 * the cell centres:
 *   ln(rho_j T_j) - ln(rho_{j-1} T_{j-1}) = -(mu_mol m_p G M / k) * integral of
 *   z / (R^3 T) dz, by the trapezoidal rule between consecutive centres,
 * with T floored at T_floor.  Each shell keeps its mass (the surface density
 * is held fixed while the vertical profile is solved).  A shell holding an
 * optically thick dust cell without a temperature (T <= 0: no packet was
 * absorbed there) cannot be balanced -- a zero temperature would collapse
 * its scale height, which is why the paper first fills such cells by the PDA
 * (Sect. 3.4, Case 3 of the vertical-structure study) -- so it keeps its
 * density; the count of such shells is returned.  A cold cell transparent at
 * every wavelength holds no mass worth the name and is floored like any T
 * below T_floor. */
static const double G_GRAV = 6.67430e-8;
static const double M_PROTON = 1.67262192369e-24;

int ora_hydrostatic(const ora_model* m, const double* T, double M_star, double mu_mol,
                    double T_floor, double* rho_out) {
  const int nmu = m->n_mu;
  const double A = mu_mol * M_PROTON * G_GRAV * M_star / K_BOLTZ;
  double* lnf = (double*)malloc(sizeof(double) * nmu);
  double* V = (double*)malloc(sizeof(double) * (size_t)m->n_r * nmu);
  ora_cell_volumes(m, V);
  int n_cold = 0;
  for (int i = 0; i < m->n_r; ++i) {
    int cold = 0;
    for (int j = 0; j < nmu; ++j) {
      const size_t c = (size_t)i * nmu + j;
      if (m->rho[c] > 0.0 && !(T[c] > 0.0) && cell_optical_width(m, (int)c) >= 1.0) cold = 1;
    }
    if (cold) {
      for (int j = 0; j < nmu; ++j) rho_out[(size_t)i * nmu + j] = m->rho[(size_t)i * nmu + j];
      ++n_cold;
      continue;
    }
    const double r = 0.5 * (m->r_edges[i] + m->r_edges[i + 1]);
    double z_prev = 0.0, h_prev = 0.0, T0 = 0.0, acc = 0.0;
    for (int j = 0; j < nmu; ++j) {
      const double mc = 0.5 * (m->mu_edges[j] + m->mu_edges[j + 1]);
      const double z = r * mc;
      const double R = r * sqrt(1.0 - mc * mc);
      const double Tj = fmax(T[(size_t)i * nmu + j], T_floor);
      const double h = z / (R * R * R * Tj);
      if (j == 0) {
        T0 = Tj;
      } else {
        acc += 0.5 * (h_prev + h) * (z - z_prev);
      }
      lnf[j] = log(T0 / Tj) - A * acc;
      z_prev = z;
      h_prev = h;
    }
    double mass = 0.0, s = 0.0;
    for (int j = 0; j < nmu; ++j) {
      const size_t c = (size_t)i * nmu + j;
      mass += m->rho[c] * V[c];
      s += exp(lnf[j]) * V[c];
    }
    for (int j = 0; j < nmu; ++j) {
      const size_t c = (size_t)i * nmu + j;
      rho_out[c] = s > 0.0 ? mass * exp(lnf[j]) / s : 0.0;
    }
  }
  free(lnf);
  free(V);
  return n_cold;
}

/* Convergence statistic of the vertical-structure loop (Sect. 2.5: the mean
 * change of the temperature between two consecutive passes against its
 * photon noise; converged below 3).  The noise comes from the pass itself:
 * its odd- and even-numbered packets are two independent half-size runs, so
 * with E_a = 2 E_half and E_b = 2 (E - E_half) the absorbed energy's
 * variance is ~ (E_a - E_b)^2 / 4 = (2 E_half - E)^2: whatever carries the
 * energy (single absorptions or MRW deposits of any size), where 1 / N_abs
 * would count absorptions as independent though one packet makes many.  The
 * relative variance of T follows with the local slope of the inversion,
 * dlnT/dlnE (a central difference of T(E) over E (1 +- 1e-4)):
 *   s2 = (dlnT/dlnE)^2 ((2 E_half - E) / E)^2.
 * Dusty cells entered by >= n_min packets with E > 0 are eligible; over the cells
 * eligible in this pass and the previous one (s2_prev >= 0),
 *   R = sqrt(sum x^2 / sum (s2 + s2_prev)),  x = (T - T_prev) / T.
 * T_prev and s2_prev [n_cells] hold the previous pass (s2_prev < 0: not
 * eligible) and are replaced by this pass's values.  out: R (0 when nothing
 * is compared), the RMS of x, the RMS noise sqrt(mean(s2 + s2_prev)), the
 * cells compared. */
void ora_conv_stat(const ora_model* m, const ora_tables* t, const double* E_abs,
                   const double* E_half, const uint32_t* visits, int n_min, double* T_prev,
                   double* s2_prev, double out[4]) {
  const int nc = m->n_r * m->n_mu;
  const double h = 1e-4;
  double* V = (double*)malloc(sizeof(double) * nc);
  ora_cell_volumes(m, V);
  double sx = 0.0, ss = 0.0;
  long long cells = 0;
  for (int c = 0; c < nc; ++c) {
    const double mass = m->rho[c] * V[c];
    const double E = E_abs[c];
    const double T = ora_T_of_E(m, t, E, mass);
    double s2 = -1.0;
    if ((long long)visits[c] >= n_min && mass > 0.0 && E > 0.0 && T > 0.0) {
      const double Tp = ora_T_of_E(m, t, E * (1.0 + h), mass);
      const double Tm = ora_T_of_E(m, t, E * (1.0 - h), mass);
      const double slope = log(Tp / Tm) / (2.0 * h);
      const double rel = (2.0 * E_half[c] - E) / E;
      s2 = slope * slope * rel * rel;
      if (s2_prev[c] >= 0.0 && T_prev[c] > 0.0) {
        const double x = (T - T_prev[c]) / T;
        sx += x * x;
        ss += s2 + s2_prev[c];
        ++cells;
      }
    }
    T_prev[c] = T;
    s2_prev[c] = s2;
  }
  free(V);
  out[0] = ss > 0.0 ? sqrt(sx / ss) : 0.0;
  out[1] = cells ? sqrt(sx / (double)cells) : 0.0;
  out[2] = cells ? sqrt(ss / (double)cells) : 0.0;
  out[3] = (double)cells;
}

/* ------------------------------------------------------------------------ */
/* Observables by integration of the source function (Sect. 2.3, Sect. 3.3)  */
/* ------------------------------------------------------------------------ */

/* Mean intensity per cell and bin (erg s^-1 cm^-2 sr^-1, integrated over the
 * bin) from a run's path-length tallies: J_k = (path_k + w_k mrw_path) /
 * (4 pi V).  Explicit flights add eps * length at their bin; an MRW step adds
 * eps * c t to the cell, spread over the bins as the walk's photons spend
 * their path: weights eta_k / chi_k normalised (the weighting that defines
 * kappa-bar, so sum_k w_k kappa_k = kappa-bar), eta at the cell's T. */
void ora_mean_intensity(const ora_model* m, const double* T, const double* path,
                        const double* mrw_path, double* J) {
  const int nl = m->n_lambda, nc = m->n_r * m->n_mu;
  double* V = (double*)malloc(sizeof(double) * nc);
  double* Bb = (double*)malloc(sizeof(double) * nl);
  double* dBb = (double*)malloc(sizeof(double) * nl);
  double* eta = (double*)malloc(sizeof(double) * nl);
  double* tmp = (double*)malloc(sizeof(double) * nl);
  ora_cell_volumes(m, V);
  const double sim = 1.0 - m->g_asym;
  for (int c = 0; c < nc; ++c) {
    const double iv = V[c] > 0.0 ? 1.0 / (4.0 * PI * V[c]) : 0.0;
    for (int k = 0; k < nl; ++k) J[(size_t)c * nl + k] = path[(size_t)c * nl + k] * iv;
    if (mrw_path && mrw_path[c] > 0.0 && T[c] > 0.0) {
      ora_planck_bins(m->lambda_edges, nl, T[c], Bb, dBb);
      eta_iterate(m, dBb, eta, tmp);
      double sw = 0.0;
      for (int k = 0; k < nl; ++k) sw += eta[k] / (m->kappa_abs[k] + m->kappa_sca[k] * sim);
      for (int k = 0; k < nl; ++k)
        J[(size_t)c * nl + k] +=
            mrw_path[c] * iv * eta[k] / (m->kappa_abs[k] + m->kappa_sca[k] * sim) / sw;
    }
  }
  free(V); free(Bb); free(dBb); free(eta); free(tmp);
}

/* Crossings of the ray x(s) = b + s n (b perpendicular to n, |n| = 1) with the
 * grid's faces inside r_out: spheres r_e (|x|^2 = |b|^2 + s^2) and cones
 * |z| = mu_e |x| (e = 1 .. n_mu-1).  Returns their count in s_out (unsorted). */
static int ray_crossings(const ora_model* m, const double b[3], const double n[3], double* s_out) {
  const int nr = m->n_r, nmu = m->n_mu;
  const double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
  const double ro = m->r_edges[nr];
  const double S = sqrt(fmax(ro * ro - bb, 0.0));
  int q = 0;
  for (int e = 0; e <= nr; ++e) {
    double d2 = m->r_edges[e] * m->r_edges[e] - bb;
    if (d2 > 0.0) {
      s_out[q++] = -sqrt(d2);
      s_out[q++] = sqrt(d2);
    }
  }
  for (int e = 1; e < nmu; ++e) {
    /* (b_z + s n_z)^2 = mu^2 (|b|^2 + s^2) */
    const double mu2 = m->mu_edges[e] * m->mu_edges[e];
    const double A = n[2] * n[2] - mu2, B = b[2] * n[2], C = b[2] * b[2] - mu2 * bb;
    if (A == 0.0) {
      if (B != 0.0) {
        double r = -C / (2.0 * B);
        if (fabs(r) < S) s_out[q++] = r;
      }
      continue;
    }
    double disc = B * B - A * C;
    if (disc <= 0.0) continue;
    double sq = sqrt(disc);
    double r1 = (-B - sq) / A, r2 = (-B + sq) / A;
    if (fabs(r1) < S) s_out[q++] = r1;
    if (fabs(r2) < S) s_out[q++] = r2;
  }
  return q;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* Isotropic-equivalent luminosity per bin seen from the directions of
 * cos(inclination) cos_i[q] (erg/s per bin: 4 pi D^2 times the flux at
 * distance D), from the formal solution of the transfer equation along
 * parallel rays towards the observer, dI/ds = rho chi (S - I), with the
 * source function of isotropic scattering
 *   S_k = (kappa_abs,k Bbar_k(T) + kappa_sca,k J_k) / chi_k
 * per cell (J nullable: no scattering source), constant over each cell
 * segment: I <- I e^(-dtau) + S (1 - e^(-dtau)) from the far side to the
 * near one.  Rays: the image plane around the star in rings -- the hole
 * [0, r_0] and every radial cell [r_i, r_{i+1}] cut into n_sub equal rings
 * -- and n_phi azimuths phi = (p + 1/2) pi / n_phi on one side of the plane
 * through the line of sight and the pole, each standing also for its mirror
 * image; a ray at the ring's mid radius carries the area
 * pi (b_hi^2 - b_lo^2) / n_phi.  The star adds its luminosity per bin (the
 * spectrum the packets are launched with) times e^(-tau) along the line of
 * sight from its centre.  out [n_inc][n_lambda]. */
/* The star's luminosity per bin (the spectrum the packets are launched
 * with) times e^(-tau) along the line of sight n from its centre; cr is
 * scratch for the crossings. */
static void star_dimmed(const ora_model* m, const ora_tables* t, const double n[3], double* cr,
                        double* out) {
  const double zero[3] = {0.0, 0.0, 0.0};
  int nx = ray_crossings(m, zero, n, cr);
  qsort(cr, nx, sizeof(double), cmp_double);
  for (int k = 0; k < m->n_lambda; ++k) {
    double tau = 0.0;
    for (int g = 0; g + 1 < nx; ++g) {
      const double len = cr[g + 1] - cr[g];
      const double sm = 0.5 * (cr[g] + cr[g + 1]);
      if (!(len > 0.0) || sm <= 0.0) continue;
      const int64_t c = ora_locate(m, sm * n[0], sm * n[1], sm * n[2]);
      if (c >= 0) tau += m->rho[c] * (m->kappa_abs[k] + m->kappa_sca[k]) * len;
    }
    const double share = t->star_cdf[k] - (k ? t->star_cdf[k - 1] : 0.0);
    out[k] = t->L_star * share * exp(-tau);
  }
}

static void raytrace(const ora_model* m, const ora_tables* t, const double* T, const double* J,
                     int n_inc, const double* cos_i, int n_sub, int n_phi, double* out,
                     double* img) {
  const int nl = m->n_lambda, nr = m->n_r, nmu = m->n_mu, nc = nr * nmu;
  double* S = (double*)malloc(sizeof(double) * (size_t)nc * nl);
  double* Bb = (double*)malloc(sizeof(double) * nl);
  double* dBb = (double*)malloc(sizeof(double) * nl);
  double* I = (double*)malloc(sizeof(double) * nl);
  double* cr = (double*)malloc(sizeof(double) * (2 * (nr + 1) + 2 * nmu + 2));
  for (int c = 0; c < nc; ++c) {
    ora_planck_bins(m->lambda_edges, nl, T[c] > 0.0 ? T[c] : 0.0, Bb, dBb);
    for (int k = 0; k < nl; ++k) {
      const double chi = m->kappa_abs[k] + m->kappa_sca[k];
      const double sca = J ? m->kappa_sca[k] * J[(size_t)c * nl + k] : 0.0;
      S[(size_t)c * nl + k] = (m->kappa_abs[k] * Bb[k] + sca) / chi;
    }
  }
  for (int q = 0; q < n_inc; ++q) {
    const double ci = cos_i[q], si = sqrt(fmax(0.0, 1.0 - ci * ci));
    const double n[3] = {si, 0.0, ci};      /* towards the observer */
    const double e1[3] = {ci, 0.0, -si};    /* image plane */
    const double e2[3] = {0.0, 1.0, 0.0};
    double* L = out ? out + (size_t)q * nl : NULL;
    if (L)
      for (int k = 0; k < nl; ++k) L[k] = 0.0;
    for (int ring = 0; ring < (nr + 1) * n_sub; ++ring) {
      const int cell = ring / n_sub, part = ring % n_sub;
      const double lo = cell == 0 ? 0.0 : m->r_edges[cell - 1];
      const double hi = m->r_edges[cell];
      const double b_lo = lo + (hi - lo) * part / n_sub;
      const double b_hi = lo + (hi - lo) * (part + 1) / n_sub;
      const double bm = 0.5 * (b_lo + b_hi);
      const double area = PI * (b_hi * b_hi - b_lo * b_lo) / n_phi;
      for (int ph = 0; ph < n_phi; ++ph) {
        const double phi = (ph + 0.5) * PI / n_phi;
        double b[3];
        for (int a = 0; a < 3; ++a) b[a] = bm * (cos(phi) * e1[a] + sin(phi) * e2[a]);
        int nx = ray_crossings(m, b, n, cr);
        qsort(cr, nx, sizeof(double), cmp_double);
        for (int k = 0; k < nl; ++k) I[k] = 0.0;
        for (int g = 0; g + 1 < nx; ++g) {
          const double len = cr[g + 1] - cr[g];
          if (!(len > 0.0)) continue;
          const double sm = 0.5 * (cr[g] + cr[g + 1]);
          const int64_t c = ora_locate(m, b[0] + sm * n[0], b[1] + sm * n[1], b[2] + sm * n[2]);
          if (c < 0 || m->rho[c] <= 0.0) continue;
          for (int k = 0; k < nl; ++k) {
            const double dtau = m->rho[c] * (m->kappa_abs[k] + m->kappa_sca[k]) * len;
            const double at = exp(-dtau);
            I[k] = I[k] * at + S[(size_t)c * nl + k] * (1.0 - at);
          }
        }
        if (img) {
          double* dst = img + (((size_t)q * (nr + 1) * n_sub + ring) * n_phi + ph) * nl;
          for (int k = 0; k < nl; ++k) dst[k] = I[k];
        }
        if (L)
          for (int k = 0; k < nl; ++k) L[k] += 4.0 * PI * I[k] * area;
      }
    }
    if (!L) continue;
    /* the star, through the cells along the line of sight from its centre */
    star_dimmed(m, t, n, cr, I);
    for (int k = 0; k < nl; ++k) L[k] += I[k];
  }
  free(S); free(Bb); free(dBb); free(I); free(cr);
}

void ora_raytrace_sed(const ora_model* m, const ora_tables* t, const double* T, const double* J,
                      int n_inc, const double* cos_i, int n_sub, int n_phi, double* out) {
  raytrace(m, t, T, J, n_inc, cos_i, n_sub, n_phi, out, NULL);
}

/* The image behind the same rays: the intensity each ray reaches the observer
 * with (erg s^-1 cm^-2 sr^-1 per bin), without the star.
 * img [n_inc][(n_r + 1) n_sub][n_phi][n_lambda]. */
void ora_raytrace_image(const ora_model* m, const ora_tables* t, const double* T,
                        const double* J, int n_inc, const double* cos_i, int n_sub, int n_phi,
                        double* img) {
  raytrace(m, t, T, J, n_inc, cos_i, n_sub, n_phi, NULL, img);
}

/* Visibility amplitudes of a ray-traced image (Sect. 3.4 shows visibility
 * curves: the normalised Fourier transform of the image at the spatial
 * frequency of a baseline), with the star as a point at the centre.  img is
 * ora_raytrace_image's [n_inc][(n_r + 1) n_sub][n_phi][n_lambda]; ray
 * (ring, p) sits at b (cos phi e1 + sin phi e2), e1 = (cos i, 0, -sin i),
 * e2 = (0, 1, 0), phi = (p + 1/2) pi / n_phi, and stands also for its mirror
 * image at -phi; each of the two carries half of pi (b_hi^2 - b_lo^2) / n_phi.
 * Baseline j: length base[2 j] (cm), position angle base[2 j + 1] (radians
 * from e1 towards e2).  At the distance D (cm), bin k is sampled at the
 * spatial frequency s = B / (lambda_k D) cycles per cm of the image plane,
 * lambda_k the bin's geometric centre:
 *   V = |sum A I e^(-2 pi i s (x cos theta + y sin theta)) + L_star,k / (4 pi)|
 *       / (sum A I + L_star,k / (4 pi)),
 * L_star,k the star dimmed along the line of sight.  V [n_inc][n_base][n_lambda]. */
void ora_visibility(const ora_model* m, const ora_tables* t, const double* img, int n_inc,
                    const double* cos_i, int n_sub, int n_phi, int n_base, const double* base,
                    double distance, double* V) {
  const int nl = m->n_lambda, nr = m->n_r, nmu = m->n_mu;
  const int n_rings = (nr + 1) * n_sub;
  double* star = (double*)malloc(sizeof(double) * nl);
  double* cr = (double*)malloc(sizeof(double) * (2 * (nr + 1) + 2 * nmu + 2));
  for (int q = 0; q < n_inc; ++q) {
    const double ci = cos_i[q], si = sqrt(fmax(0.0, 1.0 - ci * ci));
    const double n[3] = {si, 0.0, ci};
    star_dimmed(m, t, n, cr, star);
    for (int j = 0; j < n_base; ++j) {
      const double B = base[2 * j], th = base[2 * j + 1];
      for (int k = 0; k < nl; ++k) {
        const double lam = sqrt(m->lambda_edges[k] * m->lambda_edges[k + 1]);
        const double sf = B / (lam * distance);
        double re = star[k] / (4.0 * PI), im = 0.0, tot = star[k] / (4.0 * PI);
        for (int ring = 0; ring < n_rings; ++ring) {
          const int cell = ring / n_sub, part = ring % n_sub;
          const double lo = cell == 0 ? 0.0 : m->r_edges[cell - 1];
          const double hi = m->r_edges[cell];
          const double b_lo = lo + (hi - lo) * part / n_sub;
          const double b_hi = lo + (hi - lo) * (part + 1) / n_sub;
          const double bm = 0.5 * (b_lo + b_hi);
          const double half = 0.5 * PI * (b_hi * b_hi - b_lo * b_lo) / n_phi;
          for (int p = 0; p < n_phi; ++p) {
            const double phi = (p + 0.5) * PI / n_phi;
            const double x = bm * cos(phi), y = bm * sin(phi);
            const double Iv = img[(((size_t)q * n_rings + ring) * n_phi + p) * nl + k];
            for (int mirror = 0; mirror < 2; ++mirror) {
              const double yy = mirror ? -y : y;
              const double arg = -2.0 * PI * sf * (x * cos(th) + yy * sin(th));
              re += half * Iv * cos(arg);
              im += half * Iv * sin(arg);
              tot += half * Iv;
            }
          }
        }
        V[((size_t)q * n_base + j) * nl + k] = tot > 0.0 ? sqrt(re * re + im * im) / tot : 0.0;
      }
    }
  }
  free(star); free(cr);
}

void ora_update_T(const ora_model* m, const ora_tables* t, const double* E_abs, double* T) {
  int nc = m->n_r * m->n_mu;
  double* V = (double*)malloc(sizeof(double) * nc);
  ora_cell_volumes(m, V);
  for (int c = 0; c < nc; ++c) T[c] = ora_T_of_E(m, t, E_abs[c], m->rho[c] * V[c]);
  free(V);
}

/* ------------------------------------------------------------------------ */
/* Transport of packets [offset, offset + n) of a run of n_total packets.     */
/* Each packet carries eps = L_star / n_total.                                */
/* ------------------------------------------------------------------------ */
int ora_run(const ora_model* m, const ora_tables* t, const ora_opts* o, uint64_t n_packets,
            uint64_t n_total, uint64_t seed, uint64_t offset, double* E_abs, uint32_t* visits,
            uint32_t* n_abs, uint32_t* n_mrw_cell, double* sed, double* E_star,
            long long* counters, ora_packet_rec* recs, int64_t n_recs, double* E_half,
            double* path, double* mrw_path) {
  const int nl = m->n_lambda, nmu = m->n_mu, nr = m->n_r;
  const int nc = nr * nmu;
  const double eps = t->L_star / (double)n_total;
  double* V = (double*)malloc(sizeof(double) * nc);
  double* inv4pim = (double*)malloc(sizeof(double) * nc);
  ora_cell_volumes(m, V);
  for (int c = 0; c < nc; ++c) {
    double mass = m->rho[c] * V[c];
    inv4pim[c] = mass > 0.0 ? 1.0 / (4.0 * PI * mass) : 0.0;
  }
  const double r_in = m->r_edges[0];

  for (uint64_t q = 0; q < n_packets; ++q) {
    uint64_t pid = offset + q;
    rng_t rng;
    rng_init(&rng, seed, pid);
    long long n_cross = 0, n_scat = 0, n_ab = 0, n_mrw = 0, events = 0;
    int fate = 0;
    /* launch: uniform point on the stellar sphere (azimuth 0 by symmetry),
     * Lambertian outward direction, bin from the stellar spectrum */
    double p[3], d[3];
    double ws = 2.0 * rng_next(&rng) - 1.0;
    double st = sqrt(fmax(0.0, 1.0 - ws * ws));
    p[0] = m->R_star * st;
    p[1] = 0.0;
    p[2] = m->R_star * ws;
    double mup = sqrt(rng_next(&rng));
    double php = 2.0 * PI * rng_next(&rng);
    double sp = sqrt(fmax(0.0, 1.0 - mup * mup));
    double ct = cos(php), sn = sin(php);
    /* n = (st, 0, ws); e_theta = (ws, 0, -st); e_phi = (0, 1, 0) */
    d[0] = mup * st + sp * ct * ws;
    d[1] = sp * sn;
    d[2] = mup * ws - sp * ct * st;
    double xs = rng_next(&rng);
    int k = 0;
    while (k < nl - 1 && !(t->star_cdf[k] > xs)) ++k;
    double tau = -log(rng_next(&rng));
    counters[ORA_C_LAUNCH]++;
    int i = -1, j = 0, n_int = 0;

    for (;;) {
      if (++events > o->max_events) { fate = 3; break; }
      if (i < 0) {
        /* inner hole: free flight to the star or back to r_in */
        double pd = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
        double rr = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        double s;
        if (sphere_in(pd, rr - m->R_star * m->R_star, &s)) {
          for (int a = 0; a < 3; ++a) p[a] += s * d[a];
          fate = 2;
          break;
        }
        sphere_out(pd, rr - r_in * r_in, &s);
        for (int a = 0; a < 3; ++a) p[a] += s * d[a];
        i = 0;
        double r2 = (p[0] * p[0] + p[1] * p[1]) + p[2] * p[2], z2 = p[2] * p[2];
        j = 0;
        for (int e = 1; e < nmu; ++e)
          if ((m->mu_edges[e] * m->mu_edges[e]) * r2 <= z2) j = e;
        visits[(size_t)i * nmu + j]++;
        n_int = 0;
        ++n_cross;
        continue;
      }
      int c = i * nmu + j;
      double chi = m->kappa_abs[k] + m->kappa_sca[k];
      double alpha = m->rho[c] * chi;
      int face;
      double sb = face_distance(m, i, j, p, d, &face);
      double tau_b = alpha * sb;
      if (tau_b <= tau) {
        /* reach the face: move, spend optical depth, step the index */
        if (path) path[(size_t)c * nl + k] += eps * sb;
        for (int a = 0; a < 3; ++a) p[a] += sb * d[a];
        tau -= tau_b;
        ++n_cross;
        if (face == 1) {
          if (i + 1 == nr) { /* escape: SED bin by |cos i| of the direction */
            int mi = (int)(fabs(d[2]) * o->n_inc);
            if (mi >= o->n_inc) mi = o->n_inc - 1;
            sed[(size_t)k * o->n_inc + mi] += eps;
            fate = 1;
            break;
          }
          ++i;
        } else if (face == 0) {
          --i;
          if (i < 0) { n_int = 0; continue; }
        } else if (face == 2) {
          --j;
        } else {
          ++j;
        }
        visits[(size_t)i * nmu + j]++;
        n_int = 0;
        continue;
      }
      /* interaction inside the cell */
      double sint = tau / alpha;
      if (path) path[(size_t)c * nl + k] += eps * sint;
      for (int a = 0; a < 3; ++a) p[a] += sint * d[a];
      double omega = m->kappa_sca[k] / chi;
      if (rng_next(&rng) < omega) {
        ++n_scat;
        scatter_dir(&rng, m->g_asym, d);
      } else {
        ++n_ab;
        n_abs[c]++;
        double E_old = E_abs[c];
        E_abs[c] = E_old + eps;
        if (E_half && (pid & 1)) E_half[c] += eps;
        double xb = rng_next(&rng);
        if (o->frozen_T) {
          k = reemit_bin(t, nl, -1.0, o->frozen_T[c], xb);
        } else {
          double T_old = T_of_g(t, nl, E_old * inv4pim[c]);
          double T_new = T_of_g(t, nl, E_abs[c] * inv4pim[c]);
          k = reemit_bin(t, nl, T_old, T_new, xb);
        }
        iso_dir(&rng, d);
      }
      ++n_int;
      /* modified random walk (eqs. modified RW .. criterion) */
      if (o->mrw) {
        for (;;) {
          if (n_int < o->n_int_min) break;
          double Tc = o->frozen_T ? o->frozen_T[c]
                      : o->coef_T ? o->coef_T[c] : T_of_g(t, nl, E_abs[c] * inv4pim[c]);
          double Drho = t_interp(t, t->Drho, Tc);
          double lam_R = 3.0 * Drho / m->rho[c]; /* 1/(rho chi_R) */
          double dmin = min_face_distance(m, i, j, p);
          if (!(dmin > o->gamma * lam_R)) break;
          if (++events > o->max_events) break;
          double R0 = dmin * (1.0 - 1e-6);
          double s = ora_mrw_escape_s(rng_next(&rng));
          double dE = eps * ora_mrw_deposit(m, t, c, Tc, R0, s);
          /* the walk's path, c t = s R0^2 / D */
          if (mrw_path) mrw_path[c] += eps * s * R0 * R0 * m->rho[c] / t_interp(t, t->Drho, Tc);
          double nrm[3];
          iso_dir(&rng, nrm);
          for (int a = 0; a < 3; ++a) p[a] += R0 * nrm[a];
          double E_old = E_abs[c];
          E_abs[c] = E_old + dE;
          if (E_half && (pid & 1)) E_half[c] += dE;
          double xb = rng_next(&rng);
          if (o->frozen_T) {
            k = reemit_bin(t, nl, -1.0, o->frozen_T[c], xb);
          } else {
            double T_old = T_of_g(t, nl, E_old * inv4pim[c]);
            double T_new = T_of_g(t, nl, E_abs[c] * inv4pim[c]);
            k = reemit_bin(t, nl, T_old, T_new, xb);
          }
          iso_dir(&rng, d);
          ++n_mrw;
          n_mrw_cell[c]++;
        }
      }
      tau = -log(rng_next(&rng));
    }
    if (fate == 1) counters[ORA_C_ESCAPED]++;
    else if (fate == 2) { counters[ORA_C_STAR]++; *E_star += eps; }
    else counters[ORA_C_CAPPED]++;
    counters[ORA_C_CROSS] += n_cross;
    counters[ORA_C_SCAT] += n_scat;
    counters[ORA_C_ABS] += n_ab;
    counters[ORA_C_MRW] += n_mrw;
    if ((int64_t)q < n_recs) {
      ora_packet_rec* R = &recs[q];
      R->fate = fate;
      R->k = k;
      R->n_cross = n_cross;
      R->n_scat = n_scat;
      R->n_abs = n_ab;
      R->n_mrw = n_mrw;
      R->n_draws = (int64_t)rng.d;
      R->x = p[0]; R->y = p[1]; R->z = p[2];
      R->u = d[0]; R->v = d[1]; R->w = d[2];
    }
  }
  free(V);
  free(inv4pim);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* PDA (Sect. 2.2.1, eq:T diffusion): div(D grad T^4) = 0 on the region,     */
/* Dirichlet T from the Monte Carlo run on the neighbouring cells.  Finite    */
/* volumes on the (r, mu) cells: flux A_f D_f (u_b - u_a) / dist_f with the   */
/* harmonic mean of the two cells' D, taken as 2 / (1/D_a + 1/D_b) on the   */
/* cells' resistances R = 1/D = rho s / (D rho)(T) (finite even where D      */
/* overflows); zero flux at the grid edges, the pole,                        */
/* the (folded) midplane and towards dust-free cells.                         */
/* ------------------------------------------------------------------------ */
typedef struct {
  int nr, nmu;
  double *rc, *thc;        /* cell centres */
  double *Ar, *Amu;        /* face areas: Ar[i*nmu+j] face r_{i+1}; Amu[i*nmu+j] face mu_{j+1} */
} pda_geom;

static void pda_geom_init(const ora_model* m, pda_geom* g) {
  int nr = m->n_r, nmu = m->n_mu;
  g->nr = nr;
  g->nmu = nmu;
  g->rc = (double*)malloc(sizeof(double) * nr);
  g->thc = (double*)malloc(sizeof(double) * nmu);
  g->Ar = (double*)malloc(sizeof(double) * nr * nmu);
  g->Amu = (double*)malloc(sizeof(double) * nr * nmu);
  for (int i = 0; i < nr; ++i) g->rc[i] = 0.5 * (m->r_edges[i] + m->r_edges[i + 1]);
  for (int j = 0; j < nmu; ++j)
    g->thc[j] = 0.5 * (acos(m->mu_edges[j]) + acos(m->mu_edges[j + 1]));
  for (int i = 0; i < nr; ++i)
    for (int j = 0; j < nmu; ++j) {
      double rf = m->r_edges[i + 1];
      g->Ar[i * nmu + j] = 2.0 * PI * rf * rf * 2.0 * (m->mu_edges[j + 1] - m->mu_edges[j]);
      double mf = m->mu_edges[j + 1];
      double a = m->r_edges[i], b = m->r_edges[i + 1];
      g->Amu[i * nmu + j] = PI * (b * b - a * a) * 2.0 * sqrt(fmax(0.0, 1.0 - mf * mf));
    }
}

static void pda_geom_free(pda_geom* g) {
  free(g->rc); free(g->thc); free(g->Ar); free(g->Amu);
}

/* conductance of the face between cells a and b (b = a's neighbour), from
 * the cells' resistances R = 1/D */
static double face_cond(const pda_geom* g, int ia, int ja, int ib, int jb, double Ra, double Rb) {
  double A, dist;
  if (ib != ia) {
    int ilo = ia < ib ? ia : ib;
    A = g->Ar[ilo * g->nmu + ja];
    dist = fabs(g->rc[ib] - g->rc[ia]);
  } else {
    int jlo = ja < jb ? ja : jb;
    A = g->Amu[ia * g->nmu + jlo];
    dist = g->rc[ia] * fabs(g->thc[jb] - g->thc[ja]);
  }
  double Df = 2.0 / (Ra + Rb);
  return A * Df / dist;
}

static int band_cholesky_solve(int n, int bw, double* band, double* x);

/* solve with an already factored band (L in band) */
static void band_solve_factored(int n, int bw, const double* band, double* x) {
  for (int c = 0; c < n; ++c) {
    double s = x[c];
    int kk0 = c - bw < 0 ? 0 : c - bw;
    for (int kk = kk0; kk < c; ++kk) s -= band[(size_t)c * (bw + 1) + (kk - c + bw)] * x[kk];
    x[c] = s / band[(size_t)c * (bw + 1) + bw];
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = x[c];
    int kk1 = c + bw >= n ? n - 1 : c + bw;
    for (int kk = c + 1; kk <= kk1; ++kk) s -= band[(size_t)kk * (bw + 1) + (c - kk + bw)] * x[kk];
    x[c] = s / band[(size_t)c * (bw + 1) + bw];
  }
}

/* banded Cholesky, half-bandwidth bw, full-grid ordering; LL^T in place.
 * band[c][q] holds A[c][c-bw+q], q = 0..bw */
static int band_cholesky_solve(int n, int bw, double* band, double* x) {
  for (int c = 0; c < n; ++c) {
    int q0 = c - bw < 0 ? bw - c : 0;
    for (int q = q0; q <= bw; ++q) {
      int r = c - bw + q; /* column index, r <= c */
      double s = band[(size_t)c * (bw + 1) + q];
      int kk0 = (c - bw > r - bw ? c - bw : r - bw);
      if (kk0 < 0) kk0 = 0;
      for (int kk = kk0; kk < r; ++kk)
        s -= band[(size_t)c * (bw + 1) + (kk - c + bw)] * band[(size_t)r * (bw + 1) + (kk - r + bw)];
      if (r == c) {
        if (!(s > 0.0)) return -1;
        band[(size_t)c * (bw + 1) + bw] = sqrt(s);
      } else {
        band[(size_t)c * (bw + 1) + q] = s / band[(size_t)r * (bw + 1) + bw];
      }
    }
  }
  for (int c = 0; c < n; ++c) { /* L y = b */
    double s = x[c];
    int kk0 = c - bw < 0 ? 0 : c - bw;
    for (int kk = kk0; kk < c; ++kk) s -= band[(size_t)c * (bw + 1) + (kk - c + bw)] * x[kk];
    x[c] = s / band[(size_t)c * (bw + 1) + bw];
  }
  for (int c = n - 1; c >= 0; --c) { /* L^T x = y */
    double s = x[c];
    int kk1 = c + bw >= n ? n - 1 : c + bw;
    for (int kk = c + 1; kk <= kk1; ++kk) s -= band[(size_t)kk * (bw + 1) + (c - kk + bw)] * x[kk];
    x[c] = s / band[(size_t)c * (bw + 1) + bw];
  }
  return 0;
}

/* assemble and solve once: D from T_D (region) and T_D (Dirichlet cells), u
 * Dirichlet = T_bc^4.  kscale scales chi per cell (NULL = 1). */
static int pda_solve_once(const ora_model* m, const ora_tables* t, const pda_geom* g,
                          const uint8_t* reg, const double* T_D, const double* T_bc,
                          const double* kscale, int skip_cold, double* u) {
  int nr = m->n_r, nmu = m->n_mu, n = nr * nmu, bw = nmu;
  double* band = (double*)calloc((size_t)n * (bw + 1), sizeof(double));
  double* R = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) {
    double ks = kscale ? kscale[c] : 1.0;
    R[c] = m->rho[c] > 0.0 ? m->rho[c] * ks / t_interp(t, t->Drho, T_D[c]) : 0.0;
  }
  for (int c = 0; c < n; ++c) {
    if (reg[c] != 1) {
      band[(size_t)c * (bw + 1) + bw] = 1.0;
      u[c] = pow(T_bc[c], 4.0);
      continue;
    }
    u[c] = 0.0;
  }
  for (int c = 0; c < n; ++c) {
    if (reg[c] != 1) continue;
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    double diag = 0.0;
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (!(m->rho[cb] > 0.0)) continue;
      /* a neighbour without a temperature gives no boundary value */
      if (skip_cold && reg[cb] != 1 && !(T_bc[cb] > 0.0)) continue;
      double a = face_cond(g, i, j, ib, jb, R[c], R[cb]);
      diag += a;
      if (reg[cb] == 1) {
        if (cb < c) band[(size_t)c * (bw + 1) + (cb - c + bw)] = -a;
      } else {
        u[c] += a * pow(T_bc[cb], 4.0);
      }
    }
    band[(size_t)c * (bw + 1) + bw] = diag;
  }
  int rc = band_cholesky_solve(n, bw, band, u);
  free(band);
  free(R);
  return rc;
}

/* cells of `reg` (value 1) whose connected component touches no usable
 * Dirichlet neighbour (dust-bearing, outside the region, and with T > 0 when
 * T is given) are set to 2 */
static void pda_components(const ora_model* m, const double* T, uint8_t* reg) {
  int nr = m->n_r, nmu = m->n_mu, n = nr * nmu;
  int* comp = (int*)malloc(sizeof(int) * n);
  int* stack = (int*)malloc(sizeof(int) * n);
  for (int c = 0; c < n; ++c) comp[c] = -1;
  for (int c0 = 0; c0 < n; ++c0) {
    if (reg[c0] != 1 || comp[c0] >= 0) continue;
    int top = 0, touches = 0, cnt = 0;
    stack[top++] = c0;
    comp[c0] = c0;
    int* members = (int*)malloc(sizeof(int) * n);
    while (top > 0) {
      int c = stack[--top];
      members[cnt++] = c;
      int i = c / nmu, j = c % nmu;
      int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
      for (int q = 0; q < 4; ++q) {
        int ib = nb[q][0], jb = nb[q][1];
        if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
        int cb = ib * nmu + jb;
        if (!(m->rho[cb] > 0.0)) continue;
        if (reg[cb] == 1) {
          if (comp[cb] < 0) { comp[cb] = c0; stack[top++] = cb; }
        } else if (!T || T[cb] > 0.0) {
          touches = 1;
        }
      }
    }
    if (!touches)
      for (int q = 0; q < cnt; ++q) reg[members[q]] = 2;
    free(members);
  }
  free(comp);
  free(stack);
}

/* Region of the PDA (Sect. 2.2.1): the cells whose Monte Carlo temperature
 * is not trusted.  Sect. 3.1 uses two tests: few packets entered the cell, or
 * the photon statistics leave a large relative error in its temperature.
 * With N absorption events the absorbed energy has relative error 1/sqrt(N)
 * and T ~ E^(1/4) has 1/(4 sqrt(N)); a cell without events has no estimate.
 * The diffusion approximation holds only in opaque matter, so the second
 * test takes only cells of optical width >= 1 at their most opaque
 * wavelength (the first test's few-visit cells are shielded anyway): a
 * nearly empty cell of the disk's atmosphere absorbs few packets because it
 * is transparent, not because it is shielded. */
void ora_pda_region(const ora_model* m, const uint32_t* visits, const uint32_t* n_abs,
                    const uint32_t* n_mrw, int visits_min, double sigma_max, uint8_t* region) {
  int n = m->n_r * m->n_mu;
  for (int c = 0; c < n; ++c) {
    int in = 0;
    if (m->rho[c] > 0.0) {
      if ((int64_t)visits[c] < (int64_t)visits_min) in = 1;
      if (sigma_max > 0.0 && cell_optical_width(m, c) >= 1.0) {
        double N = (double)n_abs[c] + (double)n_mrw[c];
        if (N == 0.0 || 1.0 / (4.0 * sqrt(N)) > sigma_max) in = 1;
      }
    }
    region[c] = (uint8_t)in;
  }
}

int ora_pda(const ora_model* m, const ora_tables* t, const double* T_mc, const uint8_t* region_in,
            double* T_out, uint8_t* region_out, int max_sweeps, double tol, int* n_sweeps,
            double* last_change, int* converged) {
  int nr = m->n_r, nmu = m->n_mu, n = nr * nmu;
  for (int c = 0; c < n; ++c) region_out[c] = (region_in[c] && m->rho[c] > 0.0) ? 1 : 0;
  pda_components(m, T_mc, region_out);
  /* floor for the initial guess: the smallest Dirichlet temperature */
  double Tfloor = INFINITY;
  for (int c = 0; c < n; ++c) {
    if (region_out[c] != 1) continue;
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (m->rho[cb] > 0.0 && region_out[cb] != 1 && T_mc[cb] > 0.0 && T_mc[cb] < Tfloor)
        Tfloor = T_mc[cb];
    }
  }
  if (!isfinite(Tfloor)) Tfloor = 0.0;
  for (int c = 0; c < n; ++c)
    T_out[c] = (region_out[c] == 1) ? fmax(T_mc[c], Tfloor) : T_mc[c];
  pda_geom g;
  pda_geom_init(m, &g);
  double* u = (double*)malloc(sizeof(double) * n);
  /* Picard sweeps: D from the current T, one linear solve, new T.  They stop
   * when the largest relative change falls below tol, or when it stalls below
   * sqrt(tol): a sweep that changes T no less than the previous one has
   * reached the rounding floor of the linear solve (the operator couples thin
   * and thick cells with conductances many orders apart). */
  int sweeps = 0, rc = 0, conv = 0;
  double change = 0.0, prev = INFINITY;
  for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
    rc = pda_solve_once(m, t, &g, region_out, T_out, T_mc, NULL, 1, u);
    if (rc) break;
    change = 0.0;
    for (int c = 0; c < n; ++c) {
      if (region_out[c] != 1) continue;
      double Tn = pow(fmax(u[c], 0.0), 0.25);
      double ch = fabs(Tn - T_out[c]) / fmax(Tn, 1e-300);
      if (ch > change) change = ch;
      T_out[c] = Tn;
    }
    if (change < tol || (change < sqrt(tol) && change >= prev)) {
      conv = 1;
      break;
    }
    prev = change;
  }
  if (sweeps > max_sweeps) sweeps = max_sweeps;
  *n_sweeps = sweeps;
  *last_change = change;
  *converged = conv;
  free(u);
  pda_geom_free(&g);
  return rc;
}

int ora_pda_linear(const ora_model* m, const ora_tables* t, const double* T_D, const double* T_bc,
                   const double* kscale, const uint8_t* region, double* T_out) {
  int n = m->n_r * m->n_mu;
  pda_geom g;
  pda_geom_init(m, &g);
  double* u = (double*)malloc(sizeof(double) * n);
  uint8_t* reg = (uint8_t*)malloc(n);
  for (int c = 0; c < n; ++c) reg[c] = (region[c] && m->rho[c] > 0.0) ? 1 : 0;
  pda_components(m, NULL, reg);
  int rc = pda_solve_once(m, t, &g, reg, T_D, T_bc, kscale, 0, u);
  for (int c = 0; c < n; ++c) T_out[c] = reg[c] == 1 ? pow(fmax(u[c], 0.0), 0.25) : T_bc[c];
  free(u);
  free(reg);
  pda_geom_free(&g);
  return rc;
}

/* Gradient of an objective J(T) of the linear PDA solve (D frozen at T_D)
 * with respect to log rho_c and s_c of the cells listed, by the direct
 * (tangent-linear) method: A du/dp = -dr/dp for each parameter p, with the
 * residual r(u, p) = A(D(p)) u - b(D(p)) and D_c = (D rho)(T_D,c)/(rho_c s_c),
 * then dJ/dp = sum_i dJ/dT_i dT_i/du_i du_i/dp.  One factorisation, one
 * solve per parameter. */
int ora_pda_grad_direct(const ora_model* m, const ora_tables* t, const double* T_D,
                        const double* T_bc, const double* kscale, const uint8_t* region_in,
                        const double* dJdT, const int* cells, int n_req, double* g_logrho,
                        double* g_kscale) {
  int nr = m->n_r, nmu = m->n_mu, n = nr * nmu, bw = nmu;
  pda_geom g;
  pda_geom_init(m, &g);
  uint8_t* reg = (uint8_t*)malloc(n);
  for (int c = 0; c < n; ++c) reg[c] = (region_in[c] && m->rho[c] > 0.0) ? 1 : 0;
  pda_components(m, NULL, reg);
  double* R = (double*)malloc(sizeof(double) * n);
  double* ks = (double*)malloc(sizeof(double) * n);
  double* ubc = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) {
    ks[c] = kscale ? kscale[c] : 1.0;
    R[c] = m->rho[c] > 0.0 ? m->rho[c] * ks[c] / t_interp(t, t->Drho, T_D[c]) : 0.0;
    ubc[c] = pow(T_bc[c], 4.0);
  }
  /* assemble (same operator as the forward) and factor */
  double* band = (double*)calloc((size_t)n * (bw + 1), sizeof(double));
  double* u = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) {
    if (reg[c] != 1) {
      band[(size_t)c * (bw + 1) + bw] = 1.0;
      u[c] = ubc[c];
      continue;
    }
    u[c] = 0.0;
  }
  for (int c = 0; c < n; ++c) {
    if (reg[c] != 1) continue;
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    double diag = 0.0;
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (!(m->rho[cb] > 0.0)) continue;
      double a = face_cond(&g, i, j, ib, jb, R[c], R[cb]);
      diag += a;
      if (reg[cb] == 1) {
        if (cb < c) band[(size_t)c * (bw + 1) + (cb - c + bw)] = -a;
      } else {
        u[c] += a * ubc[cb];
      }
    }
    band[(size_t)c * (bw + 1) + bw] = diag;
  }
  int rc = band_cholesky_solve(n, bw, band, u); /* factors band in place, u = solution */
  double* dTdu = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c)
    dTdu[c] = (reg[c] == 1 && u[c] > 0.0) ? 0.25 * pow(u[c], -0.75) : 0.0;
  double* w = (double*)malloc(sizeof(double) * n);
  for (int r = 0; rc == 0 && r < n_req; ++r) {
    int c = cells[r];
    g_logrho[r] = 0.0;
    if (g_kscale) g_kscale[r] = 0.0;
    if (!(m->rho[c] > 0.0)) continue;
    for (int k = 0; k < n; ++k) w[k] = 0.0;
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    int any = 0;
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (!(m->rho[cb] > 0.0)) continue;
      if (reg[c] != 1 && reg[cb] != 1) continue;
      /* a_f = (A_f/dist_f) 2 / (R_c + R_b) and dR_c / dlog rho_c = R_c */
      double a1 = face_cond(&g, i, j, ib, jb, 1.0, 1.0);  /* A_f / dist_f */
      double sden = R[c] + R[cb];
      double da = -a1 * 2.0 * R[c] / (sden * sden); /* per unit log rho_c */
      if (reg[c] == 1) w[c] -= da * (u[c] - u[cb]);
      if (reg[cb] == 1) w[cb] -= da * (u[cb] - u[c]);
      any = 1;
    }
    if (!any) continue;
    band_solve_factored(n, bw, band, w);
    double s = 0.0;
    for (int k = 0; k < n; ++k)
      if (reg[k] == 1) s += dJdT[k] * dTdu[k] * w[k];
    g_logrho[r] = s;
    if (g_kscale) g_kscale[r] = s / ks[c]; /* dR/ds = R/s: the same with 1/s */
  }
  free(w);
  free(dTdu);
  free(band);
  free(u);
  free(ubc);
  free(ks);
  free(R);
  free(reg);
  pda_geom_free(&g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Nonlinear PDA for differentiation (Sect. 2.2.1, eq. T diffusion, with the */
/* diffusion coefficient D(T) of Sect. 2.2.3): Picard sweeps of the linear   */
/* solve, D from the current T, until the fixed point; Dirichlet T_bc on the */
/* other cells.  At the fixed point the residual of every region cell,       */
/*   r_c(u, p) = sum_f a_f(R_c, R_b) (u_c - u_b),  R = rho s / (D rho)(T),   */
/* a_f = (A_f / dist_f) 2 / (R_c + R_b), u = T^4, vanishes; so by the        */
/* implicit function theorem J du/dp = -dr/dp with the Jacobian J = dr/du,   */
/* which, beside the conductances, holds their dependence on u through       */
/* R(T(u)): da_f/du_x = -a_f / (R_c + R_b) dR_x/du_x for x = c, b, and       */
/* dR/du = -R (D rho)'(T) / (D rho)(T) T / (4 u) with (D rho)' the slope of  */
/* the tabulated segment.  J is not symmetric.                              */
/* ------------------------------------------------------------------------ */
int ora_pda_nl(const ora_model* m, const ora_tables* t, const double* T_bc,
               const double* kscale, const uint8_t* region_in, int max_sweeps, double tol,
               double* T_out, int* n_sweeps, double* last_change) {
  int n = m->n_r * m->n_mu;
  pda_geom g;
  pda_geom_init(m, &g);
  uint8_t* reg = (uint8_t*)malloc(n);
  for (int c = 0; c < n; ++c) reg[c] = (region_in[c] && m->rho[c] > 0.0) ? 1 : 0;
  pda_components(m, NULL, reg);
  double* u = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) T_out[c] = T_bc[c];
  int sweeps = 0, rc = 0;
  double change = 0.0, prev = INFINITY;
  for (sweeps = 1; sweeps <= max_sweeps; ++sweeps) {
    rc = pda_solve_once(m, t, &g, reg, T_out, T_bc, kscale, 0, u);
    if (rc) break;
    change = 0.0;
    for (int c = 0; c < n; ++c) {
      if (reg[c] != 1) continue;
      double Tn = pow(fmax(u[c], 0.0), 0.25);
      double ch = fabs(Tn - T_out[c]) / fmax(Tn, 1e-300);
      if (ch > change) change = ch;
      T_out[c] = Tn;
    }
    if (change < tol || (change < sqrt(tol) && change >= prev)) break;
    prev = change;
  }
  if (sweeps > max_sweeps) sweeps = max_sweeps;
  if (n_sweeps) *n_sweeps = sweeps;
  if (last_change) *last_change = change;
  free(u);
  free(reg);
  pda_geom_free(&g);
  return rc;
}

/* banded LU without pivoting of a (2 bw + 1)-diagonal matrix in place,
 * band[c][q] = A[c][c - bw + q], q = 0 .. 2 bw; then solves for x */
static int band_lu_factor(int n, int bw, double* band) {
  const int W = 2 * bw + 1;
  for (int k = 0; k < n; ++k) {
    double piv = band[(size_t)k * W + bw];
    if (!(fabs(piv) > 0.0)) return -1;
    int rmax = k + bw < n - 1 ? k + bw : n - 1;
    for (int r = k + 1; r <= rmax; ++r) {
      double* lr = &band[(size_t)r * W + (k - r + bw)];
      if (*lr == 0.0) continue;
      double l = *lr / piv;
      *lr = l;
      int cmax = k + bw < n - 1 ? k + bw : n - 1;
      for (int col = k + 1; col <= cmax; ++col)
        band[(size_t)r * W + (col - r + bw)] -= l * band[(size_t)k * W + (col - k + bw)];
    }
  }
  return 0;
}

static void band_lu_solve(int n, int bw, const double* band, double* x) {
  const int W = 2 * bw + 1;
  for (int r = 0; r < n; ++r) {
    int k0 = r - bw < 0 ? 0 : r - bw;
    double s = x[r];
    for (int k = k0; k < r; ++k) s -= band[(size_t)r * W + (k - r + bw)] * x[k];
    x[r] = s;
  }
  for (int r = n - 1; r >= 0; --r) {
    int k1 = r + bw > n - 1 ? n - 1 : r + bw;
    double s = x[r];
    for (int k = r + 1; k <= k1; ++k) s -= band[(size_t)r * W + (k - r + bw)] * x[k];
    x[r] = s / band[(size_t)r * W + bw];
  }
}

/* slope of a tabulated quantity on the segment holding T (the derivative
 * of t_interp's linear interpolation) */
static double t_slope(const ora_tables* t, const double* tab, double T) {
  int n;
  double f;
  t_segment(t, T, &n, &f);
  return (tab[n + 1] - tab[n]) / (t->T[n + 1] - t->T[n]);
}

int ora_pda_nl_grad_direct(const ora_model* m, const ora_tables* t, const double* T_bc,
                           const double* kscale, const uint8_t* region_in, int max_sweeps,
                           double tol, const double* dJdT, const int* cells, int n_req,
                           double* T_out, double* g_logrho, double* g_kscale) {
  int nr = m->n_r, nmu = m->n_mu, n = nr * nmu, bw = nmu, W = 2 * bw + 1;
  int rc = ora_pda_nl(m, t, T_bc, kscale, region_in, max_sweeps, tol, T_out, NULL, NULL);
  if (rc) return rc;
  pda_geom g;
  pda_geom_init(m, &g);
  uint8_t* reg = (uint8_t*)malloc(n);
  for (int c = 0; c < n; ++c) reg[c] = (region_in[c] && m->rho[c] > 0.0) ? 1 : 0;
  pda_components(m, NULL, reg);
  double* R = (double*)malloc(sizeof(double) * n);
  double* ks = (double*)malloc(sizeof(double) * n);
  double* u = (double*)malloc(sizeof(double) * n);
  double* dRdu = (double*)malloc(sizeof(double) * n);
  for (int c = 0; c < n; ++c) {
    ks[c] = kscale ? kscale[c] : 1.0;
    double T = T_out[c];
    double Drho = t_interp(t, t->Drho, T);
    R[c] = m->rho[c] > 0.0 ? m->rho[c] * ks[c] / Drho : 0.0;
    u[c] = pow(T, 4.0);
    dRdu[c] = 0.0;
    if (reg[c] == 1 && u[c] > 0.0 && m->rho[c] > 0.0)
      dRdu[c] = -R[c] * t_slope(t, t->Drho, T) / Drho * T / (4.0 * u[c]);
  }
  /* the Jacobian, band storage; the rows of the Dirichlet cells are the
   * identity (their u does not move) */
  double* band = (double*)calloc((size_t)n * W, sizeof(double));
  for (int c = 0; c < n; ++c) {
    if (reg[c] != 1) {
      band[(size_t)c * W + bw] = 1.0;
      continue;
    }
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (!(m->rho[cb] > 0.0)) continue;
      double a = face_cond(&g, i, j, ib, jb, R[c], R[cb]);
      double dadR = -a / (R[c] + R[cb]);
      band[(size_t)c * W + bw] += a + dadR * dRdu[c] * (u[c] - u[cb]);
      if (reg[cb] == 1)
        band[(size_t)c * W + (cb - c + bw)] += -a + dadR * dRdu[cb] * (u[c] - u[cb]);
    }
  }
  rc = band_lu_factor(n, bw, band);
  double* w = (double*)malloc(sizeof(double) * n);
  for (int r = 0; rc == 0 && r < n_req; ++r) {
    int c = cells[r];
    g_logrho[r] = 0.0;
    if (g_kscale) g_kscale[r] = 0.0;
    if (!(m->rho[c] > 0.0)) continue;
    for (int k = 0; k < n; ++k) w[k] = 0.0;
    int i = c / nmu, j = c % nmu;
    int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
    int any = 0;
    for (int q = 0; q < 4; ++q) {
      int ib = nb[q][0], jb = nb[q][1];
      if (ib < 0 || ib >= nr || jb < 0 || jb >= nmu) continue;
      int cb = ib * nmu + jb;
      if (!(m->rho[cb] > 0.0)) continue;
      if (reg[c] != 1 && reg[cb] != 1) continue;
      /* dr/dlog rho_c through R_c = rho_c s_c / (D rho)(T_c) */
      double a = face_cond(&g, i, j, ib, jb, R[c], R[cb]);
      double da = -a / (R[c] + R[cb]) * R[c];
      if (reg[c] == 1) w[c] -= da * (u[c] - u[cb]);
      if (reg[cb] == 1) w[cb] -= da * (u[cb] - u[c]);
      any = 1;
    }
    if (!any) continue;
    band_lu_solve(n, bw, band, w);
    double s = 0.0;
    for (int k = 0; k < n; ++k)
      if (reg[k] == 1 && u[k] > 0.0) s += dJdT[k] * (T_out[k] / (4.0 * u[k])) * w[k];
    g_logrho[r] = s;
    if (g_kscale) g_kscale[r] = s / ks[c];
  }
  free(w);
  free(band);
  free(dRdu);
  free(u);
  free(ks);
  free(R);
  free(reg);
  pda_geom_free(&g);
  return rc;
}
