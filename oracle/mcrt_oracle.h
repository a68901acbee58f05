/*
 * CPU oracle for Monte Carlo radiative transfer in an axisymmetric dust disk
 * with immediate reemission, the modified random walk (MRW) and the partial
 * diffusion approximation (PDA), after Min et al. (2009).
 *
 * TEST INFRASTRUCTURE.  Plain, single-threaded, FP64 and deliberately slow.
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * call it.  It shares no source with the HIP library; the two meet only in the
 * input arrays a test builds from the seeded workload generator.
 *
 * Units: cgs.  Cell id = i_r * n_mu + j_mu; j_mu = 0 is the midplane row of the
 * folded polar coordinate mu = |cos theta|.
 */
#ifndef MCRT_ORACLE_H
#define MCRT_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_r, n_mu, n_lambda;
  const double* r_edges;       /* [n_r+1] */
  const double* mu_edges;      /* [n_mu+1], 0 = midplane ... 1 = pole */
  const double* rho;           /* [n_r*n_mu] dust density */
  const double* lambda_edges;  /* [n_lambda+1] cm */
  const double* kappa_abs;     /* [n_lambda] mixture absorption opacity, cm^2/g */
  const double* kappa_sca;     /* [n_lambda] mixture scattering opacity */
  double T_star, R_star;
  double g_asym;               /* asymmetry parameter of the Henyey-Greenstein
                                  phase function of scattering (0: isotropic) */
} ora_model;

typedef struct {
  int n_T;                     /* nodes; node 0 is T = 0 */
  double T_lo, T_hi;           /* first non-zero node, last node */
  double* T;                   /* [n_T] */
  double* cdf;                 /* [n_T][n_lambda]  sum_{k'<=k} kappa_k' Bbar_k'(T_n) */
  double* Drho;                /* [n_T]  D * rho of the diffusion coefficient */
  double* kbar;                /* [n_T]  mean absorption opacity of an MRW step */
  double* star_cdf;            /* [n_lambda] cumulative star spectrum, last = 1 */
  double L_star;
  int eta_iters_max;           /* largest eta fixed-point iteration count */
} ora_tables;

typedef struct {
  int mrw;                     /* 0/1 */
  double gamma;                /* MRW criterion */
  int n_int_min;               /* interactions in the cell before MRW */
  int n_inc;                   /* SED inclination bins */
  long long max_events;        /* per-packet cap */
  const double* frozen_T;      /* NULL: running (immediate reemission) mode */
  const double* coef_T;        /* NULL: the MRW takes D, kappa-bar and its criterion at
                                  the running cell T; else at these temperatures (a
                                  previous pass's), reemission still running */
} ora_opts;

typedef struct {
  int32_t fate;                /* 1 escaped, 2 hit the star, 3 capped */
  int32_t k;                   /* final wavelength bin */
  int64_t n_cross, n_scat, n_abs, n_mrw, n_draws;
  double x, y, z, u, v, w;     /* final position and direction */
} ora_packet_rec;

enum { ORA_C_ESCAPED = 0, ORA_C_STAR, ORA_C_CAPPED, ORA_C_CROSS, ORA_C_SCAT, ORA_C_ABS,
       ORA_C_MRW, ORA_C_LAUNCH, ORA_N_COUNTERS };

/* Philox4x32-10 (Salmon et al. 2011): in-place on ctr with the given key. */
void ora_philox4x32_10(uint32_t ctr[4], const uint32_t key[2]);
/* uniform doubles of packet `pid`, draws [d0, d0+n) of its stream */
void ora_uniforms(uint64_t seed, uint64_t pid, uint64_t d0, int64_t n, double* out);

/* Planck bin integrals at one temperature: Bbar[k] = int_bin B_nu dnu and
 * dBbar[k] = int_bin dB_nu/dT dnu. */
void ora_planck_bins(const double* lambda_edges, int n_lambda, double T, double* Bbar,
                     double* dBbar);

int ora_build_tables(const ora_model* m, ora_tables* t);   /* arrays preallocated */

int64_t ora_locate(const ora_model* m, double x, double y, double z);

/* T from absorbed power E of a cell of mass `mass` */
double ora_T_of_E(const ora_model* m, const ora_tables* t, double E, double mass);

/* reemission bin for an absorption that raised the cell from T_old to T_new
 * (T_old < 0: full spectrum at T_new), xi in (0,1) */
int ora_reemit_sample(const ora_model* m, const ora_tables* t, double T_old, double T_new,
                      double xi);
/* linear-in-T table value: which = 0 D*rho, 1 kappa-bar */
double ora_table_interp(const ora_tables* t, int which, double T);

/* MRW: solve P(s) = P0 for s = D c t / R0^2 */
double ora_mrw_escape_s(double P0);
double ora_mrw_survival(double s);

int ora_run(const ora_model* m, const ora_tables* t, const ora_opts* o,
            uint64_t n_packets, uint64_t n_total, uint64_t seed, uint64_t offset,
            double* E_abs, uint32_t* visits, uint32_t* n_abs, uint32_t* n_mrw_cell,
            double* sed, double* E_star, long long* counters, ora_packet_rec* recs,
            int64_t n_recs, double* E_half, double* path, double* mrw_path);
/* E_half (nullable): absorbed energy of the odd-numbered packets alone.
 * path (nullable) [n_cells][n_lambda]: eps times the length of every explicit
 * flight, by cell and bin; mrw_path (nullable) [n_cells]: eps times the path
 * c t of every MRW step. */

/* Mean intensity J [n_cells][n_lambda] (bin-integrated, erg/s/cm^2/sr) from
 * the path tallies; the MRW path is spread over the bins with the weights
 * eta/chi at T. */
void ora_mean_intensity(const ora_model* m, const double* T, const double* path,
                        const double* mrw_path, double* J);

/* Isotropic-equivalent luminosity per bin [n_inc][n_lambda] seen at
 * cos(inclination) cos_i, by ray tracing the source function of T and J
 * (nullable) on rings of n_sub per radial cell and n_phi azimuths, plus the
 * attenuated star. */
void ora_raytrace_sed(const ora_model* m, const ora_tables* t, const double* T, const double* J,
                      int n_inc, const double* cos_i, int n_sub, int n_phi, double* out);

/* The intensity per ray and bin of the same ray set, without the star
 * (Sect. 3.3: images from the source function), img
 * [n_inc][(n_r + 1) n_sub][n_phi][n_lambda]. */
void ora_raytrace_image(const ora_model* m, const ora_tables* t, const double* T,
                        const double* J, int n_inc, const double* cos_i, int n_sub, int n_phi,
                        double* img);

/* Visibility amplitudes [n_inc][n_base][n_lambda] of such an image and the
 * dimmed star, for baselines base [n_base][2] (length cm, position angle rad)
 * at distance D (cm). */
void ora_visibility(const ora_model* m, const ora_tables* t, const double* img, int n_inc,
                    const double* cos_i, int n_sub, int n_phi, int n_base, const double* base,
                    double distance, double* V);

/* Convergence statistic of the vertical-structure loop from one pass's
 * tallies (E_half: the odd-numbered packets' share; visits: packets entering
 * each cell, >= n_min to take part) against the previous pass's T_prev and
 * relative noise s2_prev (in/out, s2_prev < 0: cell not eligible).  out: R,
 * RMS relative change, RMS noise, cells compared. */
void ora_conv_stat(const ora_model* m, const ora_tables* t, const double* E_abs,
                   const double* E_half, const uint32_t* visits, int n_min, double* T_prev,
                   double* s2_prev, double out[4]);

void ora_cell_volumes(const ora_model* m, double* V);
void ora_update_T(const ora_model* m, const ora_tables* t, const double* E_abs, double* T);

/* PDA: region_in[c] = 1 marks candidate cells.  region_out: 1 solved, 2 left at
 * the MC value (no Dirichlet neighbour), 0 outside.  converged: the Picard
 * change fell below tol, or stalled below sqrt(tol). */
int ora_pda(const ora_model* m, const ora_tables* t, const double* T_mc,
            const uint8_t* region_in, double* T_out, uint8_t* region_out,
            int max_sweeps, double tol, int* n_sweeps, double* last_change, int* converged);

/* One linear PDA solve with the diffusion coefficient frozen at T_D (the
 * differentiation workload): u = T^4 on the region, Dirichlet T_bc outside. */
int ora_pda_linear(const ora_model* m, const ora_tables* t, const double* T_D,
                   const double* T_bc, const double* kscale, const uint8_t* region,
                   double* T_out);

/* Gradient of J(T) of the linear solve above w.r.t. log rho and the
 * extinction scale s of the listed cells (direct method; dJdT [n_cells];
 * outputs [n_req]). */
int ora_pda_grad_direct(const ora_model* m, const ora_tables* t, const double* T_D,
                        const double* T_bc, const double* kscale, const uint8_t* region,
                        const double* dJdT, const int* cells, int n_req, double* g_logrho,
                        double* g_kscale);

/* Nonlinear PDA for differentiation: Picard sweeps of the linear solve (D
 * from the current T) to the fixed point, Dirichlet T_bc on the other cells,
 * starting from T_bc; the stop rule of ora_pda.  T_out [n_cells]. */
int ora_pda_nl(const ora_model* m, const ora_tables* t, const double* T_bc,
               const double* kscale, const uint8_t* region, int max_sweeps, double tol,
               double* T_out, int* n_sweeps, double* last_change);

/* Gradient of J(T) of the nonlinear PDA above w.r.t. log rho and s of the
 * listed cells, by the direct method on its Jacobian (non-symmetric, with
 * the conductances' dependence on T): T_out [n_cells], outputs [n_req]. */
int ora_pda_nl_grad_direct(const ora_model* m, const ora_tables* t, const double* T_bc,
                           const double* kscale, const uint8_t* region, int max_sweeps,
                           double tol, const double* dJdT, const int* cells, int n_req,
                           double* T_out, double* g_logrho, double* g_kscale);

/* Vertical hydrostatic equilibrium of each radial shell for the cell
 * temperatures T [n_cells] (floored at T_floor), star mass M_star (g) and mean
 * molecular weight mu_mol; each shell keeps the mass of m->rho.  rho_out
 * [n_cells].  Shells with an optically thick (width >= 1 at the most opaque
 * wavelength) dust cell at T <= 0 keep m->rho; returns their number. */
int ora_hydrostatic(const ora_model* m, const double* T, double M_star, double mu_mol,
                    double T_floor, double* rho_out);

/* The PDA region of a finished Monte Carlo run (Sect. 2.2.1; Sect. 3.1): a
 * dust-bearing cell joins when fewer than visits_min packets entered it, or
 * when it is optically thick (width >= 1 at its most opaque wavelength) and
 * the relative photon noise of its temperature, 1 / (4 sqrt(N)) with N its
 * absorption events (absorptions plus MRW deposits), exceeds sigma_max
 * (sigma_max <= 0: that branch off).  region [n_cells] gets 1 or 0. */
void ora_pda_region(const ora_model* m, const uint32_t* visits, const uint32_t* n_abs,
                    const uint32_t* n_mrw, int visits_min, double sigma_max, uint8_t* region);

/* Energy one MRW step with escape variable s in a sphere of radius R0
 * deposits in cell c at the temperature Tc, per unit packet energy. */
double ora_mrw_deposit(const ora_model* m, const ora_tables* t, int64_t c, double Tc, double R0,
                       double s);

/* Directions after scattering n times by the phase function of model g_asym:
 * for packet a, from direction din[3a..3a+2] with the two draws u[2a], u[2a+1]
 * (cosine of the scattering angle, azimuth), into dout[3a..3a+2]. */
void ora_scatter_dirs(double g, const double* u, const double* din, double* dout, int n);

#ifdef __cplusplus
}
#endif
#endif
