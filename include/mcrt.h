/*
 * mcrt -- Monte Carlo radiative transfer in axisymmetric dust disks on AMD
 * Instinct MI355X (gfx950).
 *
 * The method is that of Min, Dullemond, Dominik, de Koter & Hovenier (2009),
 * "Radiative transfer in very optically thick circumstellar disks":
 * photon packets from the star are traced through an (r, theta) dust grid
 * with immediate reemission (Sect. 2.1, after Bjorkman & Wood 2001), the
 * modified random walk accelerates packets caught in optically thick cells
 * (Sect. 2.2.2, eqs. RW .. criterion, with the diffusion coefficient of
 * Sect. 2.2.3), and the partial diffusion approximation (Sect. 2.2.1,
 * eq. T diffusion) replaces the temperature of cells with few photons.
 *
 * Conventions for every entry point
 *  - Units are cgs.  Cell id = i_r * n_mu + j_mu; j_mu = 0 is the midplane row
 *    of the folded polar coordinate mu = |cos theta| (both hemispheres belong
 *    to one cell).
 *  - Descriptor structs and the host arrays they point to are read during the
 *    call only and may be freed afterwards (the library copies them).
 *  - Pointers named *_dev are device memory owned by the caller; the library
 *    never frees them.  Calls are asynchronous on the given stream unless
 *    stated; results are valid after the stream has been synchronised.
 *  - The context owns its device state (tallies, tables, solver scratch); it
 *    is released by mcrt_destroy.  A context may be used from one host thread
 *    at a time; calls on one context must be issued on one stream (or be
 *    ordered by the caller).
 *  - Return value: MCRT_OK (0) or a negative MCRT_E_* code; nothing aborts.
 *    mcrt_strerror() describes a code; mcrt_last_error() gives the text of
 *    the last failure on the calling thread.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MCRT_OK 0
#define MCRT_E_ARG (-1)             /* invalid argument or descriptor */
#define MCRT_E_OOM (-2)             /* device allocation failed */
#define MCRT_E_HIP (-3)             /* a HIP runtime call failed */
#define MCRT_E_NOT_CONVERGED (-4)   /* PDA solver hit its iteration cap */
#define MCRT_E_STUCK (-5)           /* packets hit the per-packet event cap (reported by the
                                       synchronous mcrt_batch_run; mcrt_trace only counts
                                       them, MCRT_GET_COUNTERS) */
#define MCRT_E_SINGULAR_REGION (-6) /* a PDA region part has no Dirichlet neighbour (solved
                                       without it: informational) */

#define MCRT_TAIL_CAP 8192          /* packets the hand-off buffer of a context holds */
#define MCRT_FP64 0                 /* tracking, tallies and inversion in FP64 */
#define MCRT_FP32 1                 /* packet geometry in FP32 cell-relative coordinates;
                                       tallies, inversion and PDA in FP64 */

typedef struct mcrt_ctx mcrt_ctx;

/* Folded spherical grid.  r_edges[n_r+1] strictly increasing (the inner
 * radius r_edges[0] bounds an empty hole around the star);
 * mu_edges[n_mu+1] strictly increasing from 0 (midplane) to 1 (pole). */
typedef struct {
  int32_t n_r, n_mu;
  const double* r_edges;
  const double* mu_edges;
} mcrt_grid;

/* The star: a uniform-brightness sphere radiating as a blackbody
 * (L = 4 pi R^2 sigma T^4), centred at the origin, R_star < r_edges[0]. */
typedef struct {
  double T_star, R_star;
} mcrt_star;

/* Dust: n_species grain types in fixed mass fractions (the same mixture in
 * every cell).  Opacities are constant within each wavelength bin;
 * lambda_edges[n_lambda+1] in cm, strictly increasing.  kappa_abs and
 * kappa_sca are [n_species][n_lambda] mass absorption / isotropic scattering
 * coefficients in cm^2/g. */
typedef struct {
  int32_t n_lambda, n_species;
  const double* lambda_edges;
  const double* kappa_abs;
  const double* kappa_sca;
  const double* mass_frac;
} mcrt_dust;

/* Run options (mcrt_default_options fills the defaults noted). */
typedef struct {
  int32_t precision;     /* MCRT_FP64 (default) or MCRT_FP32 */
  int32_t mrw;           /* 1: modified random walk on (default 0) */
  double gamma;          /* MRW start: d_min > gamma / (rho chi_R)  (default 3) */
  int32_t n_int_min;     /* interactions since entering the cell before MRW (20) */
  int32_t n_T;           /* temperature-table nodes, node 0 = 0 K (256) */
  double T_lo, T_hi;     /* first non-zero and last node, K (1, 1e4) */
  int32_t n_inc;         /* SED bins in |cos i| (10) */
  int64_t max_events;    /* per-packet event cap (2^30) */
  int32_t pda_visits;    /* PDA region: cells with fewer packet entries (100) */
  int32_t pda_max_sweeps;/* Picard sweeps on D(T) (50) */
  double pda_tol;        /* Picard stop: max |dT/T| (1e-8) */
  int32_t cg_max_iter;   /* per solve (20000) */
  double cg_tol;         /* preconditioned relative residual (1e-12) */
  int32_t mrw_coef_T;    /* 0: MRW uses the running cell T; 1: the T the
                            context holds when a trace starts, once mcrt_update_T
                            or mcrt_set_T has run (the previous pass's, PDA
                            included) (0) */
  int32_t block_size;    /* trace workgroup size: 0 or 512 (one workgroup per compute
                            unit, tables and emission CDF in up to 155 KB of LDS), or
                            with FP32 tracking 768 (the same LDS, 3 wavefronts per SIMD
                            instead of 2, registers capped at 168 with some spilled) or
                            256 (LDS capped at half, so two share a compute unit; the
                            CDF then stays in L2); batched runs use 512 (0) */
  int32_t blocks_per_cu; /* trace workgroups launched per compute unit (0: as many as
                            fit at once); more than fit wait for a free slot (0) */
  int32_t pda_solver;    /* 0 auto, 1 grid-wide CG kernels, 2 one workgroup per disk (0) */
  int32_t pda_precond;   /* CG preconditioner of the one-workgroup solver: 0 Jacobi (the
                            diagonal), 1 block Jacobi on the theta lines of each radius
                            (tridiagonal blocks, solved exactly) (1); the grid-wide solver
                            uses the diagonal */
  int64_t wave_events;   /* once every packet of a launch is handed out and no
                            more packets are live than the second launch has
                            wavefronts, packets that have had at least this many
                            events move to that launch, which runs each with all
                            64 lanes of a wavefront (same draws, same events);
                            0 = never (2048).  Batched runs use each disk's value
                            and one live count over all disks. */
  double g_asym;         /* asymmetry parameter g of scattering, |g| < 1 (0): the
                            scattering angle follows the Henyey-Greenstein phase
                            function, and the diffusion quantities (MRW and PDA)
                            take the isotropic-equivalent scattering opacity
                            (1 - g) sigma (Sect. 2.2.3).  Batched runs need 0. */
  double hydro_M_star;   /* > 0: each pass of mcrt_batch_run ends with the vertical
                            hydrostatic equilibrium of this disk for that star mass
                            (g), as mcrt_hydrostatic (0: off) */
  double hydro_mu;       /* mean molecular weight of that step (2.3) */
  double pda_sigma;      /* > 0: the PDA region also takes the opaque cells (optical width
                            >= 1 at the most opaque wavelength, rho chi_max times the
                            cell's largest width) whose temperature photon noise
                            1 / (4 sqrt(N)) exceeds this, N = absorptions + MRW deposits in
                            the cell, so every such cell without an absorption (T = 0)
                            joins (the second test of Sect. 3.1; the paper uses 0.05;
                            transparent cells are not diffusive); 0: visits rule only (0) */
  int32_t conv_split;    /* 1: mcrt_trace also tallies the absorbed energy of the
                            odd-numbered packets apart (MCRT_GET_E_HALF), from which
                            mcrt_convergence takes the photon noise (0).  The converging
                            batch loop keeps that tally whatever this says. */
  int32_t j_tally;       /* 1: the context holds path-length tallies (eps times every
                            explicit flight length by cell and bin, and eps times the
                            path c t of every MRW step by cell) that mcrt_trace and
                            batched passes fill, for mcrt_mean_intensity (0: none;
                            costs 8 (n_lambda + 1) bytes per cell) */
  int32_t wave_runahead; /* 1: with FP32 tracking, the whole-wavefront launch traces each
                            run of interactions inside a cell lane-parallel: the draws,
                            kinds, reemission bins and positions of up to 64 interactions,
                            the first face crossing or MRW start among them, and one
                            compare-and-swap of the cell's tally for the run's deposits;
                            the same events as one at a time from the same tally.  Not
                            with g_asym != 0 or j_tally.  0: one event at a time (0) */
  int32_t handoff_live;  /* a single-disk trace hands packets off once at most this many
                            are live; the hand-off launch's wavefronts then take them one
                            after another (0: as many as it has wavefronts; at most
                            MCRT_TAIL_CAP, the hand-off buffer) (0) */
} mcrt_options;

void mcrt_default_options(mcrt_options* opt);

/* Create a context on the current HIP device: copies the grid, star, dust and
 * the per-cell dust density rho[n_r*n_mu] (host, g/cm^3), and builds the FP64
 * tables of Sect. 2.2.3 (Planck bin integrals, emission CDF, diffusion
 * coefficient and mean absorption opacity of the MRW).  Synchronous. */
int mcrt_setup(mcrt_ctx** out, const mcrt_grid* grid, const mcrt_star* star,
               const mcrt_dust* dust, const double* rho, const mcrt_options* opt);
void mcrt_destroy(mcrt_ctx* ctx);

/* Zero the absorbed-energy, visit, absorption, MRW, SED and event tallies. */
int mcrt_reset(mcrt_ctx* ctx, hipStream_t stream);

/* Trace packets [offset, offset + n_packets) of a run of n_total packets,
 * each carrying L_star / n_total (Sect. 2.1).  Packet p draws its random
 * numbers from Philox4x32-10 keyed by seed, counter (p, draw index).
 * Absorptions re-emit immediately from the difference of the cell's emission
 * spectrum before and after the absorption; with mrw=1 packets in optically
 * thick cells take modified-random-walk steps (Sect. 2.2.2).  Tallies add to
 * the context's.  frozen_T_dev (nullable, [n_cells] K): re-emit from the
 * full spectrum at these fixed temperatures instead (no coupling between
 * packets; a test mode).  rec_dev (nullable): mcrt_packet_rec for packets
 * [offset, offset + n_recs).  A packet that reaches max_events events ends
 * there and is counted as capped (MCRT_GET_COUNTERS, fate 3 in its record);
 * the call does not wait for the stream, so it cannot report that itself.
 * Errors: MCRT_E_ARG for a null context, n_total = 0 or a packet range
 * outside [0, n_total); MCRT_E_HIP if a launch fails. */
typedef struct {
  int32_t fate;                    /* 1 escaped, 2 hit the star, 3 capped */
  int32_t k;                       /* final wavelength bin */
  int64_t n_cross, n_scat, n_abs, n_mrw, n_draws;
  double x, y, z, u, v, w;         /* final position and direction */
} mcrt_packet_rec;

int mcrt_trace(mcrt_ctx* ctx, uint64_t n_packets, uint64_t n_total, uint64_t seed,
               uint64_t offset, const double* frozen_T_dev, mcrt_packet_rec* rec_dev,
               int64_t n_recs, hipStream_t stream);

/* Radiative equilibrium per cell (Sect. 2.1: with immediate reemission a
 * cell's temperature follows from the energy it absorbed): 4 pi m_i G(T_i) =
 * E_i with G the emission per unit mass and steradian (the sum over bins of
 * kappa_k Bbar_k(T)), linear in T between table nodes; T = 0 where nothing was
 * absorbed.  Updates the context's T and, if T_dev != NULL, copies it there
 * ([n_cells] double).  Errors: MCRT_E_ARG for a null context, MCRT_E_HIP if the
 * launch fails. */
int mcrt_update_T(mcrt_ctx* ctx, double* T_dev, hipStream_t stream);

/* Partial diffusion approximation (Sect. 2.2.1): solve div(D grad T^4) = 0
 * on the region (mask_dev[c] = 1; NULL: cells with fewer than pda_visits
 * entries, and the pda_sigma test), Dirichlet T from the Monte Carlo
 * temperature of the neighbouring dust cells that have one (a neighbour in
 * which nothing was absorbed, T = 0, gives no boundary value: its face carries
 * no flux), D = 1/(3 rho chi_R) with chi_R the Rosseland mean of the total
 * extinction (the diffusion coefficient of Sect. 2.2.3 with isotropic
 * scattering), Picard iteration on D(T), preconditioned CG (pda_precond:
 * exact theta-line blocks, or the diagonal).  Updates the context's T.
 * stats (host, nullable) receives sweeps, CG iterations and residuals; waits
 * for the stream.  MCRT_E_NOT_CONVERGED if CG hits cg_max_iter or the Picard
 * sweeps end unconverged (stats.converged);
 * MCRT_E_SINGULAR_REGION (informational) if a part of the region has no
 * Dirichlet neighbour (left at its Monte Carlo T, flagged 2). */
typedef struct {
  int32_t sweeps, cg_iters_total, cg_iters_last, n_region, n_isolated;
  double last_change, last_residual;
  int32_t converged;     /* 1: the Picard sweeps' largest relative change of T fell
                            below pda_tol, or stalled below sqrt(pda_tol) (a sweep
                            that changes T no less than the one before has reached
                            the rounding floor of the linear solve) */
} mcrt_pda_stats;

int mcrt_pda_solve(mcrt_ctx* ctx, const uint8_t* mask_dev, mcrt_pda_stats* stats,
                   hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve of
 * mcrt_pda_solve by its one-workgroup solver (pda_solver = 2), with its work
 * arrays in a fixed device array of the library -- about 4.5 MB on each
 * device the library runs on, held until the process ends -- where
 * mcrt_pda_solve allocates them on first use.  Grids of at most
 * MCRT_NOALLOC_MAX_CELLS cells (else MCRT_E_ARG, nothing launched); the
 * context's device must be current (else MCRT_E_ARG).  Every call on a device
 * shares that array, so calls that overlap in time on one device race.  A
 * linear solve kept for mcrt_pda_adjoint stays intact.  Same region, result,
 * statistics and return codes as mcrt_pda_solve with pda_solver = 2; waits for
 * the stream. */
#define MCRT_NOALLOC_MAX_CELLS 32768
int mcrt_pda_solve_noalloc(mcrt_ctx* ctx, const uint8_t* mask_dev, mcrt_pda_stats* stats,
                           hipStream_t stream);

/* Linear PDA for differentiation: eq. T diffusion on the cells with
 * mask_dev[c] = 1 (parts without a Dirichlet neighbour are left out and
 * flagged 2 in MCRT_GET_REGION) with the diffusion coefficient frozen at a
 * given temperature field, D_c = (D rho)(T_D,c) / (rho_c s_c): one linear
 * solve of the finite-volume system for u = T^4 (Jacobi-PCG), Dirichlet T_bc
 * on the other cells.  rho_dev (nullable: the context's density) and
 * kscale_dev (nullable: s = 1) are [n_cells] doubles; s scales the mass
 * extinction of a cell.  T_out_dev [n_cells] receives T (T_bc outside the
 * region).  The solution is kept for mcrt_pda_adjoint.  Waits for the stream. */
int mcrt_pda_linear(mcrt_ctx* ctx, const uint8_t* mask_dev, const double* rho_dev,
                    const double* kscale_dev, const double* T_D_dev, const double* T_bc_dev,
                    double* T_out_dev, mcrt_pda_stats* stats, hipStream_t stream);

/* Adjoint of the last mcrt_pda_linear: given dJ/dT [n_cells] for any
 * objective J of its output T, writes dJ/d(log rho_c) to g_logrho_dev and
 * (nullable) dJ/ds_c to g_kscale_dev, both [n_cells], through the
 * dependence of the diffusion coefficient (the explicit dependence of J on
 * rho, e.g. through cell masses, is the caller's).  One more symmetric solve.
 * Waits for the stream. */
int mcrt_pda_adjoint(mcrt_ctx* ctx, const double* dJdT_dev, double* g_logrho_dev,
                     double* g_kscale_dev, hipStream_t stream);

/* Nonlinear PDA for differentiation: eq. T diffusion (Sect. 2.2.1) with the
 * diffusion coefficient of the temperature itself, D_c = (D rho)(T_c) /
 * (rho_c s_c) (Sect. 2.2.3), solved by Picard sweeps of the linear solve of
 * mcrt_pda_linear -- D from the T of the previous sweep, the first from
 * T_bc -- until the largest relative change of T falls below pda_tol (or
 * stalls below its square root).  Arguments as mcrt_pda_linear without T_D;
 * T_bc [n_cells] gives the Dirichlet values outside the region and the
 * starting T inside; T_out_dev [n_cells] receives T.  stats (nullable, host):
 * sweeps, CG iterations in all, region size, last change, converged.  The
 * last sweep's linear solve is kept for mcrt_pda_nonlinear_adjoint (and is
 * what mcrt_pda_adjoint would differentiate).  MCRT_E_NOT_CONVERGED if the
 * sweeps or a CG solve hit their caps (T_out holds the last sweep).  Waits
 * for the stream. */
int mcrt_pda_nonlinear(mcrt_ctx* ctx, const uint8_t* mask_dev, const double* rho_dev,
                       const double* kscale_dev, const double* T_bc_dev, double* T_out_dev,
                       mcrt_pda_stats* stats, hipStream_t stream);

/* Adjoint of the last mcrt_pda_nonlinear: dJ/d(log rho_c) into g_logrho_dev
 * and (nullable) dJ/ds_c into g_kscale_dev, [n_cells] each, given dJ/dT
 * [n_cells] for an objective J of its output.  At the fixed point the
 * residual of the finite-volume system vanishes, so the adjoint solves
 * J^T lambda = dJ/du with the Jacobian J = dr/du of u = T^4, which holds the
 * conductances' dependence on T through D(T) (not symmetric: BiCGSTAB with a
 * diagonal preconditioner, to cg_tol, at most cg_max_iter iterations), and
 * the gradient is -lambda . dr/dp as in mcrt_pda_adjoint.  stats (nullable):
 * iterations and relative residual.  MCRT_E_ARG without a preceding
 * mcrt_pda_nonlinear on this context (or after any call that reused its
 * scratch), MCRT_E_NOT_CONVERGED at the iteration cap.  Waits for the
 * stream. */
int mcrt_pda_nonlinear_adjoint(mcrt_ctx* ctx, const double* dJdT_dev, double* g_logrho_dev,
                               double* g_kscale_dev, mcrt_pda_stats* stats, hipStream_t stream);

/* The spectral energy distribution from the escaping packets (Sect. 3.3
 * studies it at fixed inclination): escaped luminosity per wavelength bin and
 * |cos i| bin of the packet's direction, sed_dev [n_lambda][n_inc] double,
 * erg/s (not divided by the solid angle; each bin is 1/n_inc of the folded
 * |cos i| range).  Errors: MCRT_E_ARG for a null argument. */
int mcrt_sed(mcrt_ctx* ctx, double* sed_dev, hipStream_t stream);

/* Cell of each point on the axisymmetric (r, theta) grid the transport steps
 * through (Sect. 2.1; the disk of Sect. 2.4): xyz_dev [n][3] double, cell_dev
 * [n] int32 (-1 outside the grid).  r^2 = (x*x + y*y) + z*z and z*z against
 * mu_e^2 r^2, no fused multiply-add, half-open cells [r_e, r_e+1) x
 * [mu_e, mu_e+1).  Errors: MCRT_E_ARG for n < 0 or a null pointer with n > 0. */
int mcrt_locate(mcrt_ctx* ctx, const double* xyz_dev, int64_t n, int32_t* cell_dev,
                hipStream_t stream);

#define MCRT_GET_E_ABS 0    /* double [n_cells], erg/s absorbed */
#define MCRT_GET_VISITS 1   /* uint32 [n_cells], packet entries */
#define MCRT_GET_N_ABS 2    /* uint32 [n_cells], absorption events */
#define MCRT_GET_N_MRW 3    /* uint32 [n_cells], MRW steps */
#define MCRT_GET_T 4        /* double [n_cells], K */
#define MCRT_GET_REGION 5   /* uint8 [n_cells]: 1 PDA-solved, 2 isolated, 0 outside */
#define MCRT_GET_COUNTERS 6 /* uint64 [10]: escaped, star, capped, crossings,
                               scatterings, absorptions, MRW steps, launches, packets
                               handed off to the whole-wavefront launch, interactions
                               of those traced lane-parallel (wave_runahead) */
#define MCRT_GET_E_STAR 7   /* double [1], erg/s absorbed by the star */
#define MCRT_GET_RHO 9      /* double [n_cells], the context's current dust density */
#define MCRT_GET_TABLES 8   /* double: T nodes [n_T], cdf [n_T][n_lambda], D*rho [n_T],
                               kappa-bar [n_T], star cdf [n_lambda], L_star [1] */
#define MCRT_GET_HYDRO_COLD 10 /* uint32 [1]: shells the last hydrostatic step left
                                  unchanged (an opaque dust cell at T <= 0) */
#define MCRT_GET_E_HALF 11  /* double [n_cells], erg/s absorbed from the odd-numbered
                               packets alone (kept with conv_split, or by
                               mcrt_batch_converge) */
#define MCRT_GET_PATH 12    /* double [n_cells][n_lambda], eps times the explicit flight
                               lengths (j_tally; else MCRT_E_ARG) */
#define MCRT_GET_MRW_PATH 13 /* double [n_cells], eps times the MRW steps' c t (j_tally) */

/* Copy a context array into caller device memory (async, device to device):
 * the Monte Carlo tallies of Sect. 2.1 (absorbed energy, visits, absorption
 * and MRW counts), the temperature, the PDA region of Sect. 2.2.1, the event
 * counters, the tables of Sect. 2.2.3 and the density.  Errors: MCRT_E_ARG for
 * a null argument or an unknown `what`. */
int mcrt_get(mcrt_ctx* ctx, int what, void* dst_dev, hipStream_t stream);
/* Size in bytes of what mcrt_get(what) writes. */
int64_t mcrt_get_size(mcrt_ctx* ctx, int what);

/* Overwrite the context's temperature (e.g. with a PDA result or a test
 * field): T_dev [n_cells] double. */
int mcrt_set_T(mcrt_ctx* ctx, const double* T_dev, hipStream_t stream);

/* Vertical hydrostatic equilibrium (Sect. 2.5, eq. balance: dP/dz =
 * -rho G M_star z / R^3, P = k rho T / (mu_mol m_p)) for the context's
 * current temperature (floored at T_lo): along each radial shell at its mid
 * radius r, through the cell centres (z = r mu, R = r sqrt(1 - mu^2)),
 * ln(rho T) falls by mu_mol m_p G M_star / k times the trapezoidal integral
 * of z / (R^3 T) between consecutive centres, and each shell keeps its mass
 * (the surface density stays fixed).  Replaces the context's density (and
 * the cell masses the temperature inversion uses); rho_dev (nullable)
 * [n_cells] double receives a copy.  M_star in g.  One iteration of the
 * method's vertical-structure loop; tracing again gives the next T.  A shell
 * holding an opaque dust cell (optical width >= 1, as for pda_sigma) at T <= 0
 * has no temperature to balance and keeps its density (counted in
 * MCRT_GET_HYDRO_COLD): the region rule with pda_sigma > 0 fills such cells by
 * the PDA first, as the paper does (Sect. 3.4, Case 3).  Transparent cold
 * cells are floored at T_lo like any lower temperature.
 * Errors: MCRT_E_ARG for a null context, M_star < 0 or mu_mol <= 0. */
int mcrt_hydrostatic(mcrt_ctx* ctx, double M_star, double mu_mol, double* rho_dev,
                     hipStream_t stream);

/* Batched passes over many disks: for each of n_iter passes, clear the
 * tallies of every context, trace n_packets[d] packets of context d (seed
 * seeds[d] + (pass << 32); each packet carries L_star / n_packets[d]) with
 * ALL disks in one persistent launch (workgroups shared out by packet
 * count; packets still going once their disk's packets are all out continue
 * in a second launch whose workgroups are shared out by those packets),
 * invert the temperatures, and solve each disk's PDA on its
 * low-visit cells with one workgroup per disk.  Contexts whose mrw_coef_T is
 * 1 take the MRW coefficients of pass k from the temperature after pass k-1
 * (for the first pass: the T the context holds, if it holds one).
 * use_graph != 0 captures all passes in one HIP graph and submits it once.
 * Contexts whose hydro_M_star is > 0 end every pass with the vertical
 * hydrostatic equilibrium of their density for that pass's final T (the
 * method's vertical-structure loop, Sect. 2.5).
 * Every context must use MCRT_FP32 with g_asym = 0 and live on the current
 * device (else MCRT_E_ARG).  stats
 * (host, nullable) receives each disk's PDA statistics of the last pass.
 * Synchronous: returns after the stream has drained, then reports, over every
 * pass and disk: MCRT_E_NOT_CONVERGED if a PDA solve hit cg_max_iter or its
 * Picard sweeps did not reach pda_tol, else MCRT_E_STUCK if packets hit
 * max_events (the tallies of the last pass stay readable either way).  A
 * linear PDA solve kept for mcrt_pda_adjoint is dropped (its scratch is
 * reused).  The n-iteration outer loop of the method (Sect. 2.5: radiative
 * transfer repeated on an updated structure) run for a batch of models. */
int mcrt_batch_run(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets,
                   const uint64_t* seeds, int n_iter, int use_graph, mcrt_pda_stats* stats,
                   hipStream_t stream);

/* Convergence statistic of the vertical-structure loop (Sect. 2.5: the mean
 * change of the temperature structure between two consecutive passes,
 * against the error that the Monte Carlo statistics give it; converged below
 * 3 sigma), from the context's current tallies (a pass traced with
 * conv_split = 1) and the values the previous call stored in the context.
 * Per dusty cell entered by >= n_min packets with E > 0: T = T(E) (the
 * inversion of mcrt_update_T); the odd- and even-numbered packets are two
 * independent half-size runs, so the relative variance of E is
 * ((2 E_half - E) / E)^2, and that of T is (dlnT/dlnE)^2 times it, the slope
 * a central difference of T(E) over E (1 +- 1e-4).  Over the cells eligible
 * in this pass and the previous one,
 *   R = sqrt(sum x^2 / sum (s2 + s2_prev)),  x = (T - T_prev) / T.
 * first != 0: no previous pass (nothing compared, R = 0).  Stores this pass's
 * T and s2 for the next call.  out_host (nullable) [4] double: R, the RMS of
 * x, the RMS noise sqrt(mean(s2 + s2_prev)), the cells compared; when given,
 * the call waits for the stream.  Errors: MCRT_E_ARG for a null context or
 * n_min < 1. */
int mcrt_convergence(mcrt_ctx* ctx, int32_t n_min, int32_t first, double* out_host,
                     hipStream_t stream);

/* The PDA region rule of Sect. 3.1 evaluated on the context's current
 * tallies with the given parameters, whatever the context's own options say:
 * mask_dev[c] = 1 for dusty cells entered by fewer than visits_min packets
 * (visits_min <= 0: no visits test), or, with sigma_max > 0, opaque cells
 * (optical width >= 1, as for pda_sigma) whose temperature noise
 * 1 / (4 sqrt(N)) exceeds sigma_max or that absorbed nothing; else 0.  Pass
 * the mask to mcrt_pda_solve to solve a region of another rule on the same
 * tallies.  mask_dev [n_cells] uint8.  Asynchronous.  Errors: MCRT_E_ARG for
 * a null argument or sigma_max < 0. */
int mcrt_region_mask(mcrt_ctx* ctx, int32_t visits_min, double sigma_max, uint8_t* mask_dev,
                     hipStream_t stream);

/* Mean intensity of the radiation field per cell and bin (Sect. 2.3: the
 * source function the observables integrate), from the path-length tallies
 * of the traces since the last reset (j_tally = 1, else MCRT_E_ARG):
 *   J_k = (P_k + w_k P_mrw) / (4 pi V),
 * P_k the explicit flights' eps * length at bin k, P_mrw the MRW steps'
 * eps * c t, spread over the bins as a walk spends its path: w_k = eta_k /
 * chi_k normalised, the weighting that defines kappa-bar (Sect. 2.2.3), which
 * at the fixed point of eq. eta nu iter is dB_k/dT over its sum, at the
 * cell's temperature T_dev [n_cells] (nullable: the context's T).  J_dev
 * [n_cells][n_lambda] double, erg s^-1 cm^-2 sr^-1 integrated over the bin.
 * Asynchronous.  Errors: MCRT_E_ARG for a null context or J_dev, or no
 * path tallies. */
int mcrt_mean_intensity(mcrt_ctx* ctx, const double* T_dev, double* J_dev, hipStream_t stream);

/* Spectral energy distribution by integration of the source function
 * (Sect. 2.3; the paper takes T before the PDA, Sect. 3.3): the
 * isotropic-equivalent luminosity per bin (4 pi D^2 times the flux at
 * distance D, erg/s per bin) seen at n_inc inclinations cos_i_host[q]
 * (cosine of the angle to the pole, host, in [0, 1]), from the formal solution
 * dI/ds = rho chi (S - I) along parallel rays, with the isotropic-scattering
 * source function S_k = (kappa_abs,k Bbar_k(T) + kappa_sca,k J_k) / chi_k
 * constant in each cell, I <- I e^(-dtau) + S (1 - e^(-dtau)) from the far
 * side to the near one.  Rays: the image plane in rings -- the central hole
 * [0, r_0] and each radial cell [r_i, r_i+1] cut into n_sub equal rings --
 * and n_phi azimuths phi = (p + 1/2) pi / n_phi on one side of the plane of
 * the line of sight and the pole, each standing also for its mirror image,
 * a ray at the ring's mid radius carrying the area pi (b_hi^2 - b_lo^2) /
 * n_phi.  The star adds its luminosity in the bin (the launch spectrum)
 * times e^(-tau) along the line of sight from its centre.  T_dev [n_cells]
 * (nullable: the context's T); J_dev [n_cells][n_lambda] (nullable: no
 * scattering source).  L_dev [n_inc][n_lambda] double, overwritten.  The
 * context keeps a source-function buffer of 8 n_cells n_lambda bytes after
 * its first call.  Asynchronous.  Errors: MCRT_E_ARG for a null context or
 * L_dev, n_inc outside [1, 64], n_sub < 1, n_phi < 1, a cos_i outside
 * [0, 1], more than 512 bins, or g_asym != 0 (the source function here
 * scatters isotropically); MCRT_E_OOM. */
int mcrt_raytrace_sed(mcrt_ctx* ctx, const double* T_dev, const double* J_dev, int32_t n_inc,
                      const double* cos_i_host, int32_t n_sub, int32_t n_phi, double* L_dev,
                      hipStream_t stream);

/* Ray-traced images (Sect. 3.3: images among the observables from the source
 * function, the Monte Carlo T before the PDA): the intensity with which each
 * ray of mcrt_raytrace_sed's ray set reaches the observer, per bin
 * (erg s^-1 cm^-2 sr^-1 integrated over the bin), without the star.  Same
 * arguments, source function and formal solution as mcrt_raytrace_sed.
 * I_dev [n_inc][(n_r + 1) n_sub][n_phi][n_lambda] double, overwritten: ray
 * (q, ring, p) runs towards the observer along n = (sin i, 0, cos i),
 * cos i = cos_i[q], through b (cos phi e1 + sin phi e2), e1 = (cos i, 0,
 * -sin i), e2 = (0, 1, 0), with b the mid radius of ring `ring` (ring =
 * c n_sub + part: c = 0 the hole [0, r_0], c >= 1 the radial cell
 * [r_(c-1), r_c], cut into n_sub equal rings) and phi = (p + 1/2) pi / n_phi;
 * the mirror image (-phi) has the same intensity.  Sum of
 * 4 pi I pi (b_hi^2 - b_lo^2) / n_phi over the rays, plus the dimmed star, is
 * mcrt_raytrace_sed.  Asynchronous.  Errors: as mcrt_raytrace_sed. */
int mcrt_raytrace_image(mcrt_ctx* ctx, const double* T_dev, const double* J_dev, int32_t n_inc,
                        const double* cos_i_host, int32_t n_sub, int32_t n_phi, double* I_dev,
                        hipStream_t stream);

/* Visibility amplitudes of a ray-traced image (Sect. 3.4 shows visibility
 * curves of the disks: the Fourier transform of the image at a baseline's
 * spatial frequency over the total flux).  I_dev: the image of
 * mcrt_raytrace_image with the same n_inc, cos_i_host, n_sub and n_phi
 * (device, not modified); the star joins as a point at the centre with its
 * luminosity per bin dimmed along the line of sight.  Ray (ring, p) sits at
 * x = b cos phi, y = b sin phi on the image-plane axes of mcrt_raytrace_image
 * and stands also for its mirror image at -y, each carrying half of
 * pi (b_hi^2 - b_lo^2) / n_phi.  baselines_host [n_base][2]: projected length
 * (cm) and position angle (radians from the x axis towards y).  At the
 * distance `distance` (cm), bin k is sampled at s = B / (lambda_k distance)
 * cycles per cm, lambda_k the bin's geometric centre:
 *   V = |sum A I e^(-2 pi i s (x cos theta + y sin theta)) + L_star,k / 4 pi|
 *       / (sum A I + L_star,k / 4 pi).
 * V_dev [n_inc][n_base][n_lambda] double, overwritten.  The partial sums
 * use the context's source-function buffer (8 n_cells n_lambda bytes,
 * allocated on first use), so a visibility call and a ray tracing call on one
 * context must not overlap.  Asynchronous.  Errors: MCRT_E_ARG for null
 * pointers, n_inc, n_base outside [1, 64], n_sub or n_phi < 1, a cos_i
 * outside [0, 1], a negative or non-finite baseline, distance <= 0, more than
 * 512 bins, or n_inc n_base > n_cells / 3; MCRT_E_OOM. */
int mcrt_visibility(mcrt_ctx* ctx, const double* I_dev, int32_t n_inc, const double* cos_i_host,
                    int32_t n_sub, int32_t n_phi, int32_t n_base, const double* baselines_host,
                    double distance, double* V_dev, hipStream_t stream);

/* Outcome of mcrt_batch_converge for one disk. */
typedef struct {
  int32_t passes;          /* passes run */
  int32_t converged_pass;  /* first pass (0-based) whose R fell below the threshold, -1 */
  double R_last;           /* the statistic of the last pass (0 after a single pass) */
  double dT_rms;           /* its RMS relative change of T */
  double noise_rms;        /* its RMS photon noise of that change */
  int32_t cells;           /* cells it compared */
} mcrt_conv_stats;

/* The vertical-structure loop run to convergence (Sect. 2.5): the passes of
 * mcrt_batch_run (pass k with seeds[d] + (k << 32), one HIP graph per pass
 * when use_graph != 0), each followed on the device by mcrt_convergence for
 * every disk (n_min packets per cell; the split tally is kept for the call),
 * until every disk's statistic R has fallen below `threshold` (the paper's
 * 3) or max_iter passes have run; at least 2 passes.  Disks that converge
 * before the others keep iterating with them.  conv (host, nullable)
 * [n_disks]; R_hist (host, nullable) [n_disks][max_iter] receives each pass's
 * R (0 for pass 0, -1 for passes not run); stats as for mcrt_batch_run.
 * Returns as mcrt_batch_run, or MCRT_E_NOT_CONVERGED when some disk did not
 * converge within max_iter passes (its conv entry says which).  Errors:
 * MCRT_E_ARG as for mcrt_batch_run, or max_iter < 2, threshold <= 0. */
int mcrt_batch_converge(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets,
                        const uint64_t* seeds, int max_iter, int32_t n_min, double threshold,
                        int use_graph, mcrt_pda_stats* stats, mcrt_conv_stats* conv,
                        double* R_hist, hipStream_t stream);

/* The PDA step of mcrt_batch_run alone (Sect. 2.2.1, eq. T diffusion; the
 * region rule of each context, Sect. 3.1): every context's region solved from
 * the temperature the context holds (Dirichlet data and first guess), one
 * workgroup per disk, all disks in one launch, in place on each context's T
 * and region.  Every context needs pda_visits > 0 or pda_sigma > 0 and the
 * current device (else MCRT_E_ARG).  stats (host, nullable) [n_disks].
 * Synchronous.  Returns MCRT_E_NOT_CONVERGED if a solve hit a cap, else
 * MCRT_E_SINGULAR_REGION (informational) if a region part of some disk had no
 * Dirichlet neighbour.  A linear PDA solve kept for mcrt_pda_adjoint is
 * dropped. */
int mcrt_batch_pda(mcrt_ctx** ctxs, int n_disks, mcrt_pda_stats* stats, hipStream_t stream);

const char* mcrt_strerror(int code);
const char* mcrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
