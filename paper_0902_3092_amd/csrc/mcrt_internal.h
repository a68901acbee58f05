// Internal declarations of the mcrt library: the context, the device-side
// parameter blocks and the kernel launchers.  Not part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "mcrt.h"

namespace mcrt {

// Counters, in the order of MCRT_GET_COUNTERS.
enum { C_ESCAPED = 0, C_STAR, C_CAPPED, C_CROSS, C_SCAT, C_ABS, C_MRW, C_LAUNCH, C_HANDED,
       C_RUN, N_COUNTERS };

// Nodes of the MRW escape-time table: s as a function of v = ln(-ln P0).
constexpr int MRW_TAB_N = 512;
constexpr double MRW_TAB_V0 = -38.0;
constexpr double MRW_TAB_V1 = 4.0;

// Read-only model data on the device (FP64).
struct DevModel {
  int n_r, n_mu, n_lambda, n_T, n_inc;
  const double* r_edges;   // [n_r+1]
  const double* r2;        // [n_r+1] r_e * r_e
  const double* mu_edges;  // [n_mu+1]
  const double* mu2;       // [n_mu+1] mu_e * mu_e
  const double* smu;       // [n_mu+1] sqrt(1 - mu_e^2)
  const double* rho;       // [n_cells]
  const double* inv4pim;   // [n_cells] 1 / (4 pi m), 0 for empty cells
  const double* Tn;        // [n_T] table nodes
  const double* cdf;       // [n_T][n_lambda] cumulative kappa_k Bbar_k(T_n)
  const double* G;         // [n_T] cdf[n][n_lambda-1]
  const double* Drho;      // [n_T] D * rho
  const double* kbar;      // [n_T] mean absorption opacity of an MRW step
  const double* star_cdf;  // [n_lambda]
  const double* chi;       // [n_lambda] extinction per mass
  const double* omega;     // [n_lambda] albedo
  const double* mrw_tab;   // [MRW_TAB_N] s at nodes of v
  const float* cdf32;      // [n_T][n_lambda] FP32 copy
  const float* star_cdf32; // [n_lambda]
  const float* chi32;      // [n_lambda]
  const float* omega32;    // [n_lambda]
  const int* g_guide;      // [N_GUIDE] largest n with G[n] <= exp(lnG0 + b / inv_du)
  const double* inv_dT;    // [n_T] 1 / (T[n+1] - T[n])  (last entry unused)
  const double* g_slope;   // [n_T] (T[n+1] - T[n]) / (G[n+1] - G[n])
  const double* cell_len;  // [n_cells] largest width of the cell (radial, or polar with
                           // the midplane row spanning both hemispheres)
  double chi_max;          // largest extinction per mass over the bins: a cell's optical
                           // width at its most opaque wavelength is (rho chi_max) cell_len
  const double* lam;       // [n_lambda+1] wavelength bin edges, cm
  const double* planck_a;  // [64] series coefficients of t / (e^t - 1)
  double lnT_lo, inv_dlnT; // T nodes 1..n_T-1 = T_lo exp((n-1) dlnT)
  double lnG0, inv_du;     // guide bins over ln g
  double R_star, L_star;
};

constexpr int N_GUIDE = 1024;

// Mutable per-run tallies.
struct DevTally {
  double* E_abs;               // [n_cells]
  uint32_t* visits;            // [n_cells]
  uint32_t* n_abs;             // [n_cells]
  uint32_t* n_mrw;             // [n_cells]
  double* sed;                 // [n_lambda][n_inc]
  double* E_star;              // [1]
  unsigned long long* counters;// [N_COUNTERS]
  double* E_half;              // [n_cells] the odd-numbered packets' share (null: not kept)
  double* path;                // [n_cells][n_lambda] eps * flight length (null: not kept)
  double* mrw_path;            // [n_cells] eps * c t of the MRW steps (with path)
};

struct TraceArgs {
  DevModel m;
  DevTally t;
  double eps;                  // L_star / n_total
  uint32_t key0, key1;
  uint64_t offset, n_packets;
  unsigned long long* next;    // work counter, zeroed before the launch
  int mrw, n_int_min;
  double gamma;
  long long max_events;
  const double* frozen_T;      // nullable
  const double* T_coef;        // nullable: fixed T for the MRW coefficients
  mcrt_packet_rec* recs;       // nullable
  int64_t n_recs;
  int vis_lds;                 // FP32 path: visit counts in a per-workgroup LDS histogram
  // hand-off of long packets to the whole-wavefront tail launch (tail null: off)
  long long wave_events;       // events after which a packet is handed off
  void* tail;                  // [tail_cap] packet states
  unsigned int* tail_count;    // states written (may exceed tail_cap: the rest stay)
  unsigned int* tail_next;     // next state for a tail wavefront to take (after tail_count)
  int tail_cap;
  // hand-offs wait until few packets are left: once the launch's packets are
  // all out, each wavefront adds its live packets to *live (and itself to
  // *waves_in) and subtracts those that leave; packets are handed off once
  // all n_waves wavefronts are counted and *live <= live_handoff
  long long* live;
  unsigned int* waves_in;
  unsigned int n_waves, live_handoff;  // live_handoff from the options: 0 = the launch's waves
  double g_asym;               // Henyey-Greenstein asymmetry parameter (0: isotropic)
  int runahead;                // FP32 whole-wavefront mode: runs of interactions lane-parallel
};
constexpr int TAIL_STATE_BYTES = 512;
constexpr int TAIL_CAP = 8192;

// Per-context outcome counters that no single call can report itself: kernels
// of a batched pass (or a graph) run long after the host call returned.
struct DevHealth {
  unsigned int hydro_cold;     // shells the last hydrostatic step left unchanged
  unsigned int pda_fails;      // batched PDA solves that hit a cap since the batch began
  unsigned long long capped;   // packets capped at max_events, summed over batched passes
};

}  // namespace mcrt

struct mcrt_ctx {
  int device = 0;
  int n_cu = 0;
  mcrt_options opt;
  int n_r = 0, n_mu = 0, n_lambda = 0, n_cells = 0;
  double L_star = 0.0;
  mcrt::DevModel m{};
  mcrt::DevTally t{};
  // owned device allocations
  double* d_T = nullptr;        // current temperature
  double* d_T_prev = nullptr;   // temperature of the previous pass (MRW coefficients)
  uint8_t* d_region = nullptr;
  mcrt::DevHealth* d_health = nullptr;
  double* d_E_half = nullptr;   // split tally (inside the cleared tally span)
  double* d_conv = nullptr;     // convergence state: T [n_cells], s2 [n_cells], sums [8]
  void* d_paths = nullptr;      // path tallies (j_tally): path [n_cells][n_lambda], mrw [n_cells]
  double* d_src = nullptr;      // source function of the ray tracer [n_cells][n_lambda]
  unsigned long long* d_next = nullptr;
  void* d_tail = nullptr;             // hand-off buffer of long packets (TAIL_CAP states + count)
  void* d_blob = nullptr;       // model + tables
  void* d_tally_blob = nullptr;
  void* d_pda_blob = nullptr;   // PDA solver scratch
  size_t pda_bytes = 0;
  bool have_T_prev = false;
  void* d_lin_args = nullptr;        // argument slot of the linear PDA / adjoint
  const double* lin_rho = nullptr;   // density of the last linear forward
  bool lin_ready = false;
  bool nl_ready = false;               // the kept linear solve ends a nonlinear forward
  void* d_nl = nullptr;                // nonlinear PDA adjoint scratch
  // host copies
  std::string err;
};

namespace mcrt {
int launch_trace(mcrt_ctx* ctx, const TraceArgs& a, hipStream_t s);
int launch_locate(mcrt_ctx* ctx, const double* xyz, int64_t n, int32_t* cell, hipStream_t s);
int launch_update_T(mcrt_ctx* ctx, hipStream_t s);
int launch_zero(void* p, size_t bytes, hipStream_t s);
int launch_hydrostatic(mcrt_ctx* ctx, double A, double T_floor, hipStream_t s);
double hydro_A(double M_star, double mu_mol);  // mu_mol m_p G M_star / k
int pda_solve(mcrt_ctx* ctx, const uint8_t* mask, mcrt_pda_stats* st, hipStream_t s);
void set_error(mcrt_ctx* ctx, const std::string& msg);
int pda_linear(mcrt_ctx* ctx, const uint8_t* mask, const double* rho, const double* kscale,
               const double* T_D, const double* T_bc, double* T_out, mcrt_pda_stats* st,
               hipStream_t s);
int pda_adjoint(mcrt_ctx* ctx, const double* dJdT, double* g_logrho, double* g_kscale,
                mcrt_pda_stats* st, hipStream_t s);
int pda_nonlinear(mcrt_ctx* ctx, const uint8_t* mask, const double* rho, const double* kscale,
                  const double* T_bc, double* T_out, mcrt_pda_stats* st, hipStream_t s);
int pda_nl_adjoint(mcrt_ctx* ctx, const double* dJdT, double* g_logrho, double* g_kscale,
                   mcrt_pda_stats* st, hipStream_t s);
// batches
size_t pda_wg_args_size();
int pda_batch_fill(mcrt_ctx** ctxs, int n, void* host);
int pda_batch_launch(const void* d_args, int n, hipStream_t s);
mcrt_pda_stats* pda_stats_slot(mcrt_ctx* ctx);
int launch_copy(double* dst, const double* src, size_t n, hipStream_t s);
// convergence statistic of the context's tallies against its stored pass;
// the result (R, rms change, rms noise, cells) lands in conv_result(ctx)
int launch_convergence(mcrt_ctx* ctx, int n_min, int first, hipStream_t s);
const double* conv_result(const mcrt_ctx* ctx);
// the PDA region rule with the given parameters, into a mask
int launch_region_mask(mcrt_ctx* ctx, int visits_min, double sigma, uint8_t* out, hipStream_t s);
// observables: J from the path tallies; the SED by ray tracing
int launch_mean_intensity(mcrt_ctx* ctx, const double* T, double* J, hipStream_t s);
int launch_raytrace(mcrt_ctx* ctx, const double* T, const double* J, int n_inc,
                    const double* cos_i_host, int n_sub, int n_phi, double* L, hipStream_t s);
size_t trace_fp32_lds(const DevModel& M, bool with_cdf);
size_t trace_fp32_lds_cap();
int trace_fp32_blocks_per_cu(size_t lds, bool cdf_lds);
int prepare_trace_fp32_batch(size_t lds, bool cdf_lds);
int launch_trace_fp32_batch(const TraceArgs* d_args, const int* d_block_disk, int n_disks,
                            int n_blocks, size_t lds, bool cdf_lds, hipStream_t s);
TraceArgs make_trace_args(mcrt_ctx* ctx, uint64_t n_packets, uint64_t n_total, uint64_t seed,
                          uint64_t offset, const double* frozen_T, mcrt_packet_rec* recs,
                          int64_t n_recs);
}  // namespace mcrt
