// Many disks, several passes: {trace -> temperature -> PDA} x n_iter over a
// batch of contexts, each pass one persistent trace launch for all disks and
// one workgroup-per-disk PDA launch, optionally captured in a HIP graph and
// replayed as one submission.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mcrt_internal.h"

namespace {
size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int fail_batch(int code, const std::string& msg) {
  mcrt::set_error(nullptr, msg);
  return code;
}

// After a pass's trace: add its capped packets to the context's running sum
// (the pass's counters are cleared when the next pass starts).
__global__ void add_capped_kernel(const unsigned long long* counters, mcrt::DevHealth* h) {
  if (threadIdx.x == 0 && blockIdx.x == 0) h->capped += counters[mcrt::C_CAPPED];
}

int check_batch(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets, const uint64_t* seeds,
                int n_iter) {
  if (!ctxs || n_disks < 1 || !n_packets || !seeds || n_iter < 1)
    return fail_batch(MCRT_E_ARG, "bad batch arguments");
  for (int d = 0; d < n_disks; ++d) {
    if (!ctxs[d] || n_packets[d] == 0) return fail_batch(MCRT_E_ARG, "bad context or packet count");
    if (ctxs[d]->opt.precision != MCRT_FP32)
      return fail_batch(MCRT_E_ARG, "batched runs use FP32 tracking (precision = MCRT_FP32)");
    if (ctxs[d]->opt.g_asym != 0.0)
      return fail_batch(MCRT_E_ARG, "batched runs scatter isotropically (g_asym = 0)");
    if (ctxs[d]->device != ctxs[0]->device) return fail_batch(MCRT_E_ARG, "contexts on one device");
  }
  return MCRT_OK;
}

// Clear the outcome counters of a batch; the batch overwrites the PDA
// scratch (and, with the hydrostatic step, the density) that a linear PDA
// solve left for its adjoint.
int begin_batch(mcrt_ctx** ctxs, int n_disks, hipStream_t s) {
  for (int d = 0; d < n_disks; ++d) {
    ctxs[d]->lin_ready = false;
    if (mcrt::launch_zero(ctxs[d]->d_health, sizeof(mcrt::DevHealth), s) != MCRT_OK)
      return fail_batch(MCRT_E_HIP, "clearing the batch counters failed");
  }
  return MCRT_OK;
}

// Passes it0 .. it0 + n_iter - 1 of a batch (pass k traces with seed
// seeds[d] + (k << 32)), queued on s -- captured in one HIP graph when
// use_graph -- and waited for.  conv_n_min > 0: each pass also keeps the
// split tally and ends its Monte Carlo part with the convergence statistic
// (the first pass of the batch, k = 0, only stores its values).
int run_passes(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets, const uint64_t* seeds,
               int it0, int n_iter, bool use_graph, int conv_n_min, hipStream_t s) {
  mcrt_ctx* c0 = ctxs[0];
  // launch shape: LDS for the largest disk, workgroups shared by packets
  size_t lds = 0;
  for (int d = 0; d < n_disks; ++d) lds = std::max(lds, mcrt::trace_fp32_lds(ctxs[d]->m, true));
  const bool cdf_lds = lds <= mcrt::trace_fp32_lds_cap();
  if (!cdf_lds) {  // every disk reads its emission CDF from L2 instead
    lds = 0;
    for (int d = 0; d < n_disks; ++d) lds = std::max(lds, mcrt::trace_fp32_lds(ctxs[d]->m, false));
  }
  // room for the visit histograms of the disks whose tables and histogram fit
  for (int d = 0; d < n_disks; ++d) {
    size_t want = mcrt::trace_fp32_lds(ctxs[d]->m, cdf_lds) + (size_t)4 * ctxs[d]->n_cells;
    if (want <= mcrt::trace_fp32_lds_cap()) lds = std::max(lds, want);
  }
  const int per_cu = mcrt::trace_fp32_blocks_per_cu(lds, cdf_lds);
  const long long total_blocks = std::max<long long>((long long)c0->n_cu * per_cu, n_disks);
  double sumN = 0.0;
  for (int d = 0; d < n_disks; ++d) sumN += (double)n_packets[d];
  std::vector<int> nb(n_disks);
  long long used = 0;
  for (int d = 0; d < n_disks; ++d) {
    long long want = (long long)std::floor((double)total_blocks * (double)n_packets[d] / sumN);
    long long need = ((long long)n_packets[d] + 511) / 512;
    nb[d] = (int)std::max<long long>(1, std::min(want, need));
    used += nb[d];
  }
  std::vector<int> block_disk;
  block_disk.reserve(used);
  for (int d = 0; d < n_disks; ++d)
    for (int b = 0; b < nb[d]; ++b) block_disk.push_back(d);
  // arguments for every pass, uploaded before any work is queued
  const size_t targs = sizeof(mcrt::TraceArgs);
  std::vector<mcrt::TraceArgs> ta((size_t)n_iter * n_disks);
  for (int q = 0; q < n_iter; ++q)
    for (int d = 0; d < n_disks; ++d) {
      const int it = it0 + q;
      mcrt_ctx* c = ctxs[d];
      mcrt::TraceArgs a = mcrt::make_trace_args(c, n_packets[d], n_packets[d],
                                                seeds[d] + ((uint64_t)it << 32), 0, nullptr,
                                                nullptr, 0);
      if (conv_n_min > 0) a.t.E_half = c->d_E_half;
      // passes after the first may take the MRW coefficients from the
      // previous pass's (PDA-corrected) temperature
      a.T_coef = (c->opt.mrw_coef_T == 1 && (it > 0 || c->have_T_prev)) ? c->d_T_prev : nullptr;
      a.vis_lds = mcrt::trace_fp32_lds(c->m, cdf_lds) + (size_t)4 * c->n_cells <= lds;
      ta[(size_t)q * n_disks + d] = a;
    }
  const size_t pda_bytes = mcrt::pda_wg_args_size() * n_disks;
  std::vector<char> pda_host(pda_bytes);
  int rc = mcrt::pda_batch_fill(ctxs, n_disks, pda_host.data());
  if (rc) return rc;
  size_t bytes = al(ta.size() * targs) + al(block_disk.size() * sizeof(int)) + al(pda_bytes) +
                 al(16);
  void* blob = nullptr;
  if (hipMalloc(&blob, bytes) != hipSuccess) return fail_batch(MCRT_E_OOM, "batch arguments");
  char* q = (char*)blob;
  mcrt::TraceArgs* d_ta = (mcrt::TraceArgs*)q;
  q += al(ta.size() * targs);
  int* d_bd = (int*)q;
  q += al(block_disk.size() * sizeof(int));
  void* d_pda = q;
  q += al(pda_bytes);
  // one live count for the whole batch: hand-offs wait until all disks'
  // packets are out and no more are live than the hand-off launch has
  // wavefronts
  long long* d_live = (long long*)q;
  unsigned int* d_waves_in = (unsigned int*)(d_live + 1);
  const unsigned waves = (unsigned)block_disk.size() * 8u;  // 512-thread workgroups
  for (auto& a : ta) {
    a.live = d_live;
    a.waves_in = d_waves_in;
    a.n_waves = sumN <= (double)waves ? 0u : waves;  // a small batch needs no count
    a.live_handoff = waves;
  }
  hipError_t e = hipMemcpy(d_ta, ta.data(), ta.size() * targs, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d_bd, block_disk.data(), block_disk.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_pda, pda_host.data(), pda_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipFree(blob);
    return fail_batch(MCRT_E_HIP, "batch argument upload");
  }
  mcrt::prepare_trace_fp32_batch(lds, cdf_lds);
  // the passes
  auto enqueue = [&](hipStream_t s) -> int {
    for (int qi = 0; qi < n_iter; ++qi) {
      const int it = it0 + qi;
      for (int d = 0; d < n_disks; ++d) {
        mcrt_ctx* c = ctxs[d];
        // tallies, split tally and work counter
        size_t tally = (size_t)((char*)c->d_next - (char*)c->t.E_abs) + 8;
        int r = mcrt::launch_zero(c->t.E_abs, tally, s);
        if (r) return r;
        if (c->t.path) {
          r = mcrt::launch_zero(c->d_paths, (size_t)((char*)(c->t.mrw_path + c->n_cells) -
                                                     (char*)c->d_paths), s);
          if (r) return r;
        }
        const mcrt::TraceArgs& a = ta[(size_t)qi * n_disks + d];
        if (a.tail_count) {
          r = mcrt::launch_zero(a.tail_count, 8, s);  // and tail_next
          if (r) return r;
        }
        if (a.T_coef) {
          r = mcrt::launch_copy(c->d_T_prev, c->d_T, (size_t)c->n_cells, s);
          if (r) return r;
        }
      }
      int r = mcrt::launch_zero(d_live, 16, s);  // the live count and its wavefronts
      if (r) return r;
      r = mcrt::launch_trace_fp32_batch(d_ta + (size_t)qi * n_disks, d_bd, n_disks,
                                        (int)block_disk.size(), lds, cdf_lds, s);
      if (r) return r;
      for (int d = 0; d < n_disks; ++d) {
        hipLaunchKernelGGL(add_capped_kernel, dim3(1), dim3(64), 0, s, ctxs[d]->t.counters,
                           ctxs[d]->d_health);
        if (hipGetLastError() != hipSuccess) return MCRT_E_HIP;
      }
      for (int d = 0; d < n_disks; ++d) {
        r = mcrt::launch_update_T(ctxs[d], s);
        if (r) return r;
        if (conv_n_min > 0) {
          r = mcrt::launch_convergence(ctxs[d], conv_n_min, it == 0 ? 1 : 0, s);
          if (r) return r;
        }
      }
      r = mcrt::pda_batch_launch(d_pda, n_disks, s);
      if (r) return r;
      for (int d = 0; d < n_disks; ++d) {
        mcrt_ctx* c = ctxs[d];
        if (c->opt.hydro_M_star > 0.0) {
          r = mcrt::launch_hydrostatic(
              c, mcrt::hydro_A(c->opt.hydro_M_star, c->opt.hydro_mu), c->opt.T_lo, s);
          if (r) return r;
        }
      }
    }
    return MCRT_OK;
  };
  int status = MCRT_OK;
  if (use_graph) {
    // capture on a stream of our own (the caller's may be the null stream,
    // which cannot be captured), then submit the graph on the caller's stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      status = enqueue(cs);
      hipError_t e2 = hipStreamEndCapture(cs, &graph);
      if (status == MCRT_OK && e2 == hipSuccess)
        e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (status == MCRT_OK && e2 == hipSuccess) e2 = hipGraphLaunch(exec, s);
      if (status == MCRT_OK && e2 != hipSuccess) {
        mcrt::set_error(nullptr, std::string("graph: ") + hipGetErrorString(e2));
        status = MCRT_E_HIP;
      }
    } else {
      mcrt::set_error(nullptr, std::string("stream capture: ") + hipGetErrorString(e));
      status = MCRT_E_HIP;
    }
    if (hipStreamSynchronize(s) != hipSuccess && status == MCRT_OK) status = MCRT_E_HIP;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
  } else {
    status = enqueue(s);
    if (hipStreamSynchronize(s) != hipSuccess && status == MCRT_OK) status = MCRT_E_HIP;
  }
  if (status == MCRT_OK)
    for (int d = 0; d < n_disks; ++d)
      if (ctxs[d]->opt.mrw_coef_T == 1) ctxs[d]->have_T_prev = true;
  (void)hipFree(blob);
  return status;
}

// The PDA statistics of the last pass, then the outcome of every pass: a PDA
// solve that hit its iteration cap, or packets that hit the event cap, in
// any pass of any disk.
int end_batch(mcrt_ctx** ctxs, int n_disks, mcrt_pda_stats* stats) {
  if (stats) {
    for (int d = 0; d < n_disks; ++d)
      if (hipMemcpy(&stats[d], mcrt::pda_stats_slot(ctxs[d]), sizeof(mcrt_pda_stats),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return fail_batch(MCRT_E_HIP, "reading the PDA statistics failed");
  }
  unsigned long long fails = 0, capped = 0;
  int first_fail = -1, first_capped = -1;
  for (int d = 0; d < n_disks; ++d) {
    mcrt::DevHealth h{};
    if (hipMemcpy(&h, ctxs[d]->d_health, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess)
      return fail_batch(MCRT_E_HIP, "reading the batch counters failed");
    if (h.pda_fails && first_fail < 0) first_fail = d;
    if (h.capped && first_capped < 0) first_capped = d;
    fails += h.pda_fails;
    capped += h.capped;
  }
  if (fails)
    return fail_batch(MCRT_E_NOT_CONVERGED,
                      std::to_string(fails) + " PDA solve(s) hit an iteration cap (first: disk " +
                          std::to_string(first_fail) + ")");
  if (capped)
    return fail_batch(MCRT_E_STUCK, std::to_string(capped) +
                                        " packet(s) hit the event cap (first: disk " +
                                        std::to_string(first_capped) + ")");
  return MCRT_OK;
}
}  // namespace

extern "C" int mcrt_batch_run(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets,
                              const uint64_t* seeds, int n_iter, int use_graph,
                              mcrt_pda_stats* stats, hipStream_t s) {
  int rc = check_batch(ctxs, n_disks, n_packets, seeds, n_iter);
  if (rc) return rc;
  rc = begin_batch(ctxs, n_disks, s);
  if (rc) return rc;
  rc = run_passes(ctxs, n_disks, n_packets, seeds, 0, n_iter, use_graph != 0, 0, s);
  if (rc) return rc;
  return end_batch(ctxs, n_disks, stats);
}

extern "C" int mcrt_batch_converge(mcrt_ctx** ctxs, int n_disks, const uint64_t* n_packets,
                                   const uint64_t* seeds, int max_iter, int32_t n_min,
                                   double threshold, int use_graph, mcrt_pda_stats* stats,
                                   mcrt_conv_stats* conv, double* R_hist, hipStream_t s) {
  int rc = check_batch(ctxs, n_disks, n_packets, seeds, max_iter);
  if (rc) return rc;
  if (max_iter < 2 || n_min < 1 || !(threshold > 0.0))
    return fail_batch(MCRT_E_ARG, "max_iter >= 2, n_min >= 1 and threshold > 0 needed");
  rc = begin_batch(ctxs, n_disks, s);
  if (rc) return rc;
  std::vector<mcrt_conv_stats> cs(n_disks);
  for (auto& c : cs) c = mcrt_conv_stats{0, -1, 0.0, 0.0, 0.0, 0};
  if (R_hist)
    for (size_t k = 0; k < (size_t)n_disks * max_iter; ++k) R_hist[k] = -1.0;
  std::vector<double> res(4);
  int it = 0;
  for (; it < max_iter; ++it) {
    rc = run_passes(ctxs, n_disks, n_packets, seeds, it, 1, use_graph != 0, n_min, s);
    if (rc) return rc;
    bool all = true;
    for (int d = 0; d < n_disks; ++d) {
      if (hipMemcpy(res.data(), mcrt::conv_result(ctxs[d]), 4 * sizeof(double),
                    hipMemcpyDeviceToHost) != hipSuccess)
        return fail_batch(MCRT_E_HIP, "reading the convergence statistic failed");
      mcrt_conv_stats& c = cs[d];
      c.passes = it + 1;
      c.R_last = res[0];
      c.dT_rms = res[1];
      c.noise_rms = res[2];
      c.cells = (int32_t)res[3];
      if (R_hist) R_hist[(size_t)d * max_iter + it] = res[0];
      if (it > 0 && c.converged_pass < 0 && c.cells > 0 && res[0] < threshold)
        c.converged_pass = it;
      all = all && c.converged_pass >= 0;
    }
    if (all) break;
  }
  if (conv)
    for (int d = 0; d < n_disks; ++d) conv[d] = cs[d];
  rc = end_batch(ctxs, n_disks, stats);
  if (rc) return rc;
  for (int d = 0; d < n_disks; ++d)
    if (cs[d].converged_pass < 0)
      return fail_batch(MCRT_E_NOT_CONVERGED,
                        "disk " + std::to_string(d) + " did not converge in " +
                            std::to_string(max_iter) + " passes");
  return MCRT_OK;
}

// The PDA step of a batched pass alone: every context's region (its rule on
// its current tallies) solved from its current temperature, one workgroup per
// disk, all disks in one launch.
extern "C" int mcrt_batch_pda(mcrt_ctx** ctxs, int n_disks, mcrt_pda_stats* stats,
                              hipStream_t s) {
  if (!ctxs || n_disks < 1) return fail_batch(MCRT_E_ARG, "bad batch arguments");
  for (int d = 0; d < n_disks; ++d) {
    if (!ctxs[d]) return fail_batch(MCRT_E_ARG, "null context");
    if (ctxs[d]->device != ctxs[0]->device) return fail_batch(MCRT_E_ARG, "contexts on one device");
    if (ctxs[d]->opt.pda_visits <= 0 && !(ctxs[d]->opt.pda_sigma > 0.0))
      return fail_batch(MCRT_E_ARG, "a context has no PDA region rule (pda_visits, pda_sigma)");
  }
  const size_t pda_bytes = mcrt::pda_wg_args_size() * n_disks;
  std::vector<char> host(pda_bytes);
  int rc = mcrt::pda_batch_fill(ctxs, n_disks, host.data());
  if (rc) return rc;
  void* blob = nullptr;
  if (hipMalloc(&blob, pda_bytes) != hipSuccess) return fail_batch(MCRT_E_OOM, "batch arguments");
  int status = MCRT_OK;
  if (hipMemcpy(blob, host.data(), pda_bytes, hipMemcpyHostToDevice) != hipSuccess)
    status = fail_batch(MCRT_E_HIP, "batch argument upload");
  for (int d = 0; d < n_disks && status == MCRT_OK; ++d) {
    ctxs[d]->lin_ready = false;
    if (mcrt::launch_zero(ctxs[d]->d_health, sizeof(mcrt::DevHealth), s) != MCRT_OK)
      status = fail_batch(MCRT_E_HIP, "clearing the batch counters failed");
  }
  if (status == MCRT_OK && mcrt::pda_batch_launch(blob, n_disks, s) != MCRT_OK)
    status = fail_batch(MCRT_E_HIP, "batched PDA launch failed");
  if (hipStreamSynchronize(s) != hipSuccess && status == MCRT_OK)
    status = fail_batch(MCRT_E_HIP, "batched PDA failed");
  bool isolated = false;
  unsigned fails = 0;
  for (int d = 0; d < n_disks && status == MCRT_OK; ++d) {
    mcrt_pda_stats st{};
    mcrt::DevHealth h{};
    if (hipMemcpy(&st, mcrt::pda_stats_slot(ctxs[d]), sizeof(st), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        hipMemcpy(&h, ctxs[d]->d_health, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
      status = fail_batch(MCRT_E_HIP, "reading the batched PDA statistics failed");
      break;
    }
    if (stats) stats[d] = st;
    isolated |= st.n_isolated > 0;
    fails += h.pda_fails;
  }
  (void)hipFree(blob);
  if (status == MCRT_OK && fails)
    status = fail_batch(MCRT_E_NOT_CONVERGED,
                        std::to_string(fails) + " PDA solve(s) hit an iteration cap");
  if (status == MCRT_OK && isolated) status = MCRT_E_SINGULAR_REGION;
  return status;
}
