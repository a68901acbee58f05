"""Absorbed energy of the HIP path against the oracle, cell by cell, where the
two sides follow the same packets.

* Frozen temperature, MRW on, on the grid and opacities of the 1e-2 Msun
  workload (100 x 60 cells, 100 bins, gamma = 3, 20 interactions first): every
  packet draws the same numbers on both sides, so the absorbed energy of each
  cell -- absorptions plus MRW deposits eps rho kappa-bar l (Sect. 2.2.2) --
  agrees to summation order, and the integer tallies exactly.
* Immediate reemission with the running temperature (Sect. 2.1), packets
  traced one per launch so the GPU takes the absorptions in the oracle's order:
  each reemission draws its bin from the difference of the emission spectra
  between the tally before and after it, and the MRW uses the running cell
  temperature; records, tallies and energies agree packet after packet.

Packets whose events differ (a face reached within rounding, which the two
sides' different arithmetic can decide either way) are rare; the comparison
runs on the maximal ranges of packets that agree, traced again by offset.
"""
import os
import sys

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

sys.path.insert(0, os.path.dirname(__file__))
from frozen_runs import agreeing_runs, same_records  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mcrt(torch_cuda):
    from paper_0902_3092_amd import mcrt as M
    M.lib()
    return M


def test_frozen_T_absorbed_energy_with_mrw_on_bench_grid(mcrt, oracle_mod, torch_cuda):
    torch = torch_cuda
    d, o = W.config("mrw_pda")
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    mc = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    Tf = np.ascontiguousarray((400.0 * rc[:, None] ** -0.5 * (1 + 0.5 * mc[None, :])).reshape(-1))
    n, seed = 30000, 71
    kw = dict(mrw=True, gamma=o.gamma, n_int_min=o.n_int_min)
    ora = oracle_mod.Oracle(d)
    ctx, st, agree = agreeing_runs(mcrt, lambda: mcrt.Context(d, **kw), ora, n, seed, Tf, torch,
                                   **kw)
    assert agree >= 0.999, agree
    assert st["counters"][6] > 10000                      # MRW steps taken
    E_g = ctx.get(mcrt.GET_E_ABS).cpu().numpy()
    assert np.allclose(E_g, st["E_abs"], rtol=1e-10, atol=0)
    for what, key in ((mcrt.GET_VISITS, "visits"), (mcrt.GET_N_ABS, "n_abs"),
                      (mcrt.GET_N_MRW, "n_mrw")):
        got = ctx.get(what).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, st[key]), key
    # the MRW cells carry most of the deposited energy in this frozen field
    mrw_cells = st["n_mrw"] > 0
    assert mrw_cells.sum() > 50
    assert np.allclose(ctx.sed().cpu().numpy(), st["sed"], rtol=1e-10, atol=0)
    assert float(ctx.get(mcrt.GET_E_STAR).cpu()[0]) == pytest.approx(st["E_star"][0], rel=1e-12)


@pytest.mark.parametrize("wave_events", [0, 1])
def test_running_T_packet_order_parity(mcrt, oracle_mod, torch_cuda, wave_events):
    """One packet per launch (wave_events = 1: each runs in the whole-wavefront
    launch after its first event), running temperature, MRW on a thick disk:
    the GPU follows the oracle's serial run packet by packet, up to the first
    packet whose events differ; the absorbed energy after that prefix agrees
    cell by cell."""
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)
    kw = dict(mrw=True, gamma=2.0, n_int_min=5)
    N, seed = 300, 19
    ctx = mcrt.Context(d, wave_events=wave_events, **kw)
    ctx.reset()
    recs, E_g = [], []
    for p in range(N):
        r = ctx.trace(1, seed, n_total=N, offset=p, n_recs=1)
        recs.append(mcrt.Context.records_numpy(r)[0])
        E_g.append(ctx.get(mcrt.GET_E_ABS).cpu().numpy())
    torch.cuda.synchronize()
    g = np.array(recs, dtype=recs[0].dtype)
    ora = oracle_mod.Oracle(d)
    st, o_recs, E_o = None, [], []
    for p in range(N):
        st = ora.run(1, seed, n_total=N, offset=p, n_recs=1, state=st, **kw)
        o_recs.append(st["recs"][0])
        E_o.append(st["E_abs"].copy())
    o = np.array(o_recs, dtype=o_recs[0].dtype)
    same = same_records(g, o)
    m = N if same.all() else int(np.argmin(same))
    print("packets agreeing before the first difference: %d of %d; absorptions %d, MRW steps %d"
          % (m, N, o["n_abs"][:m].sum(), o["n_mrw"][:m].sum()))
    assert m >= 0.97 * N, m
    assert (o["n_abs"][:m].sum() > 200) and (o["n_mrw"][:m].sum() > 20)
    last = m - 1
    Eg, Eo = E_g[last], E_o[last]
    assert np.allclose(Eg, Eo, rtol=1e-10, atol=0)
    # the temperature of every cell then agrees, through the same inversion
    T_g = ctx.update_T().cpu().numpy() if m == N else None
    if T_g is not None:
        assert np.allclose(T_g, ora.update_T(Eo), rtol=1e-12, atol=0)
