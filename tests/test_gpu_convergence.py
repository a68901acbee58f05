"""The convergence decision of the vertical-structure loop on the device
(Sect. 2.5: the change of the temperature between consecutive passes against
its Monte Carlo error, converged below 3 sigma).

* The odd-numbered packets' tally (conv_split) and the statistic
  (mcrt_convergence) against the oracle, on two frozen-temperature passes of
  the 1e-2 Msun workload that both sides trace packet for packet.
* mcrt_batch_converge: the loop stops at the first pass whose statistic is
  below the threshold (a huge threshold: pass 1; an unreachable one: every
  pass runs and MCRT_E_NOT_CONVERGED comes back), and on the workload with
  the hydrostatic step it records the statistic of every pass.
"""
import os
import sys

import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

sys.path.insert(0, os.path.dirname(__file__))
from frozen_runs import agreeing_runs  # noqa: E402

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


def test_split_tally_and_statistic_match_oracle(mcrt, oracle_mod, torch_cuda):
    """FP64 tracking deposits what the oracle does up to summation order (FP32
    tracking follows the oracle in distribution only; its split tally is
    checked against its own odd-numbered packets in test_gpu_raytrace.py)."""
    torch = torch_cuda
    precision, rtol = "fp64", 1e-10
    d, o = W.config("mrw_pda")
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    mc = 0.5 * (d.mu_edges[:-1] + d.mu_edges[1:])
    Tf = np.ascontiguousarray((400.0 * rc[:, None] ** -0.5 * (1 + 0.5 * mc[None, :])).reshape(-1))
    kw = dict(mrw=True, gamma=o.gamma, n_int_min=o.n_int_min)
    make = lambda: mcrt.Context(d, precision=precision, conv_split=1, **kw)
    ora = oracle_mod.Oracle(d)
    T_prev, s2_prev = np.zeros(ora.n_cells), -np.ones(ora.n_cells)
    ctx = None
    n_min = 30
    for p, seed in enumerate((71, 72)):
        ctx, st, agree = agreeing_runs(mcrt, make, ora, 20000, seed, Tf, torch, ctx=ctx, **kw)
        assert agree >= 0.999
        E_half = ctx.get(mcrt.GET_E_HALF).cpu().numpy()
        assert np.allclose(E_half, st["E_half"], rtol=rtol, atol=0)
        assert 0.05 < E_half.sum() / st["E_abs"].sum() < 0.95   # a few walks carry much
        g = ctx.convergence(n_min=n_min, first=(p == 0))
        want = ora.conv_stat(st, T_prev, s2_prev, n_min=n_min)
        print(precision, "pass", p, "GPU", g, "oracle", want)
        assert g[3] == want[3]
        assert np.allclose(g[:3], want[:3], rtol=10 * rtol, atol=0)
    assert want[3] > 500 and want[0] > 0


def _ctx(mcrt, **kw):
    d, o = W.config("mrw_pda")
    return mcrt.Context(d, precision="fp32", mrw=True, gamma=o.gamma, n_int_min=o.n_int_min,
                        pda_visits=o.pda_visits, n_T=o.n_T, **kw)


def test_loop_stops_at_the_threshold(mcrt, torch_cuda):
    ctx = _ctx(mcrt)
    _, rec, rc = mcrt.batch_converge([ctx], [200000], [5], max_iter=4, threshold=1e9)
    assert rc == mcrt.OK and rec[0]["passes"] == 2 and rec[0]["converged_pass"] == 1
    assert rec[0]["R"][0] == 0.0 and rec[0]["R"][1] > 0.0 and rec[0]["cells"] > 100
    ctx2 = _ctx(mcrt)
    _, rec, rc = mcrt.batch_converge([ctx2], [200000], [5], max_iter=3, threshold=1e-9,
                                     use_graph=False)
    assert rc == mcrt.E_NOT_CONVERGED
    assert rec[0]["passes"] == 3 and rec[0]["converged_pass"] == -1 and len(rec[0]["R"]) == 3


def test_vertical_structure_loop_converges(mcrt, torch_cuda):
    """The 1e-2 Msun workload with the hydrostatic step (M_star 2.5 Msun, mu
    2.3) at 1e6 packets per pass, beside the same disk without the step (an
    unchanged structure, the same seeds): without the step consecutive passes
    differ by their noise alone (R ~ 1); the step's change of the structure
    adds to that; both loops end below 3.  (At 1e6 packets a cell's T carries
    ~10 % noise, so the 3-sigma test of the mean over the structure passes
    while the structure still moves by up to ~2.8 times that.)"""
    torch = torch_cuda
    hyd = _ctx(mcrt, hydro_M_star=2.5 * W.M_SUN, hydro_mu=2.3)
    flat = _ctx(mcrt)
    _, rec, rc = mcrt.batch_converge([hyd, flat], [1000000, 1000000], [9, 9], max_iter=10)
    torch.cuda.synchronize()
    print("with the hydrostatic step:", rec[0])
    print("unchanged structure:", rec[1])
    assert rc == mcrt.OK
    h, f = rec
    assert f["converged_pass"] == 1 and 0.7 < f["R"][1] < 1.5
    assert h["converged_pass"] >= 1 and h["R_last"] < 3.0 and h["cells"] > 1000
    # the step moves the structure beyond the noise of an unchanged one
    assert h["R"][1] > f["R"][1]
    assert h["dT_rms"] ** 2 - h["noise_rms"] ** 2 > 2 * max(f["dT_rms"] ** 2 - f["noise_rms"] ** 2,
                                                             0.0)
