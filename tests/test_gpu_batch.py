"""Batched passes (mcrt_batch_run): several disks of different grids in one
persistent trace launch and one workgroup-per-disk PDA launch, with and without
graph capture, against the same disks run one at a time.

In optically thick cells a few long random walks carry most of the absorbed
energy, so single runs scatter widely: the comparison uses seed ensembles and
their empirical standard errors on both sides."""
import numpy as np
import pytest

from paper_0902_3092_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _disks():
    return [W.make_disk("b0", M_dust_msun=1e-4, n_r=20, n_mu=16, n_lambda=30),
            W.make_disk("b1", M_dust_msun=3e-3, n_r=34, n_mu=22, n_lambda=30, hr0=0.04),
            W.make_disk("b2", M_dust_msun=1e-5, n_r=12, n_mu=10, n_lambda=30, hr0=0.02)]


def _ctx(mcrt, d):
    return mcrt.Context(d, precision="fp32", mrw=True, gamma=3.0, n_int_min=20, pda_visits=30)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_matches_single_disk_runs(torch_cuda, use_graph):
    torch = torch_cuda
    from paper_0902_3092_amd import mcrt
    disks = _disks()
    npk = [200000, 100000, 60000]
    K = 6
    ctxs = [_ctx(mcrt, d) for d in disks]
    singles = [_ctx(mcrt, d) for d in disks]
    TB = [[] for _ in disks]
    TS = [[] for _ in disks]
    NB = [[] for _ in disks]
    for k in range(K):
        seeds = [100 * k + 11 + d for d in range(len(disks))]
        stats = mcrt.batch_run(ctxs, npk, seeds, n_iter=2, use_graph=use_graph)
        torch.cuda.synchronize()
        for d, (ctx, one, n, sd, st) in enumerate(zip(ctxs, singles, npk, seeds, stats)):
            L = ctx.tables()["L_star"]
            c = ctx.counters()
            assert c["launch"] == n and c["capped"] == 0
            sed = ctx.sed().cpu().numpy()
            E_star = ctx.get(mcrt.GET_E_STAR).cpu().numpy()[0]
            assert (sed.sum() + E_star) / L == pytest.approx(1.0, abs=1e-6)
            reg = ctx.get(mcrt.GET_REGION).cpu().numpy()
            assert st["n_region"] == int((reg == 1).sum())
            assert st["converged"] == 1
            TB[d].append(ctx.get(mcrt.GET_T).cpu().numpy())
            NB[d].append(ctx.get(mcrt.GET_N_ABS).cpu().numpy())
            # the same disk on its own: trace + T + PDA with the last pass's seed
            one.reset()
            one.trace(n, sd + (1 << 32))
            one.update_T()
            one.pda_solve()
            torch.cuda.synchronize()
            TS[d].append(one.get(mcrt.GET_T).cpu().numpy())
    for d in range(len(disks)):
        tb, ts = np.array(TB[d]), np.array(TS[d])
        ok = (np.array(NB[d]).min(0) > 200) & (tb.min(0) > 0) & (ts.min(0) > 0)
        assert ok.sum() >= 3
        se = np.sqrt(tb.var(0, ddof=1) / K + ts.var(0, ddof=1) / K)[ok]
        diff = (tb.mean(0) - ts.mean(0))[ok]
        rel = np.abs(diff) / ts.mean(0)[ok]
        good = (np.abs(diff) < 4 * se) | (rel < 0.01)
        assert good.mean() >= 0.9, (d, np.sort(rel)[-5:])


def test_batch_rejects_fp64_contexts(torch_cuda):
    from paper_0902_3092_amd import mcrt
    d = _disks()[0]
    ctx = mcrt.Context(d, precision="fp64")
    with pytest.raises(mcrt.McrtError):
        mcrt.batch_run([ctx], [1000], [1], n_iter=1)

