"""The autotuner on the GPU: it times its candidates on a small disk and the
options it returns run an ordinary pass."""
import pytest

from paper_0902_3092_amd import workloads as W

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


def test_autotune_small_disk(mcrt, torch_cuda, tmp_path):
    """Candidates timed, the choice cached, and a context built from it
    traces every packet."""
    from paper_0902_3092_amd import autotune as A
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=3e-3, n_r=20, n_mu=14, n_lambda=24)
    phys = dict(precision="fp32", mrw=True, gamma=3.0, n_int_min=20, pda_visits=100)
    p = str(tmp_path / "tune.json")
    e = A.tune(d, n_packets=20000, seeds=(3,), wave_events=(512, 2048), pda_repeats=1,
               path=p, **phys)
    assert set(e["trace_s"]) == {"512", "2048"}
    assert set(e["shape_s"]) == {"512/0", "768/0", "256/0", "256/1"}
    assert set(e["calls_s"]) == {"1", "2", "4"}
    o = e["options"]
    assert o["wave_events"] in (512, 2048) and o["block_size"] in (256, 512, 768)
    assert o["calls_per_pass"] in (1, 2, 4) and o["pda_solver"] in (1, 2)
    opts = A.options_for(d, 20000, path=p, **phys)
    assert "calls_per_pass" not in opts and opts["block_size"] == o["block_size"]
    ctx = mcrt.Context(d, **phys, **opts)
    ctx.reset()
    A.trace_pass(ctx, 20000, 9, A.calls_per_pass(d, 20000, path=p, **phys))
    ctx.update_T()
    ctx.pda_solve()
    torch.cuda.synchronize()
    c = ctx.counters()
    assert c["launch"] == 20000 and c["escaped"] + c["star"] == 20000


@pytest.mark.parametrize("shape", [(256, 0), (256, 1), (512, 2), (768, 0)])
def test_launch_shapes_trace_the_same_packets(mcrt, torch_cuda, shape):
    """Frozen temperature: every launch shape traces each packet to the same
    events, so the integer tallies agree exactly with the default shape's and
    the absorbed energy to summation order."""
    import numpy as np
    torch = torch_cuda
    d = W.small_disk(M_dust_msun=1e-2, n_r=20, n_mu=14, n_lambda=24)
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    Tf = torch.from_numpy(np.ascontiguousarray(np.repeat(300.0 * rc ** -0.5, d.n_mu))).cuda()
    out = []
    for bs, cu in ((512, 0), shape):
        ctx = mcrt.Context(d, precision="fp32", mrw=True, block_size=bs, blocks_per_cu=cu)
        ctx.reset()
        ctx.trace(50000, 4, frozen_T=Tf)
        torch.cuda.synchronize()
        out.append([ctx.get(w).cpu().numpy() for w in (mcrt.GET_VISITS, mcrt.GET_N_ABS,
                                                       mcrt.GET_N_MRW, mcrt.GET_E_ABS)])
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)
    assert np.allclose(out[0][3], out[1][3], rtol=1e-12, atol=0)


def test_fp64_rejects_the_small_workgroup(mcrt, torch_cuda):
    d = W.small_disk()
    with pytest.raises(mcrt.McrtError):
        mcrt.Context(d, precision="fp64", block_size=256)
