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
    assert e["options"]["wave_events"] in (512, 2048)
    assert e["options"]["pda_solver"] in (1, 2)
    assert A.options_for(d, 20000, path=p, **phys) == e["options"]
    ctx = mcrt.Context(d, **phys, **e["options"])
    ctx.reset()
    ctx.trace(20000, 9)
    ctx.update_T()
    ctx.pda_solve()
    torch.cuda.synchronize()
    c = ctx.counters()
    assert c["launch"] == 20000 and c["escaped"] + c["star"] == 20000
