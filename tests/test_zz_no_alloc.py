"""mcrt_pda_solve_noalloc -- the PDA solve for callers that cannot allocate
device memory -- against mcrt_pda_solve with the same one-workgroup solver,
through the C-ABI: two calls in a row on the library's fixed scratch, the
second on a smaller grid, each on a fresh context and on the allocating path;
same region (exactly), temperatures to the CG tolerance, same statistics; a
grid beyond the fixed size is refused before anything runs."""
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


@pytest.fixture(scope="module")
def mcrt(torch_cuda):
    from paper_0902_3092_amd import mcrt as M
    M.lib()
    return M


def test_noalloc_pda_matches_allocating_solve(mcrt, torch_cuda):
    """Per case: one trace, then the allocating solve and the fixed-scratch
    solve from the same Monte Carlo temperature on the same context.  The
    fixed-scratch calls run back to back, the second on a smaller grid (the
    scratch keeps the first call's contents)."""
    torch = torch_cuda
    big, _ = W.config("mrw_pda")                                     # 100 x 60 cells
    small = W.make_disk("s", M_dust_msun=3e-3, n_r=30, n_mu=20, n_lambda=40)
    cases = [(big, 100000, 5, dict(pda_visits=100)),
             (small, 30000, 6, dict(pda_visits=100, pda_sigma=0.05))]
    for d, n, seed, kw in cases:
        ctx = mcrt.Context(d, precision="fp32", mrw=True, gamma=3.0, n_int_min=20, pda_solver=2,
                           **kw)
        ctx.reset()
        ctx.trace(n, seed)
        T_mc = ctx.update_T().clone()
        st1 = ctx.pda_solve()                                        # allocating
        T1, reg1 = ctx.get(mcrt.GET_T).cpu().numpy(), ctx.get(mcrt.GET_REGION).cpu().numpy()
        ctx.set_T(T_mc)
        st2 = ctx.pda_solve_noalloc()                                # fixed scratch
        torch.cuda.synchronize()
        T2, reg2 = ctx.get(mcrt.GET_T).cpu().numpy(), ctx.get(mcrt.GET_REGION).cpu().numpy()
        assert np.array_equal(reg1, reg2)
        assert st2["n_region"] == st1["n_region"] > 0
        assert st2["n_isolated"] == st1["n_isolated"]
        assert st2["sweeps"] == st1["sweeps"] and st2["rc"] == st1["rc"]
        assert abs(st2["cg_iters_total"] - st1["cg_iters_total"]) <= st1["sweeps"]
        assert np.allclose(T2, T1, rtol=1e-9, atol=0)


def test_noalloc_refuses_grids_beyond_its_scratch(mcrt, torch_cuda):
    torch = torch_cuda
    d = W.make_disk("x", M_dust_msun=1e-3, n_r=200, n_mu=200, n_lambda=8)  # 40000 cells
    ctx = mcrt.Context(d, precision="fp32")
    T = torch.full((ctx.n_cells,), 100.0, dtype=torch.float64, device="cuda")
    ctx.set_T(T)
    with pytest.raises(mcrt.McrtError) as e:
        ctx.pda_solve_noalloc(torch.ones(ctx.n_cells, dtype=torch.uint8, device="cuda"))
    assert e.value.code == mcrt.E_ARG
    assert torch.equal(ctx.get(mcrt.GET_T), T)                       # nothing ran
