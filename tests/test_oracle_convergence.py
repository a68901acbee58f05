"""Pins of the oracle's convergence statistic for the vertical-structure loop
(Sect. 2.5: the change of the temperature between consecutive passes against
its Monte Carlo error, converged below 3 sigma) and of the split tally it
rests on.

* The odd-numbered packets' tally equals, bit for bit, a run of those packets
  alone (frozen temperature, so the packets do not interact).
* Special cases of the noise estimate: halves that agree give no noise; all
  the energy in one half gives a relative spread of E of 1, carried to T by
  the slope of the inversion.
* The estimate against brute force: over independent runs of the 1e-2 Msun
  workload, the spread of each cell's temperature matches the mean of the
  split estimates; in the cells where MRW deposits carry the energy the
  split estimate is low (the halves share the running temperature), and
  1 / (16 N_abs) -- which counts absorptions as if independent -- misses the
  spread there by orders of magnitude.
* Consecutive independent passes of an unchanged structure give R ~ 1; a
  change of T well beyond the noise gives R above 3.
"""
import numpy as np
import pytest
from multiprocessing import get_context

from paper_0902_3092_amd import workloads as W


def test_odd_tally_is_the_odd_packets_alone(oracle_mod):
    d = W.small_disk(M_dust_msun=1e-1, n_r=14, n_mu=10, n_lambda=24)
    ora = oracle_mod.Oracle(d)
    rc = 0.5 * (d.r_edges[:-1] + d.r_edges[1:]) / W.AU
    Tf = np.ascontiguousarray(np.repeat(300.0 * rc ** -0.5, d.n_mu))
    kw = dict(mrw=True, gamma=2.0, n_int_min=5, frozen_T=Tf)
    n = 400
    full = ora.run(n, 7, **kw)
    odd, even = None, None
    for p in range(n):
        if p & 1:
            odd = ora.run(1, 7, n_total=n, offset=p, state=odd, **kw)
        else:
            even = ora.run(1, 7, n_total=n, offset=p, state=even, **kw)
    assert full["n_mrw"].sum() > 100
    assert np.array_equal(full["E_half"], odd["E_abs"])
    assert np.allclose(full["E_abs"] - full["E_half"], even["E_abs"], rtol=1e-12, atol=0)
    assert np.all(odd["E_half"] == odd["E_abs"]) and np.all(even["E_half"] == 0)


def test_noise_special_cases(oracle_mod):
    d = W.small_disk(M_dust_msun=1e-3, n_r=8, n_mu=6, n_lambda=16)
    ora = oracle_mod.Oracle(d)
    rng = np.random.default_rng(3)
    # absorbed energy per unit mass of the order a pass gives
    E = rng.uniform(0.5, 2.0, ora.n_cells) * ora.mass * (ora.L_star / ora.mass.sum())
    st = dict(E_abs=E, E_half=0.5 * E, visits=np.full(ora.n_cells, 500, np.uint32))
    T_prev, s2 = np.zeros(ora.n_cells), -np.ones(ora.n_cells)
    R, dx, noise, cells = ora.conv_stat(st, T_prev, s2)
    assert cells == 0 and R == 0.0                    # first pass: nothing to compare
    dusty = ora.mass > 0
    assert np.all(s2[dusty] == 0.0) and np.all(s2[~dusty] < 0)
    assert np.allclose(T_prev, ora.update_T(E), rtol=1e-14, atol=0)
    # all the energy in the odd half: the relative spread of E is 1, and T
    # follows with the slope of its inversion (about 1/5 here, where the
    # emission grows as kappa_P T^4 with kappa_P ~ T)
    st["E_half"] = E.copy()
    ora.conv_stat(st, T_prev, s2)
    # (the local slope of the tabulated inversion, read over +-1e-4 in E)
    slope = np.array([np.log(ora.T_of_E(e * 1.0001, m) / ora.T_of_E(e * 0.9999, m)) / 2e-4
                      for e, m in zip(E[dusty], ora.mass[dusty])])
    assert np.allclose(np.sqrt(s2[dusty]), slope, rtol=1e-9, atol=0)
    assert np.all((slope > 0.15) & (slope < 0.26))
    # too few packets: not eligible
    st["visits"][:] = 500
    st["visits"][dusty.nonzero()[0][:5]] = 10
    ora.conv_stat(st, T_prev, s2, n_min=100)
    assert (s2 >= 0).sum() == dusty.sum() - 5


def _pass(args):
    import oracle
    k, n = args
    d, o = W.config("mrw_pda")
    ora = oracle.Oracle(d, n_T=o.n_T)
    st = ora.run(n, 100 + k, mrw=True, gamma=o.gamma, n_int_min=o.n_int_min)
    return {key: st[key] for key in ("E_abs", "E_half", "n_abs", "n_mrw", "visits")}


@pytest.fixture(scope="module")
def passes():
    """Sixteen independent passes of the 1e-2 Msun workload, 1e5 packets."""
    with get_context("fork").Pool(8) as pool:
        return pool.map(_pass, [(k, 100000) for k in range(16)])


def test_split_noise_against_run_to_run_spread(oracle_mod, passes):
    d, o = W.config("mrw_pda")
    ora = oracle_mod.Oracle(d, n_T=o.n_T)
    Ts, S2, N, M = [], [], [], []
    for st in passes:
        T_prev, s2 = np.zeros(ora.n_cells), -np.ones(ora.n_cells)
        ora.conv_stat(st, T_prev, s2)
        Ts.append(T_prev)
        S2.append(s2)
        N.append(st["n_abs"].astype(np.float64))
        M.append(st["n_mrw"])
    Ts, S2, N, M = np.array(Ts), np.array(S2), np.array(N), np.array(M)
    ok = (S2.min(0) >= 0) & (N.min(0) > 0)
    assert ok.sum() >= 500
    var = Ts.var(0, ddof=1) / Ts.mean(0) ** 2
    ratio = var[ok].sum() / S2.mean(0)[ok].sum()
    mrw = ok & (M.min(0) > 0)
    assert mrw.sum() >= 20
    ratio_mrw = var[mrw].sum() / S2.mean(0)[mrw].sum()
    ratio_N = var[mrw].sum() / (1.0 / (16.0 * N)).mean(0)[mrw].sum()
    print("empirical / split estimate %.2f over %d cells, %.2f over the %d MRW cells, where "
          "empirical / (1/16N) is %.0f" % (ratio, ok.sum(), ratio_mrw, mrw.sum(), ratio_N))
    assert 0.8 < ratio < 1.25
    # in the MRW cells the halves share the running temperature, which a big
    # deposit raises for both: their positive covariance makes the split
    # estimate low there (by ~2.6 over these 29 cells)
    assert 1.0 < ratio_mrw < 5.0
    assert ratio_N > 20


def test_statistic_without_and_with_change(oracle_mod, passes):
    d, o = W.config("mrw_pda")
    ora = oracle_mod.Oracle(d, n_T=o.n_T)
    T_prev, s2 = np.zeros(ora.n_cells), -np.ones(ora.n_cells)
    ora.conv_stat(passes[0], T_prev, s2)
    Rs = []
    for st in passes[1:]:
        R, dx, noise, cells = ora.conv_stat(st, T_prev, s2)
        assert cells >= 40 and dx > 0 and noise > 0
        Rs.append(R)
    print("R over consecutive unchanged passes:", np.round(Rs, 2))
    assert 0.5 < float(np.mean(np.square(Rs))) < 1.5
    assert max(Rs) < 3.0          # an unchanged structure reads as converged
    # at 1e5 packets a cell's T carries ~10 % noise (R weighs the cells
    # equally, the paper's mean over the structure); a change of the previous
    # temperature by half of it is well outside
    T_prev *= 1.5
    R, dx, noise, cells = ora.conv_stat(passes[0], T_prev, s2)
    print("after a 50 %% change: R %.2f, rms change %.3f, rms noise %.3f" % (R, dx, noise))
    assert R > 3.0 and dx > 0.3
