"""Pins for the sub-cycled radiation step oracle (Section 3.2.1, sub-step
series and coupling-limited sub-step; Section 5.1.1 0D coupling set-up).

* The geometric series sums to the step, grows by q, reduces to equal steps at
  q = 1, and the series for (2n, sqrt q) splits every sub-step of (n, q) into
  two: a nested refinement.
* The coupling limit equals its closed form for one cell and a brute-force
  minimum over a small random grid; an equilibrium grid does not limit.
* On the paper's 0D coupling set-up (golden/e1_coupling.txt) the
  coupling-limited sub-steps keep every sub-step's relative temperature
  change below dbar (the purpose the paper gives the factor), and both
  schedules converge at first order to an implicit Runge-Kutta solution of the
  ODE pair as dbar, or the nested series, is refined.
"""
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import fld_oracle as O
from oracle import fld_substep as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "e1_coupling.txt")
K_B = 1.380649e-16
M_H = 1.6735575e-24


def golden():
    out = {}
    for line in open(GOLD):
        line = line.strip()
        if line and not line.startswith("#"):
            k, *v = line.split()
            out[k] = [float(x) for x in v] if len(v) > 1 else float(v[0])
    return out


@pytest.mark.parametrize("dt,q,n", [(1.0, 1.5, 7), (3e-7, 1.01, 200), (2.5e3, 1.999, 30), (1e-9, 1.0, 13)])
def test_geometric_series_invariants(dt, q, n):
    h = S.geometric_substeps(dt, q, n)
    assert len(h) == n and np.all(h > 0)
    assert math.fsum(h) == pytest.approx(dt, rel=1e-14)
    np.testing.assert_allclose(h[1:] / h[:-1], q, rtol=1e-13)
    if q == 1.0:
        np.testing.assert_array_equal(h, np.full(n, dt / n))
    assert S.geometric_substeps(dt, q, 1)[0] == dt


@pytest.mark.parametrize("q,n", [(1.3, 10), (1.05, 64)])
def test_geometric_series_nests(q, n):
    coarse = S.geometric_substeps(1.0, q, n)
    fine = S.geometric_substeps(1.0, math.sqrt(q), 2 * n)
    np.testing.assert_allclose(fine[0::2] + fine[1::2], coarse, rtol=1e-13)


def test_coupling_limit_closed_form_and_brute_force():
    E, T, rho, kP, cv, dbar = 1e12, 4.9, 1e-7, 0.4, 2.06e8, 0.02
    G0 = kP * rho * O.C_LIGHT * (O.A_RAD * T ** 4 - E)
    one = S.coupling_dt(np.array([[E]]), np.array([[T]]), np.array([[rho]]), np.array([[kP]]), np.array([[cv]]), dbar)
    assert one == pytest.approx(dbar * T * rho * cv / abs(G0), rel=1e-15)
    rng = np.random.default_rng(3)
    shp = (3, 4)
    T = 10 ** rng.uniform(3, 6, shp)
    E = O.A_RAD * T ** 4 * 10 ** rng.uniform(-1, 1, shp)
    rho, kP, cv = 10 ** rng.uniform(-9, -6, shp), 10 ** rng.uniform(-2, 2, shp), 10 ** rng.uniform(7, 9, shp)
    best = math.inf
    for j in range(shp[0]):
        for i in range(shp[1]):
            g = kP[j, i] * rho[j, i] * O.C_LIGHT * (O.A_RAD * T[j, i] ** 4 - E[j, i])
            best = min(best, 0.05 * T[j, i] * rho[j, i] * cv[j, i] / abs(g))
    assert S.coupling_dt(E, T, rho, kP, cv, 0.05) == pytest.approx(best, rel=1e-14)
    eq = S.coupling_dt(O.A_RAD * T ** 4, T, rho, kP, cv, 0.05)
    assert eq == math.inf


def e1_state(eg0, nx=16):
    g = golden()
    rho, kP = g["rho_g_per_cm3"], g["kappa_P_cm2_per_g"]
    cv = 3.0 * K_B / (2.0 * g["mu"] * M_H)
    shape = (1, nx)
    f = dict(geom=O.CARTESIAN, xf=np.linspace(0.0, 1.0, nx + 1), yf=np.linspace(0.0, 1.0, 2),
             E=np.full(shape, g["E_r_erg_per_cm3"]), T=np.full(shape, eg0 / (rho * cv)), rho=np.full(shape, rho),
             kappa_R=np.full(shape, 1e10 / rho), kappa_P=np.full(shape, kP), c_v=np.full(shape, cv),
             bcs=[O.BCSpec()] * 4)
    return f, g, cv


def ode_eg(eg0, ts, g, cv):
    """Gas energy of the ODE pair at the times ts (implicit Runge-Kutta)."""
    rho, kP = g["rho_g_per_cm3"], g["kappa_P_cm2_per_g"]
    k, CV = kP * rho * O.C_LIGHT, rho * cv

    def rhs(t, y):
        s = k * (y[0] - O.A_RAD * (y[1] / CV) ** 4)
        return [-s, s]

    ts = np.asarray(ts, dtype=np.float64)
    sol = solve_ivp(rhs, (0.0, ts[-1]), [g["E_r_erg_per_cm3"], eg0], method="Radau", rtol=1e-11,
                    atol=[1e-3, 1e-12], t_eval=ts)
    return sol.y[1]


def run(f, dt, **kw):
    return S.substep(f["geom"], f["xf"], f["yf"], f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"],
                     dt, f["bcs"], **kw)


@pytest.mark.parametrize("eg0", [1e2, 1e10])
def test_e1_coupling_limited_substeps(eg0):
    f, g, cv = e1_state(eg0)
    dt = 3e-7
    errs = []
    for dbar in (0.04, 0.02):
        r = run(f, dt, dbar=dbar)
        assert math.fsum(r.dts) == pytest.approx(dt, rel=1e-12)
        # replay the sub-steps: every cell stays uniform, and the relative
        # temperature change of each sub-step is bounded by dbar
        Ts = [f["T"][0, 0]]
        E, T = f["E"], f["T"]
        for h in r.dts:
            s = O.step(f["geom"], f["xf"], f["yf"], E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], h, f["bcs"])
            E, T = s.E, s.T
            assert np.ptp(T) <= 1e-12 * T.max()
            Ts.append(T[0, 0])
        np.testing.assert_array_equal(T, r.T)
        Ts = np.array(Ts)
        assert np.max(np.abs(np.diff(Ts)) / Ts[:-1]) <= dbar * (1 + 1e-9)
        # largest error along the trajectory against the ODE pair
        ref = ode_eg(eg0, np.cumsum(r.dts), g, cv)
        errs.append(np.max(np.abs(Ts[1:] * f["rho"][0, 0] * cv - ref) / ref))
    assert errs[1] < 0.02
    assert 1.5 < errs[0] / errs[1] < 2.5, errs  # first order: near 2 (zeroth: near 1)


def test_e1_geometric_series_first_order():
    eg0 = 1e6
    f, g, cv = e1_state(eg0)
    dt = 2e-7
    # the (240, q^(1/4)) series is nested in the (120, q^(1/2)) one: compare
    # both at the coarse sub-step ends along the trajectory (a coarser pair
    # still changes T by most of itself in its first sub-step)
    ts = np.cumsum(S.geometric_substeps(dt, 1.2 ** 0.5, 120))
    ref = ode_eg(eg0, ts, g, cv)
    errs = []
    for q, n in ((1.2 ** 0.5, 120), (1.2 ** 0.25, 240)):
        egs = []
        E, T = f["E"], f["T"]
        for h in S.geometric_substeps(dt, q, n):
            s = O.step(f["geom"], f["xf"], f["yf"], E, T, f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], h, f["bcs"])
            E, T = s.E, s.T
            egs.append(T[0, 0] * f["rho"][0, 0] * cv)
        r = run(f, dt, n_sub=n, q=q)
        assert len(r.dts) == n
        np.testing.assert_array_equal(r.T, T)
        egs = np.array(egs)[n // 120 - 1::n // 120]
        errs.append(np.max(np.abs(egs - ref) / ref))
    assert errs[1] < 0.05
    assert 1.5 < errs[0] / errs[1] < 2.5, errs  # first order: near 2 (zeroth: near 1)


def test_single_substep_is_one_step():
    f, g, cv = e1_state(1e6, nx=4)
    r = run(f, 1e-9, n_sub=1, q=1.5)
    s = O.step(f["geom"], f["xf"], f["yf"], f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"], 1e-9,
               f["bcs"])
    np.testing.assert_array_equal(r.E, s.E)
    np.testing.assert_array_equal(r.T, s.T)
