"""Pins for the temperature-dependent heat capacity of the sub-step oracle
(Section 3.2.1: the radiation-subsystem algorithm recomputes C_V before every
sub-step; Section 5.1.2: a nonlinear gas energy is linearised with
C_V = d e_g / dT).

The power law c_v(T) = c_v,ref (T / T_ref)^p stands in for a nonlinear
equation of state.  Its gas energy per volume is
    e_g(T) = rho c_v,ref T_ref / (p + 1) (T / T_ref)^(p + 1),
so the 0D coupling set-up of Section 5.1.1 (golden/e1_coupling.txt) becomes
the ODE pair dE/dt = k (a T^4 - E), rho c_v(T) dT/dt = -k (a T^4 - E),
k = kappa_P rho c, which conserves E + e_g(T).

* The law's values at T_ref and at 2 T_ref, and p = 0 leaving the step as
  it is with no law.
* Cooling gas from e_g = 1e10 erg/cm^3 with p = 1.5: the sub-stepped scheme
  converges at first order to an implicit Runge-Kutta solution of the ODE
  pair (coupling-limited and nested geometric schedules), while the scheme
  that keeps c_v fixed converges to another trajectory (40 % off at the
  end): a law applied the wrong way round, or not re-evaluated per
  sub-step, fails here.
* The drift of E + e_g(T) falls at first order with the sub-step.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import fld_oracle as O
from oracle import fld_substep as S

K_B = 1.380649e-16
M_H = 1.6735575e-24
# Section 5.1.1 set-up (the values of golden/e1_coupling.txt)
E_R, RHO, KAPPA_P, MU = 1.0e12, 1.0e-7, 0.4, 0.6


def state(eg0, nx=8):
    cv = 3.0 * K_B / (2.0 * MU * M_H)
    shape = (1, nx)
    return dict(geom=O.CARTESIAN, xf=np.linspace(0.0, 1.0, nx + 1), yf=np.linspace(0.0, 1.0, 2),
                E=np.full(shape, E_R), T=np.full(shape, eg0 / (RHO * cv)), rho=np.full(shape, RHO),
                kappa_R=np.full(shape, 1e10 / RHO), kappa_P=np.full(shape, KAPPA_P), c_v=np.full(shape, cv),
                bcs=[O.BCSpec()] * 4), cv


def ode_T(T0, ts, cv, T_ref, p):
    k = KAPPA_P * RHO * O.C_LIGHT

    def rhs(t, y):
        s = k * (y[0] - O.A_RAD * y[1] ** 4)
        return [-s, s / (RHO * cv * (y[1] / T_ref) ** p)]

    sol = solve_ivp(rhs, (0.0, ts[-1]), [E_R, T0], method="Radau", rtol=1e-11, atol=[1e-3, 1e-12 * T0],
                    t_eval=ts)
    return sol.y[1]


def run(f, dt, **kw):
    return S.substep(f["geom"], f["xf"], f["yf"], f["E"], f["T"], f["rho"], f["kappa_R"], f["kappa_P"], f["c_v"],
                     dt, f["bcs"], **kw)


def trajectory(f, dts, cv, law):
    """T after each sub-step, replayed one O.step at a time."""
    E, T, Ts = f["E"], f["T"], []
    for h in dts:
        c = cv if law is None else S.cv_power_law(f["c_v"], T, *law)
        s = O.step(f["geom"], f["xf"], f["yf"], E, T, f["rho"], f["kappa_R"], f["kappa_P"], c, h, f["bcs"])
        E, T = s.E, s.T
        assert np.ptp(T) <= 1e-12 * T.max()
        Ts.append(T[0, 0])
    return np.array(Ts), E[0, 0]


def test_power_law_values_and_p0():
    c = np.array([[2.0, 3.0]])
    np.testing.assert_array_equal(S.cv_power_law(c, np.array([[7.0, 7.0]]), 7.0, 1.5), c)
    np.testing.assert_allclose(S.cv_power_law(c, np.array([[14.0, 3.5]]), 7.0, 1.5),
                               [[2.0 * 2.0 ** 1.5, 3.0 * 0.5 ** 1.5]], rtol=1e-15)
    with pytest.raises(ValueError):
        S.cv_power_law(c, c, 0.0, 1.0)
    f, cv = state(1e10, nx=4)
    a = run(f, 1e-8, n_sub=3, q=1.5, cv_law=(1e6, 0.0))
    b = run(f, 1e-8, n_sub=3, q=1.5)
    np.testing.assert_array_equal(a.T, b.T)
    np.testing.assert_array_equal(a.E, b.E)


def test_cooling_coupling_limited_first_order():
    f, cv = state(1e10)
    T0 = f["T"][0, 0]
    law = ((E_R / O.A_RAD) ** 0.25, 1.5)
    dt = 3e-7
    errs, fixed = [], []
    for dbar in (0.04, 0.02):
        r = run(f, dt, dbar=dbar, cv_law=law)
        assert math.fsum(r.dts) == pytest.approx(dt, rel=1e-12)
        Ts, _ = trajectory(f, r.dts, cv, law)
        np.testing.assert_array_equal(Ts[-1], r.T[0, 0])
        # each sub-step's limit used the law's C_V at its start
        assert np.max(np.abs(np.diff(np.r_[T0, Ts])) / np.r_[T0, Ts][:-1]) <= dbar * (1 + 1e-9)
        ref = ode_T(T0, np.cumsum(r.dts), cv, *law)
        errs.append(np.max(np.abs(Ts - ref) / ref))
        r0 = run(f, dt, dbar=dbar)
        fixed.append(abs(r0.T[0, 0] - ref[-1]) / ref[-1])
    assert errs[1] < 0.05
    assert 1.5 < errs[0] / errs[1] < 2.5, errs  # first order: near 2
    assert min(fixed) > 0.2, fixed  # the fixed-c_v scheme follows another ODE


def test_cooling_geometric_series_first_order_and_energy():
    f, cv = state(1e10)
    T0 = f["T"][0, 0]
    T_ref, p = (E_R / O.A_RAD) ** 0.25, 1.5
    dt = 3e-7
    # nested series (q^(1/4), 240) inside (q^(1/2), 120), compared at the
    # coarse sub-step ends; equal sub-steps overshoot in the stiff first one
    ts = np.cumsum(S.geometric_substeps(dt, 1.2 ** 0.5, 120))
    ref = ode_T(T0, ts, cv, T_ref, p)

    def e_g(T):
        return RHO * cv * T_ref / (p + 1.0) * (T / T_ref) ** (p + 1.0)

    total0 = E_R + e_g(T0)
    errs, drift = [], []
    for q, n in ((1.2 ** 0.5, 120), (1.2 ** 0.25, 240)):
        r = run(f, dt, n_sub=n, q=q, cv_law=(T_ref, p))
        Ts, E_end = trajectory(f, r.dts, cv, (T_ref, p))
        np.testing.assert_array_equal(Ts[-1], r.T[0, 0])
        Ts = Ts[n // 120 - 1::n // 120]
        errs.append(np.max(np.abs(Ts - ref) / ref))
        drift.append(abs(E_end + e_g(r.T[0, 0]) - total0) / total0)
    assert errs[1] < 0.1
    assert 1.5 < errs[0] / errs[1] < 2.5, errs
    assert 1.5 < drift[0] / drift[1] < 2.5, drift
