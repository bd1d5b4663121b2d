"""FP64 CPU oracle for the sub-cycled radiation step (Section 3.2.1, the
sub-step paragraph after the gas-energy linearisation).

TEST INFRASTRUCTURE ONLY, like ``fld_oracle``: only the tests, the smoke check
and the benchmark's CPU leg may use it.  It calls ``fld_oracle.step`` for each
sub-step and adds nothing but the choice of the sub-step lengths:

* Prescribed geometric series (Section 3.2.1, sub-timestep equation): for a
  step Delta t split into n sub-steps with geometric factor q,
      dt_i = dt_0 q^(i-1),  i = 1..n,   dt_0 = Delta t (1 - q) / (1 - q^n);
  q = 1 is read as the limit of that formula, n equal sub-steps Delta t / n;
  n = 1 is the step itself, dt_0 = Delta t exactly.
* Coupling-limited sub-steps (Section 3.2.1, global sub-step equation):
      dt = min(Delta t_remain, min over cells of dbar T C_V / |G0|),
      G0 = kappa_P rho c (a_R T^4 - E),
  evaluated from the state at the start of each sub-step.  Readings: C_V is
  per unit volume (rho c_v, as in the step itself), so the paper's rho C_V
  with C_V per gram is rho c_v here; the limit is taken over every cell of
  the grid (the sub-step is global, one linear system); a cell in exact
  equilibrium (G0 = 0) does not limit; the loop ends once the remaining time
  is at most 1e-12 Delta t, and fails after max_sub sub-steps.

Opacities and rho are held fixed over the sub-steps (they are inputs of the
radiation step); E and T advance.  The heat capacity is recomputed from T at
the start of every sub-step (the radiation-subsystem algorithm returns to its
C_V step before each sub-step) when a temperature law is given: the analytic
power law
      c_v(T) = c_v,ref (T / T_ref)^p,
c_v,ref being the caller's c_v array (its value at T_ref), stands in for a
nonlinear equation of state; p = 0, or no law, keeps c_v fixed.  Each
sub-step then linearises the gas energy about its own start, C_V = rho c_v(T)
(the paper's linearised coupling equation for a nonlinear gas energy).

Parity status: pinned by tests/test_oracle_substep.py (the series' closed-form
invariants, the temperature-change bound that dbar is meant to enforce on the
paper's 0D coupling set-up, and first-order convergence of both schedules to
an implicit Runge-Kutta solution of that set-up's ODE pair) and
tests/test_oracle_cv_law.py (the power law's values, its p = 0 case, and
first-order convergence of the sub-stepped scheme to the ODE pair with the
temperature-dependent heat capacity, which the fixed-c_v scheme misses).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from . import fld_oracle as O


def geometric_substeps(dt: float, q: float, n: int) -> np.ndarray:
    """The n sub-step lengths of the geometric series (Section 3.2.1)."""
    if n < 1 or not (q > 0.0) or not (dt > 0.0):
        raise ValueError("need n >= 1, q > 0, dt > 0")
    i = np.arange(1, n + 1, dtype=np.float64)
    if n == 1:
        return np.array([float(dt)])  # dt_0 = dt exactly (the formula's quotient rounds)
    if q == 1.0:
        return np.full(n, dt / n)
    dt0 = dt * (1.0 - q) / (1.0 - q ** n)
    return dt0 * q ** (i - 1.0)


def coupling_dt(E, T, rho, kappa_P, c_v, dbar: float) -> float:
    """min over cells of dbar T C_V / |G0| (Section 3.2.1); inf if no cell couples."""
    E = np.asarray(E, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    G0 = np.asarray(kappa_P) * np.asarray(rho) * O.C_LIGHT * (O.A_RAD * T ** 4 - E)
    CV = np.asarray(rho) * np.asarray(c_v)
    with np.errstate(divide="ignore"):
        lim = np.where(G0 != 0.0, dbar * T * CV / np.abs(G0), np.inf)
    return float(lim.min())


def cv_power_law(c_v_ref, T, T_ref: float, p: float) -> np.ndarray:
    """Specific heat at temperature T of the power-law stand-in for a nonlinear
    equation of state: c_v,ref (T / T_ref)^p."""
    if not (T_ref > 0.0) or not math.isfinite(p):
        raise ValueError("need T_ref > 0 and a finite p")
    return np.asarray(c_v_ref, dtype=np.float64) * (np.asarray(T, dtype=np.float64) / T_ref) ** p


@dataclasses.dataclass
class SubstepResult:
    E: np.ndarray
    T: np.ndarray
    dts: List[float]


def substep(geom, xf, yf, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, *, n_sub: int = 1, q: float = 1.0,
            dbar: float = 0.0, max_sub: int = 10000, limiter=O.LIMITER_LP, fx=None, fy=None,
            cv_law=None) -> SubstepResult:
    """One radiation step of length dt taken in sub-steps: the geometric series
    (n_sub, q) when dbar == 0, else coupling-limited sub-steps with factor dbar.
    fx, fy: face mass fluxes of the advection term, applied in every sub-step.
    cv_law: None, or (T_ref, p) of the power law, c_v then being its c_v,ref."""
    E = np.asarray(E, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    dts: List[float] = []

    def heat_capacity(T):
        if cv_law is None or cv_law[1] == 0.0:
            return c_v
        return cv_power_law(c_v, T, cv_law[0], cv_law[1])

    if dbar == 0.0:
        for h in geometric_substeps(dt, q, n_sub):
            r = O.step(geom, xf, yf, E, T, rho, kappa_R, kappa_P, heat_capacity(T), float(h), bcs, limiter, fx, fy)
            E, T = r.E, r.T
            dts.append(float(h))
        return SubstepResult(E, T, dts)
    if not (dbar > 0.0):
        raise ValueError("dbar must be >= 0")
    remain = float(dt)
    while remain > 1e-12 * dt:
        if len(dts) == max_sub:
            raise RuntimeError("sub-step limit reached")
        cv_k = heat_capacity(T)
        h = min(remain, coupling_dt(E, T, rho, kappa_P, cv_k, dbar))
        r = O.step(geom, xf, yf, E, T, rho, kappa_R, kappa_P, cv_k, h, bcs, limiter, fx, fy)
        E, T = r.E, r.T
        dts.append(h)
        remain -= h
    return SubstepResult(E, T, dts)


def substep_problem(prob, **kw) -> SubstepResult:
    return substep(prob.geom, prob.x_faces, prob.y_faces, prob.E, prob.T, prob.rho, prob.kappa_R, prob.kappa_P,
                   prob.c_v, prob.dt, O.bcs_from_problem(prob), **kw)
