"""FP64 CPU oracle for the sub-cycled radiation step (Section 3.2.1, the
sub-step paragraph after the gas-energy linearisation, the flux formula and
the radiation-subsystem algorithm that closes the section).

TEST INFRASTRUCTURE ONLY, like ``fld_oracle``: only the tests, the smoke check
and the benchmark's CPU leg may use it.

The step follows the paper's order of work:

1. S_adv of every cell from the state at the start of the step (E^n), and the
   series of sub-step lengths.
2. g, D and alpha at every interface, D from E^n (interior faces and the
   boundary faces alike).
3. C_V of every cell (from the current sub-step's T when a temperature law is
   given).
4.-6. The phi/psi coefficients of the sub-step with its own length dt_k
   (alpha = dt_k / h and beta = kappa_P rho c dt_k; D, g and S_adv from steps
   1-2), assembly, solve, and the gas update.
7. While sub-steps remain, alpha (the sub-step length) is updated and the
   work returns to step 3: D and S_adv are not recomputed.
8. The face flux, F = D^n sum_k alpha_k (E_lo^k - E_hi^k) / Delta t, i.e. the
   sub-step fluxes with the fixed D^n weighted by dt_k / Delta t (boundary
   faces: their fixed boundary terms, likewise weighted).

Sub-step lengths:

* Prescribed geometric series (Section 3.2.1, sub-timestep equation): for a
  step Delta t split into n sub-steps with geometric factor q,
      dt_i = dt_0 q^(i-1),  i = 1..n,   dt_0 = Delta t (1 - q) / (1 - q^n);
  q = 1 is read as the limit of that formula, n equal sub-steps Delta t / n;
  n = 1 is the step itself, dt_0 = Delta t exactly.
* Coupling-limited sub-steps (Section 3.2.1, global sub-step equation):
      dt = min(Delta t_remain, min over cells of dbar T C_V / |G0|),
      G0 = kappa_P rho c (a_R T^4 - E),
  evaluated from the state at the start of every sub-step.  Readings: C_V is
  per unit volume (rho c_v, as in the step itself), so the paper's rho C_V
  with C_V per gram is rho c_v here; the limit is taken over every cell of
  the grid (the sub-step is global, one linear system); a cell in exact
  equilibrium (G0 = 0) does not limit; the loop ends once the remaining time
  is at most 1e-12 Delta t, and fails after max_sub sub-steps.

Opacities and rho are held fixed over the sub-steps (they are inputs of the
radiation step); E and T advance.  The heat capacity is recomputed from T at
the start of every sub-step (step 3) when a temperature law is given: the
analytic power law
      c_v(T) = c_v,ref (T / T_ref)^p,
c_v,ref being the caller's c_v array (its value at T_ref), stands in for a
nonlinear equation of state; p = 0, or no law, keeps c_v fixed.  Each
sub-step then linearises the gas energy about its own start, C_V = rho c_v(T)
(the paper's linearised coupling equation for a nonlinear gas energy).

Parity status: pinned by tests/test_oracle_substep.py (the series' closed-form
invariants; the temperature-change bound that dbar is meant to enforce on the
paper's 0D coupling set-up and first-order convergence of both schedules to an
implicit Runge-Kutta solution of that set-up's ODE pair; without gas coupling
on a medium whose D depends on E, the sub-cycled E equals the product of the
sub-steps' resolvents built densely from the step-start operator, and every
cell closes its balance with the averaged flux and Delta t S_adv(E^n)),
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
    Fx: np.ndarray     # [ny][nx+1] face flux averaged over the step (step 8)
    Fy: np.ndarray     # [ny+1][nx]


def substep(geom, xf, yf, E, T, rho, kappa_R, kappa_P, c_v, dt, bcs, *, n_sub: int = 1, q: float = 1.0,
            dbar: float = 0.0, max_sub: int = 10000, limiter=O.LIMITER_LP, fx=None, fy=None,
            cv_law=None) -> SubstepResult:
    """One radiation step of length dt taken in sub-steps: the geometric series
    (n_sub, q) when dbar == 0, else coupling-limited sub-steps with factor dbar.
    fx, fy: face mass fluxes of the advection term (S_adv from the step's
    start, applied in every sub-step for its length).
    cv_law: None, or (T_ref, p) of the power law, c_v then being its c_v,ref."""
    E_n = np.asarray(E, dtype=np.float64)
    E = E_n
    T = np.asarray(T, dtype=np.float64)
    sig = np.asarray(kappa_R, dtype=np.float64) * np.asarray(rho, dtype=np.float64)
    ny, nx = E.shape
    dts: List[float] = []
    Fx = np.zeros((ny, nx + 1))
    Fy = np.zeros((ny + 1, nx))

    def heat_capacity(T):
        if cv_law is None or cv_law[1] == 0.0:
            return c_v
        return cv_power_law(c_v, T, cv_law[0], cv_law[1])

    def one(E, T, cv_k, h):
        # steps 4-6 for a sub-step of length h: D and S_adv from E^n (steps
        # 1-2), the time derivative from the sub-step's own E
        A = O.assemble(geom, xf, yf, E, T, rho, kappa_R, kappa_P, cv_k, h, bcs, limiter, fx, fy, E_op=E_n)
        E_new = O.solve(A)
        T_new = O.gas_update(A, T, E_new)
        gx, gy = O.face_fluxes(A, E_n, E_new, sig, h, bcs, limiter)
        Fx[...] += (h / dt) * gx
        Fy[...] += (h / dt) * gy
        return E_new, T_new

    if dbar == 0.0:
        for h in geometric_substeps(dt, q, n_sub):
            E, T = one(E, T, heat_capacity(T), float(h))
            dts.append(float(h))
        return SubstepResult(E, T, dts, Fx, Fy)
    if not (dbar > 0.0):
        raise ValueError("dbar must be >= 0")
    remain = float(dt)
    while remain > 1e-12 * dt:
        if len(dts) == max_sub:
            raise RuntimeError("sub-step limit reached")
        cv_k = heat_capacity(T)
        h = min(remain, coupling_dt(E, T, rho, kappa_P, cv_k, dbar))
        E, T = one(E, T, cv_k, h)
        dts.append(h)
        remain -= h
    return SubstepResult(E, T, dts, Fx, Fy)


def substep_problem(prob, **kw) -> SubstepResult:
    return substep(prob.geom, prob.x_faces, prob.y_faces, prob.E, prob.T, prob.rho, prob.kappa_R, prob.kappa_P,
                   prob.c_v, prob.dt, O.bcs_from_problem(prob), **kw)
