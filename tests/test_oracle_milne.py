"""Pins for the Milne boundary (Section 5.2 radiative-shock set-up: the
blackbody-absorber condition E = -2/(3 rho kappa_R) dE/dn, Castor 2004 ch. 11).

A slab fed a fixed flux F through one side and closed by the Milne condition
on the other has, in steady state without gas coupling, the linear profile
E(x) = E_b + (F / D)(L - x) with E_b = 2/(3 sigma) F / D; with the
diffusion-limit coefficient D = c / (3 sigma) this is Marshak's vacuum
relation E_b = 2 F / c.  The scheme holds the linear profile exactly at the
cell centres; the steady outflow equals the inflow for any limiter; and the
condition is the same on either side (mirror symmetry).
"""
import numpy as np
import pytest

from oracle import fld_oracle as O


def slab(N, F, sig, milne_side, lim, L=2.0, dt=1e6, xf=None):
    xf = np.linspace(0.0, L, N + 1) if xf is None else xf
    one = np.ones((1, N))
    bcs = [O.BCSpec(O.FLUX_IN, F), O.BCSpec(O.MILNE)] + [O.BCSpec()] * 2
    if milne_side == 0:
        bcs[0], bcs[1] = O.BCSpec(O.MILNE), O.BCSpec(O.FLUX_IN, F)
    E = one * 1e3
    r = O.step(O.CARTESIAN, xf, np.array([0.0, 1.0]), E, 1e3 * one, one, sig * one, 0.0 * one, one, dt, bcs, lim)
    return xf, r


@pytest.mark.parametrize("N", [16, 100])
def test_steady_slab_linear_profile_diffusion_limit(N):
    F, sig, L = 3.0e12, 5.0, 2.0
    xf, r = slab(N, F, sig, 1, O.LIMITER_DIFFUSION, L=L)
    D = O.C_LIGHT / (3.0 * sig)
    xc = 0.5 * (xf[1:] + xf[:-1])
    exact = 2.0 * F / O.C_LIGHT + F / D * (L - xc)
    np.testing.assert_allclose(r.E[0], exact, rtol=1e-9)


def test_marshak_limit_at_the_face():
    # the last cell's centre value tends to E_b = 2F/c as the cell shrinks
    F, sig = 1.0e10, 2.0
    errs = []
    for N in (10, 100, 1000):
        xf, r = slab(N, F, sig, 1, O.LIMITER_DIFFUSION, L=1.0)
        errs.append(abs(r.E[0, -1] / (2.0 * F / O.C_LIGHT) - 1.0))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-2


@pytest.mark.parametrize("lim", [O.LIMITER_LP, O.LIMITER_MINERBO, O.LIMITER_DIFFUSION])
def test_steady_outflow_equals_inflow(lim):
    F, sig = 7.0e11, 0.3
    xf = np.cumsum(np.r_[0.0, np.random.default_rng(2).uniform(0.5, 1.5, 40)])
    xf, r = slab(40, F, sig, 1, lim, xf=xf)
    A = r.A
    h1 = xf[-1] - 0.5 * (xf[-1] + xf[-2])
    a = 2.0 / (3.0 * sig * h1)
    lam = O.LIMITERS[lim](np.array([1.5]))[0]
    out = O.C_LIGHT * lam / sig * r.E[0, -1] / (h1 * (1.0 + a))
    assert out == pytest.approx(F, rel=1e-9)
    assert A.bdiag[0, -1] > 0 and A.brhs[0, -1] == 0.0


def test_mirror_symmetry():
    F, sig = 2.0e11, 1.7
    _, right = slab(30, F, sig, 1, O.LIMITER_LP)
    _, left = slab(30, F, sig, 0, O.LIMITER_LP)
    np.testing.assert_allclose(left.E[0, ::-1], right.E[0], rtol=1e-12)
