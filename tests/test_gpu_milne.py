"""Milne boundary (blackbody absorber, Section 5.2 set-up) through the C ABI
against the oracle: on a stretched Cartesian and a spherical-polar recipe in
place of their outer boundaries, in both precisions, and the steady slab
whose centre values follow the analytic linear profile."""
import numpy as np
import pytest

import fld_workloads as W
from oracle import fld_oracle as O
from gpu_helpers import gpu_step, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,kw,side", [("c1", dict(nx=48, ny=40), 1), ("c1", dict(nx=48, ny=40), 2),
                                          ("c5", dict(nx=64, ny=48), 1)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_milne_side_matches_oracle(lib, name, kw, side, prec):
    prob = W.make(name, **kw)
    prob.bc[side] = W.BC(W.BC_MILNE)
    ref = O.step_problem(prob)
    E, T, info = gpu_step(lib, torch, prob, precision=prec, rel_tol=1e-12, norm=1)
    assert info["status"] == 0
    assert rel_l2(E, ref.E) < 1e-10 and rel_l2(T, ref.T) < 1e-10


def test_steady_slab_on_gpu(lib):
    N, F, sig, L = 100, 3.0e12, 5.0, 2.0
    xf = np.linspace(0.0, L, N + 1)
    one = np.ones((1, N))
    prob = W.Problem("slab", W.GEOM_CARTESIAN, xf, np.array([0.0, 1.0]), 1e3 * one, 1e3 * one, one.copy(),
                     sig * one, 0.0 * one, one.copy(), 1e6,
                     [W.BC(W.BC_FLUX_IN, F), W.BC(W.BC_MILNE), W.BC(), W.BC()])
    E, T, info = gpu_step(lib, torch, prob, precision="fp64", limiter=2, rel_tol=1e-12, norm=1)
    assert info["status"] == 0
    xc = 0.5 * (xf[1:] + xf[:-1])
    D = O.C_LIGHT / (3.0 * sig)
    np.testing.assert_allclose(E[0], 2.0 * F / O.C_LIGHT + F / D * (L - xc), rtol=1e-9)
