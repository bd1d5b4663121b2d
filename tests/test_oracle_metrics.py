"""Pins for the oracle's grid metrics (Section 3.2.1: g = dS/dV, alpha at volume centres).

Volumes, areas and volume centres are checked against numerical quadrature of
their defining integrals (scipy), total volumes against closed forms, and face
areas against the divergence theorem for fields whose divergence is known.
"""
import numpy as np
import pytest
from scipy import integrate

from oracle import fld_oracle as O
import fld_workloads as W


def sph_grid(nx=7, ny=5):
    return W.log_faces(nx, 1e11, 1e14), W.theta_faces(ny)


def test_cartesian_total_volume_and_divergence():
    xf = W.stretched_faces(9, 1.0, 1.3)
    yf = W.stretched_faces(6, 2.0, 0.8)
    m = O.metrics(O.CARTESIAN, xf, yf)
    assert m.dV.sum() == pytest.approx((xf[-1] - xf[0]) * (yf[-1] - yf[0]), rel=1e-14)
    # F = x e_x has div F = 1: x_{i+1/2} dS - x_{i-1/2} dS = dV
    lhs = xf[None, 1:] * m.dSx[:, 1:] - xf[None, :-1] * m.dSx[:, :-1]
    np.testing.assert_allclose(lhs, m.dV, rtol=1e-12)
    lhs = yf[1:, None] * m.dSy[1:, :] - yf[:-1, None] * m.dSy[:-1, :]
    np.testing.assert_allclose(lhs, m.dV, rtol=1e-12)
    # centre distances: cell centres at midpoints
    xc = 0.5 * (xf[1:] + xf[:-1])
    np.testing.assert_allclose(m.hLx[0, 1:-1] + m.hRx[0, 1:-1], np.diff(xc), rtol=1e-14)


def test_spherical_total_volume():
    xf, yf = sph_grid(11, 9)
    m = O.metrics(O.SPHERICAL, xf, yf)
    assert m.dV.sum() == pytest.approx((xf[-1] ** 3 - xf[0] ** 3) / 3.0 * 2.0, rel=1e-13)


def test_spherical_cell_quadrature():
    xf, yf = sph_grid(4, 3)
    xf = np.linspace(1.0, 3.0, 5)  # moderate radii so quadrature is well conditioned
    m = O.metrics(O.SPHERICAL, xf, yf)
    for j in range(3):
        for i in range(4):
            r0, r1, t0, t1 = xf[i], xf[i + 1], yf[j], yf[j + 1]
            vol = integrate.dblquad(lambda t, r: r * r * np.sin(t), r0, r1, t0, t1, epsabs=0, epsrel=1e-13)[0]
            assert m.dV[j, i] == pytest.approx(vol, rel=1e-11)
            rc = integrate.dblquad(lambda t, r: r ** 3 * np.sin(t), r0, r1, t0, t1, epsabs=0, epsrel=1e-13)[0] / vol
            tc = integrate.dblquad(lambda t, r: t * r * r * np.sin(t), r0, r1, t0, t1, epsabs=0, epsrel=1e-13)[0] / vol
            # h_R of the cell's left face = r_c - r_-, h_R of its lower theta face = r_c (th_c - th_-)
            assert m.hRx[j, i] == pytest.approx(rc - r0, rel=1e-11)
            assert m.hRy[j, i] == pytest.approx(rc * (tc - t0), rel=1e-10)
            assert m.hLx[j, i + 1] == pytest.approx(r1 - rc, rel=1e-11)
            assert m.hLy[j + 1, i] == pytest.approx(rc * (t1 - tc), rel=1e-10)
            # r-face area: integral of r_f^2 sin t over the face
            area = integrate.quad(lambda t: r0 * r0 * np.sin(t), t0, t1, epsabs=0, epsrel=1e-13)[0]
            assert m.dSx[j, i] == pytest.approx(area, rel=1e-11)
            area = integrate.quad(lambda r: r * np.sin(t0), r0, r1, epsabs=0, epsrel=1e-13)[0]
            assert m.dSy[j, i] == pytest.approx(area, rel=1e-11, abs=1e-14)


def test_spherical_divergence_theorem():
    xf, yf = sph_grid(8, 6)
    m = O.metrics(O.SPHERICAL, xf, yf)
    # F = r e_r, div F = 3: r_+ dS_+ - r_- dS_- = 3 dV
    lhs = xf[None, 1:] * m.dSx[:, 1:] - xf[None, :-1] * m.dSx[:, :-1]
    np.testing.assert_allclose(lhs, 3.0 * m.dV, rtol=1e-12)
    # constant field e_z = cos t e_r - sin t e_t has zero net flux through each cell.
    # r-face flux integrates cos t sin t over the face: r_f^2 (sin^2 t+ - sin^2 t-)/2
    sp, sm = np.sin(yf[1:]) ** 2, np.sin(yf[:-1]) ** 2
    flux_r = (xf[None, 1:] ** 2 - xf[None, :-1] ** 2) * (0.5 * (sp - sm))[:, None]
    # theta-face flux is -sin(t_f) times the face area
    st = np.sin(yf)[:, None]
    flux_t = -(st[1:] * m.dSy[1:, :] - st[:-1] * m.dSy[:-1, :])
    np.testing.assert_allclose(flux_r + flux_t, 0.0, atol=1e-12 * np.abs(flux_r).max())


def test_axis_faces_have_no_area():
    xf, yf = sph_grid(5, 4)
    m = O.metrics(O.SPHERICAL, xf, yf)
    assert np.all(m.dSy[0, :] == 0.0)
    assert np.all(np.abs(m.dSy[-1, :]) < 1e-15 * m.dSy.max())


def test_theta_centre_offset_high_precision():
    # the volume-weighted mean angle of thin cells, at the poles and elsewhere,
    # against 40-digit quadrature of its definition
    import mpmath as mp
    mp.mp.dps = 40
    for a, h in [(0.0, 1e-4), (0.0, 6.1e-3), (1.3, 3e-3), (np.pi - 6.1e-3, 6.1e-3), (0.2, 0.29), (0.4, 0.7),
                 (np.pi - 1e-3, 1e-3)]:
        A, H = mp.mpf(a), mp.mpf(h)
        num = mp.quad(lambda u: u * mp.sin(A + u), [0, H])
        den = mp.quad(lambda u: mp.sin(A + u), [0, H])
        want = float(num / den)
        got = float(O.theta_centre_offset(np.array([a]), np.array([h]))[0])
        assert got == pytest.approx(want, rel=2e-15), (a, h)


def test_spherical_thin_shell_volumes_high_precision():
    import mpmath as mp
    mp.mp.dps = 40
    xf = np.array([1e11, 1e11 * (1 + 3.37e-3)])
    yf = np.array([0.0, np.pi / 2048, np.pi / 2])
    m = O.metrics(O.SPHERICAL, xf, yf)
    r0, r1 = mp.mpf(xf[0]), mp.mpf(xf[1])
    for j in range(2):
        t0, t1 = mp.mpf(yf[j]), mp.mpf(yf[j + 1])
        want = float((r1 ** 3 - r0 ** 3) / 3 * (mp.cos(t0) - mp.cos(t1)))
        assert m.dV[j, 0] == pytest.approx(want, rel=1e-15)
