"""Pins for the oracle's flux limiters (Section 2: FLD closure and limiter).

The Levermore-Pomraning form is checked against a 50-digit evaluation of its
definition with mpmath; the asymptotic limits of Section 2 (thick: lambda ->
1/3, thin: lambda R -> 1) are checked for every limiter; the Minerbo form is
checked for continuity at R = 3/2 where both branches give 2/9.
"""
import mpmath
import numpy as np
import pytest

from oracle import fld_oracle as O

mpmath.mp.dps = 50


def lp_exact(R):
    R = mpmath.mpf(R)
    return float((mpmath.coth(R) - 1 / R) / R)


def test_lp_matches_high_precision_definition():
    Rs = np.concatenate([np.logspace(-9, 6, 301), [0.0999999, 0.1, 0.1000001, 1.0, 3.0]])
    got = O.limiter_lp(Rs)
    want = np.array([lp_exact(r) for r in Rs])
    rel = np.abs(got / want - 1.0)
    assert rel.max() < 1e-13, (Rs[rel.argmax()], rel.max())


@pytest.mark.parametrize("lim", [O.limiter_lp, O.limiter_minerbo])
def test_asymptotic_limits(lim):
    assert lim(np.array([0.0]))[0] == pytest.approx(1.0 / 3.0, rel=1e-15)
    big = np.array([1e6, 1e8, 1e10])
    lr = lim(big) * big
    assert np.all(np.abs(lr - 1.0) < 3.0 / np.sqrt(big))  # lambda R -> 1 (free streaming)
    Rs = np.logspace(-6, 8, 2000)
    lam = lim(Rs)
    assert np.all(np.diff(lam) <= 1e-17)  # monotone non-increasing
    assert np.all((lam > 0) & (lam <= 1.0 / 3.0 + 1e-16))


def test_minerbo_continuous_at_three_halves():
    lo = 2.0 / (3.0 + np.sqrt(9.0 + 12.0 * 1.5 ** 2))
    hi = 1.0 / (1.0 + 1.5 + np.sqrt(1.0 + 2.0 * 1.5))
    assert lo == pytest.approx(2.0 / 9.0, rel=1e-15)
    assert hi == pytest.approx(2.0 / 9.0, rel=1e-15)
    eps = 1e-9
    v = O.limiter_minerbo(np.array([1.5 - eps, 1.5, 1.5 + eps]))
    assert np.all(np.abs(v - 2.0 / 9.0) < 1e-8)


def test_thick_limit_diffusion_coefficient():
    # tiny gradient: D -> c / (3 sigma), the optically thick limit of Section 2
    sig = np.array([1e7, 1e-3, 2.5])
    E = np.array([1.0, 3.0, 7.0])
    D = O.face_D(sig, sig, np.full(3, 0.5), np.full(3, 0.5), E, E * (1 + 1e-12), O.limiter_lp)
    np.testing.assert_allclose(D, O.C_LIGHT / (3.0 * sig), rtol=1e-12)


def test_thin_limit_face_flux_is_cE():
    # sigma -> 0: |D dE/h| -> c E_f with E_f the face-interpolated E (free streaming)
    rng = np.random.default_rng(0)
    EL, ER = rng.uniform(1, 2, 50), rng.uniform(3, 4, 50)
    hL, hR = rng.uniform(0.2, 1, 50), rng.uniform(0.2, 1, 50)
    sig = np.full(50, 1e-12)
    D = O.face_D(sig, sig, hL, hR, EL, ER, O.limiter_lp)
    flux = D * np.abs(ER - EL) / (hL + hR)
    Ef = (hR * EL + hL * ER) / (hL + hR)
    R = np.abs(ER - EL) / ((hL + hR) * sig * Ef)
    assert np.all(np.abs(flux / (O.C_LIGHT * Ef) - 1.0) < 2.0 / R)
