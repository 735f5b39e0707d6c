"""Pins of the chemical-potential tuning oracle (oracle/mutune.py).

With zero fields the force bias vanishes (G stays diagonal), every walker follows the same
deterministic path and <N>(mu) = 2 sum_K 1/(1 + exp(beta (lambda eps_K + h_K - mu))) in closed
form, so the root is known independently (scipy brentq).  Newton with the frozen-path
derivative (here the exact derivative) must reach it to 1e-9; the paper's bracket-and-fit to
the accuracy of a straight-line fit over +-2.5% around a 1% bracket.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import ueg, mutune

KW = dict(n_elec=14, rs=1.0, theta=0.5, nmax2=2, dtau=0.05, stab_every=5)


def _closed_form_root(n_target):
    s = ueg.UEGSystem(**KW)
    lev = s.kscale * s.eps + s.hK

    def n_of(mu):
        return 2.0 * np.sum(1.0 / (1.0 + np.exp(s.beta * (lev - mu)))) - n_target
    return brentq(n_of, lev.min() - 50.0 / s.beta, lev.max() + 50.0 / s.beta, xtol=1e-15), s


def test_zero_field_number_is_fermi_dirac():
    mu_star, s = _closed_form_root(14.0)
    z = [np.zeros((s.n_slices, s.NQ), dtype=np.complex128)] * 2
    for mu in (mu_star - 0.3, mu_star, mu_star + 0.2):
        n, err, dn = mutune.ensemble_number(KW, z, mu, derivative=True)
        lev = s.kscale * s.eps + s.hK
        f = 1.0 / (1.0 + np.exp(s.beta * (lev - mu)))
        assert n == pytest.approx(2.0 * f.sum(), rel=1e-12)
        assert dn == pytest.approx(2.0 * s.beta * np.sum(f * (1.0 - f)), rel=1e-9)
        assert err == pytest.approx(0.0, abs=1e-12)


def test_newton_reaches_the_closed_form_root():
    mu_star, s = _closed_form_root(14.0)
    z = [np.zeros((s.n_slices, s.NQ), dtype=np.complex128)]
    out = mutune.newton(KW, z, 14.0, s.mu_T, tol=1e-12)
    assert out["mu"] == pytest.approx(mu_star, abs=1e-9)
    assert out["runs"] <= 8


def test_bracket_fit_reaches_the_root_to_fit_accuracy():
    mu_star, s = _closed_form_root(14.0)
    z = [np.zeros((s.n_slices, s.NQ), dtype=np.complex128)]
    out = mutune.bracket_fit(KW, z, 14.0, s.mu_T + 0.5)
    scale = max(abs(out["mu_tilde"]), 1.0 / s.beta)
    assert abs(out["mu_tilde"] - mu_star) <= 0.01 * scale     # the 1% bracket
    assert abs(out["mu"] - mu_star) <= 1e-3 * scale           # a line over +-2.5% of a smooth curve
    assert abs(out["mu"] - mu_star) < abs(out["mu_tilde"] - mu_star) + 1e-12
    mus = [t[0] for t in out["trace"][-5:]]
    assert np.allclose(np.diff(mus), 0.0125 * scale)
