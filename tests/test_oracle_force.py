"""Pins of the oracle's link derivative (force) of the multi-shift pseudofermion action
S = sum_i r_i phi^+ (sigma_i - D_eo D_oe)^-1 phi: central finite differences of S itself,
computed by independent CG solves on perturbed links, along random directions in the space of
fat links and of Naik links; and its symmetry under the exchange of the two parities' roles."""
import numpy as np
import pytest

import oracle
from ksinputs import make_gauge, gaussian_source, GaugeField


@pytest.fixture(scope="module")
def setup():
    g = make_gauge((4, 4, 4, 6), 0.5, 71)
    phi = gaussian_source(g.volume // 2, 72)
    sigmas = np.array([0.05, 0.2, 0.9])
    residues = np.array([0.3, 0.7, 1.9])
    xs, _, _, _ = oracle.multishift_cg(g, sigmas, phi, 1e-13)
    fv, fw = oracle.force_outer(g, residues, xs)
    return g, phi, sigmas, residues, fv, fw


def directional(f, d):
    """2 Re sum Tr[d F] over directions and sites."""
    return 2.0 * float(np.einsum("mxab,mxba->", d, f).real)


@pytest.mark.parametrize("which", ["fat", "naik"])
def test_force_matches_finite_differences(setup, which):
    g, phi, sigmas, residues, fv, fw = setup
    rng = np.random.default_rng(73 if which == "fat" else 74)
    d = rng.standard_normal(g.fat.shape) + 1j * rng.standard_normal(g.fat.shape)
    eps = 1e-5

    def action(sign):
        fat = g.fat + sign * eps * d if which == "fat" else g.fat
        naik = g.naik + sign * eps * d if which == "naik" else g.naik
        return oracle.rational_action(GaugeField(g.dims, fat, naik), residues, sigmas, phi)

    fd = (action(+1) - action(-1)) / (2 * eps)
    an = directional(d, fv if which == "fat" else fw)
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_force_of_one_shift_scales_with_its_residue(setup):
    g, phi, sigmas, residues, _, _ = setup
    x, _ = oracle.cg(g, sigmas[0], phi, 1e-13)
    f1v, f1w = oracle.force_outer(g, [1.0], [x])
    f2v, f2w = oracle.force_outer(g, [2.5], [x])
    assert np.allclose(f2v, 2.5 * f1v, rtol=1e-14, atol=0) and np.allclose(f2w, 2.5 * f1w,
                                                                            rtol=1e-14, atol=0)


def test_force_free_field_direction(setup):
    """Along the direction d = i V (a unitary rotation of each link's phase, to first order)
    the action's derivative is 2 Re Tr[i V F]: checked against the finite difference of the
    action under V -> exp(i t) V, a different perturbation path with the same tangent."""
    g, phi, sigmas, residues, fv, _ = setup
    t = 1e-5
    sp = oracle.rational_action(GaugeField(g.dims, np.exp(1j * t) * g.fat, g.naik), residues,
                                sigmas, phi)
    sm = oracle.rational_action(GaugeField(g.dims, np.exp(-1j * t) * g.fat, g.naik), residues,
                                sigmas, phi)
    an = directional(1j * g.fat, fv)
    assert abs((sp - sm) / (2 * t) - an) <= 1e-6 * max(abs(an), 1e-8 * np.abs(fv).sum())
