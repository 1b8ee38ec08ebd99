"""Pins of the transport oracle (oracle/transport.py): pure-species and
identical-species limits, binary closed forms written out by hand, and the
zero-degree homogeneity of the mixture rules in the mass fractions."""

import numpy as np
import pytest

import mechs
from oracle import transport as tr
from pyro_synth.transport import draw_transport


def _mech(tmp_path, W):
    S = len(W)
    return mechs.make(str(tmp_path / "t.pyromech"), W=W, nasa_low=mechs.constant_cp(S, 3.5, 0, 20),
                      reactions=[dict(reac=[(0, 1)], prod=[(1, 1)], arrh=(0.0, 0.0, 0.0))])


def test_fits_evaluate_the_printed_polynomials():
    """mu = sqrt(T) p^2, kappa = sqrt(T) q, D = sqrt(T) r with p, q, r the
    quartics in ln T, written out term by term for one species and pair."""
    v, c, d = draw_transport(4, seed=11)
    T = np.array([350.0, 1000.0, 2800.0])
    L = np.log(T)
    p = v[2, 0] + v[2, 1] * L + v[2, 2] * L**2 + v[2, 3] * L**3 + v[2, 4] * L**4
    np.testing.assert_allclose(tr.species_viscosities(v, T)[2], np.sqrt(T) * p * p, rtol=1e-13)
    q = c[1, 0] + c[1, 1] * L + c[1, 2] * L**2 + c[1, 3] * L**3 + c[1, 4] * L**4
    np.testing.assert_allclose(tr.species_conductivities(c, T)[1], np.sqrt(T) * q, rtol=1e-13)
    r = d[0, 3, 0] + d[0, 3, 1] * L + d[0, 3, 2] * L**2 + d[0, 3, 3] * L**3 + d[0, 3, 4] * L**4
    np.testing.assert_allclose(tr.binary_diffusivities(d, T)[0, 3], np.sqrt(T) * r, rtol=1e-13)


def test_pure_species_limits(tmp_path):
    """X = e_k: Phi_kk = (1 + 1)^2/sqrt(16) = 1, so mu = mu_k; kappa =
    (kappa_k + kappa_k)/2."""
    m = _mech(tmp_path, [0.002, 0.016, 0.028, 0.032])
    v, c, d = draw_transport(4, seed=3)
    T = np.array([600.0, 1500.0])
    for k in range(4):
        Y = np.zeros((4, 2))
        Y[k] = 1.0
        np.testing.assert_allclose(tr.mixture_viscosity(m, v, T, Y),
                                   tr.species_viscosities(v, T)[k], rtol=1e-14)
        np.testing.assert_allclose(tr.mixture_conductivity(m, c, T, Y),
                                   tr.species_conductivities(c, T)[k], rtol=1e-14)


def test_identical_species_behave_as_one(tmp_path):
    """Two species with the same molar mass and fits: every Phi is 1 and the
    mixture has the common properties."""
    m = _mech(tmp_path, [0.028, 0.028])
    v, c, d = draw_transport(2, seed=5)
    v[1] = v[0]
    c[1] = c[0]
    T = np.array([800.0, 2200.0])
    Y = np.array([[0.3, 0.8], [0.7, 0.2]])
    np.testing.assert_allclose(tr.mixture_viscosity(m, v, T, Y),
                               tr.species_viscosities(v, T)[0], rtol=1e-14)
    np.testing.assert_allclose(tr.mixture_conductivity(m, c, T, Y),
                               tr.species_conductivities(c, T)[0], rtol=1e-14)


def test_binary_closed_forms(tmp_path):
    """Binary mixture: mu = X1 mu1/(X1 + X2 Phi12) + X2 mu2/(X1 Phi21 + X2),
    kappa = (X1 k1 + X2 k2 + 1/(X1/k1 + X2/k2))/2, D_1m = (1 - Y1) D12/X2."""
    W = np.array([0.004, 0.032])
    m = _mech(tmp_path, list(W))
    v, c, d = draw_transport(2, seed=9)
    T = np.array([500.0, 1900.0])
    Y = np.array([[0.25, 0.6], [0.75, 0.4]])
    X = (Y / W[:, None]) / (Y / W[:, None]).sum(axis=0)
    mu = tr.species_viscosities(v, T)
    k = tr.species_conductivities(c, T)
    D = tr.binary_diffusivities(d, T)
    p12 = (1 + (mu[0] / mu[1]) ** 0.5 * (W[1] / W[0]) ** 0.25) ** 2 / (8 * (1 + W[0] / W[1])) ** 0.5
    p21 = (1 + (mu[1] / mu[0]) ** 0.5 * (W[0] / W[1]) ** 0.25) ** 2 / (8 * (1 + W[1] / W[0])) ** 0.5
    np.testing.assert_allclose(tr.mixture_viscosity(m, v, T, Y),
                               X[0] * mu[0] / (X[0] + X[1] * p12) + X[1] * mu[1] / (X[0] * p21 + X[1]),
                               rtol=1e-13)
    np.testing.assert_allclose(tr.mixture_conductivity(m, c, T, Y),
                               0.5 * (X[0] * k[0] + X[1] * k[1] + 1 / (X[0] / k[0] + X[1] / k[1])),
                               rtol=1e-13)
    Dm = tr.mixture_diffusivities(m, d, T, Y)
    np.testing.assert_allclose(Dm[0], (1 - Y[0]) * D[0, 1] / X[1], rtol=1e-13)
    np.testing.assert_allclose(Dm[1], (1 - Y[1]) * D[1, 0] / X[0], rtol=1e-13)
    # Wilke's coefficients satisfy Phi21 = Phi12 (mu2/mu1)(W1/W2)
    np.testing.assert_allclose(p21, p12 * (mu[1] / mu[0]) * (W[0] / W[1]), rtol=1e-13)


def test_mixture_rules_ignore_the_scale_of_Y(mech0):
    v, c, d = draw_transport(mech0.S)
    rng = np.random.default_rng(4)
    Y = rng.dirichlet(np.ones(mech0.S), 5).T
    T = rng.uniform(400, 2500, 5)
    for f, coef in ((tr.mixture_viscosity, v), (tr.mixture_conductivity, c)):
        np.testing.assert_allclose(f(mech0, coef, T, 3.0 * Y), f(mech0, coef, T, Y), rtol=1e-13)
