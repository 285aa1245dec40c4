"""Pins of the oracle's forward-mode derivative d(lnZ/V)/d(beta) (CPU only)."""

import math

import numpy as np
import pytest

from oracle import exact as E
from oracle import hotrg as H
from oracle import tangent as TG


@pytest.mark.parametrize("kind,d,q,h,beta,chi,steps", [
    ("ising", 2, 2, 0.0, 0.44, 16, 4),
    ("ising", 2, 2, 0.3, 0.5, 16, 4),
    ("ising", 3, 2, 0.0, 0.2216544, 16, 3),
    ("potts", 3, 3, 0.0, 0.55, 9, 1),
    ("potts", 2, 3, 0.0, 0.9, 81, 2),
])
def test_tangent_equals_exact_torus_gradient(kind, d, q, h, beta, chi, steps):
    # untruncated steps: d lnZ/d beta of the torus by exhaustive enumeration
    m = H.Model(kind, d, q, h=h)
    l0, dl0, recs = TG.run_with_tangent(m, beta, chi, steps)
    z0, dz0 = E.torus_log_z(kind, beta, (1,) * d, q=q, h=h)
    assert dl0 == pytest.approx(dz0, abs=1e-13)
    for p, (l, dl) in enumerate(recs, 1):
        L = H.lattice_shape(d, p)
        z, dz = E.torus_log_z(kind, beta, L, q=q, h=h)
        assert l == pytest.approx(z / np.prod(L), abs=1e-13)
        assert dl == pytest.approx(dz / np.prod(L), abs=1e-13)


@pytest.mark.parametrize("d,chi,beta,steps", [(2, 6, 0.42, 10), (3, 4, 0.22, 8)])
def test_tangent_is_the_limit_of_central_differences(d, chi, beta, steps):
    # central differences converge to the tangent as h^2 (ratio 4 when h halves), and
    # Richardson extrapolation agrees with it to O(h^4)
    m = H.Model("ising", d)
    _, _, recs = TG.run_with_tangent(m, beta, chi, steps)

    def fd(hh):
        _, rp = H.run(m, beta + hh, chi, steps)
        _, rm = H.run(m, beta - hh, chi, steps)
        return np.array([(a.lnz_per_site - b.lnz_per_site) / (2 * hh) for a, b in zip(rp, rm)])

    g = np.array([r[1] for r in recs])
    f1, f2 = fd(1e-3), fd(5e-4)
    e1, e2 = g - f1, g - f2
    ratio = e1 / e2
    assert np.all(np.abs(ratio - 4.0) < 0.05), ratio
    rich = (4 * f2 - f1) / 3
    assert np.max(np.abs(rich - g) / np.abs(g)) < 1e-7


def test_tangent_matches_onsager_energy():
    # 2D Ising: -d(lnZ/N)/d beta is Onsager's internal energy (textbook closed form)
    for T, tol in ((2.5, 1e-4), (2.0, 1e-4)):
        b = 1.0 / T
        _, _, recs = TG.run_with_tangent(H.Model("ising", 2), b, 16, 20)
        u = -recs[-1][1]
        assert u == pytest.approx(E.onsager_energy_per_site(b), rel=tol)


def test_onsager_energy_matches_quadrature_derivative():
    # the closed form for u against a central difference of the free-energy quadrature
    b, h = 0.4, 1e-4
    fd = (E.onsager_lnz_per_site(b + h) - E.onsager_lnz_per_site(b - h)) / (2 * h)
    assert -fd == pytest.approx(E.onsager_energy_per_site(b), rel=1e-7)
