"""Exact results that pin the oracle (TEST INFRASTRUCTURE ONLY).

* Exhaustive partition functions of tiny periodic tori, straight from the
  definition of Z in Section 2 (eq. 2):  Z = sum_sigma prod_<ij> W(s_i, s_j) prod_i V(s_i),
  with one bond from every site to its +e_mu neighbour (mod L_mu).  L_mu = 1 gives a
  self-bond, L_mu = 2 a double bond: exactly what the trace of an untruncated
  coarse-grained tensor contracts.
* Onsager's free energy of the 2D square-lattice Ising model (J = 1, h = 0), a
  textbook closed form that is not in the paper; evaluated by quadrature in two
  independent forms.
"""

from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, special


def _site_index(coord, L):
    idx = 0
    for x, l in zip(coord, L):
        idx = idx * l + x
    return idx


def torus_bonds(L):
    """List of (i, j, mu) bonds of a periodic torus of shape L."""
    bonds = []
    for coord in itertools.product(*[range(l) for l in L]):
        i = _site_index(coord, L)
        for mu in range(len(L)):
            nb = list(coord)
            nb[mu] = (nb[mu] + 1) % L[mu]
            bonds.append((i, _site_index(nb, L), mu))
    return bonds


def _spin_values(model: str, q: int):
    if model == "ising":
        return np.array([1.0, -1.0])
    return np.arange(q, dtype=float)


def torus_log_z(model: str, beta: float, L, q: int = 2, J: float = 1.0, h: float = 0.0):
    """ln Z of the periodic torus L by enumerating all q^N configurations.

    Returns (lnZ, dlnZ/dbeta).  Ising: f = beta J s s', g = beta h s.  Potts: f = beta J delta.
    """
    if model == "ising":
        q = 2
    N = int(np.prod(L))
    if q ** N > 2 ** 22:
        raise ValueError("torus too large for enumeration")
    bonds = torus_bonds(L)
    s = _spin_values(model, q)
    states = np.array(list(itertools.product(range(q), repeat=N)), dtype=np.int64)
    # S = d(-H/kT)/d(beta) for each configuration
    S = np.zeros(states.shape[0])
    for (i, j, _mu) in bonds:
        if model == "ising":
            S += J * s[states[:, i]] * s[states[:, j]]
        else:
            S += J * (states[:, i] == states[:, j])
    if model == "ising" and h != 0.0:
        S += h * s[states].sum(axis=1)
    logw = beta * S
    m = logw.max()
    w = np.exp(logw - m)
    Z = w.sum()
    lnZ = m + math.log(Z)
    dlnZ = float((w * S).sum() / Z)
    return lnZ, dlnZ


def onsager_lnz_per_site(beta: float) -> float:
    """Onsager: lnZ/N = ln(2 cosh 2b) + (1/pi) int_0^{pi/2} ln[(1 + sqrt(1 - k^2 sin^2 t)) / 2] dt,
    k = 2 sinh 2b / cosh^2 2b."""
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2

    def integrand(t):
        return math.log((1.0 + math.sqrt(max(0.0, 1.0 - k * k * math.sin(t) ** 2))) / 2.0)

    val, _ = integrate.quad(integrand, 0.0, math.pi / 2, epsabs=1e-14, epsrel=1e-14, limit=500)
    return math.log(2.0 * math.cosh(2 * beta)) + val / math.pi


def onsager_lnz_per_site_double(beta: float) -> float:
    """Second form: lnZ/N = ln 2 + 1/(2 pi^2) int_0^pi int_0^pi ln[cosh^2 2b - sinh 2b (cos t1 + cos t2)]."""
    c2 = math.cosh(2 * beta) ** 2
    s2 = math.sinh(2 * beta)

    def inner(t2):
        f = lambda t1: math.log(c2 - s2 * (math.cos(t1) + math.cos(t2)))
        return integrate.quad(f, 0.0, math.pi, epsabs=1e-13, epsrel=1e-13, limit=400)[0]

    val, _ = integrate.quad(inner, 0.0, math.pi, epsabs=1e-12, epsrel=1e-12, limit=400)
    return math.log(2.0) + val / (2.0 * math.pi ** 2)


def onsager_energy_per_site(beta: float) -> float:
    """Internal energy per site u = -d(lnZ/N)/dbeta for the 2D Ising model (J = 1):
    u = -coth(2b) [1 + (2/pi) (2 tanh^2(2b) - 1) K(k)],  k = 2 sinh 2b / cosh^2 2b."""
    k = 2.0 * math.sinh(2 * beta) / math.cosh(2 * beta) ** 2
    K = special.ellipk(k * k)          # scipy uses the parameter m = k^2
    t = math.tanh(2 * beta)
    return -(1.0 / t) * (1.0 + (2.0 / math.pi) * (2.0 * t * t - 1.0) * K)
