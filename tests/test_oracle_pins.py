"""Pins of the FP64 oracle against things other than itself (CPU only).

Each test names what fixes the expected value: a definition evaluated by brute
force, a closed form, a textbook result, or an invariance of the method.
"""

import math

import numpy as np
import pytest

from oracle import exact as E
from oracle import hotrg as H
from tests import layout as LYp
from tests import seeded_inputs as SI


# --------------------------------------------------------------------------
# Section 2: weights, bond factor, initial tensor
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind,q", [("ising", 2), ("potts", 3), ("potts", 4)])
@pytest.mark.parametrize("beta", [0.0, 0.3, 1.1])
def test_bond_factor_reproduces_w(kind, q, beta):
    W, _ = H.boltzmann_weights(kind, beta, q)
    X = H.bond_factor(W)
    np.testing.assert_allclose(X @ X.T, W, rtol=1e-13, atol=1e-13)


def test_antiferromagnet_is_rejected():
    W, _ = H.boltzmann_weights("ising", 0.5, J=-1.0)
    with pytest.raises(ValueError):
        H.bond_factor(W)


@pytest.mark.parametrize("d", [2, 3, 4])
@pytest.mark.parametrize("kind,q", [("ising", 2), ("potts", 3)])
def test_initial_trace_closed_form(d, kind, q):
    # Tr T0 = sum_s V_s W_ss^d: a single site with d self-bonds.  h = 0: q e^{d beta J}
    beta = 0.37
    W, V = H.boltzmann_weights(kind, beta, q)
    T0 = H.initial_tensor(W, V, d)
    assert T0.shape == (q,) * (2 * d)
    assert H.trace(T0) == pytest.approx(q * math.exp(d * beta), rel=1e-14)


def test_initial_tensor_ising_entries():
    # W = U diag(2 cosh b, 2 sinh b) U^T with U = [[1, 1], [1, -1]] / sqrt 2, so the bond
    # channels carry X_{s,cosh} = sqrt(cosh b) and X_{s,sinh} = s sqrt(sinh b).  T0 entries:
    # 2 cosh(b)^{#cosh legs/2} sinh(b)^{#sinh legs/2} when the number of sinh legs is even, else 0.
    beta = 0.41
    W, V = H.boltzmann_weights("ising", beta)
    lam = np.linalg.eigvalsh(W)
    kc = int(np.argmax(lam))          # index of the cosh channel in the oracle's basis
    ks = 1 - kc
    T0 = H.initial_tensor(W, V, 2)
    ch, sh = math.cosh(beta), math.sinh(beta)
    assert T0[kc, kc, kc, kc] == pytest.approx(2 * ch ** 2, rel=1e-14)
    assert T0[ks, ks, ks, ks] == pytest.approx(2 * sh ** 2, rel=1e-14)
    assert T0[kc, ks, ks, ks] == pytest.approx(0.0, abs=1e-14)
    assert abs(T0[ks, ks, kc, kc]) == pytest.approx(2 * ch * sh, rel=1e-14)


# --------------------------------------------------------------------------
# Whole steps while nothing is truncated: exact tori by brute force
# --------------------------------------------------------------------------

def _check_tori(model, beta, chi, steps, tol=1e-13):
    lnz0, recs = H.run(model, beta, chi, steps)
    L0 = (1,) * model.d
    z0, _ = E.torus_log_z(model.kind, beta, L0, q=model.q, J=model.J, h=model.h)
    assert lnz0 == pytest.approx(z0, abs=tol)
    for r in recs:
        L = H.lattice_shape(model.d, r.p)
        z, _ = E.torus_log_z(model.kind, beta, L, q=model.q, J=model.J, h=model.h)
        assert r.lnz_per_site == pytest.approx(z / np.prod(L), abs=tol), (r.p, L)


@pytest.mark.parametrize("beta", [0.2, 0.4406868, 0.7])
def test_2d_ising_tori_up_to_4x4(beta):
    _check_tori(H.Model("ising", 2), beta, chi=16, steps=4)


def test_2d_ising_2x1_closed_form():
    # Z(2x1 torus) = 2 e^{4b} + 2: one double bond along x, two self-bonds along y
    beta = 0.3
    _, recs = H.run(H.Model("ising", 2), beta, chi=4, steps=1)
    assert recs[0].lnz_per_site == pytest.approx(math.log(2 * math.exp(4 * beta) + 2) / 2, rel=1e-15)


@pytest.mark.parametrize("beta", [0.15, 0.2216544, 0.3])
def test_3d_ising_tori_up_to_2x2x2(beta):
    _check_tori(H.Model("ising", 3), beta, chi=16, steps=3)


@pytest.mark.parametrize("beta", [0.1, 0.1497, 0.3])
def test_4d_ising_2x1x1x1_torus(beta):
    # one untruncated 4D step (every leg of dimension <= 4): the 2-site torus, by enumeration
    _check_tori(H.Model("ising", 4), beta, chi=4, steps=1)


def test_4d_ising_2x1x1x1_closed_form():
    # 2x1x1x1 torus: the two sites share two bonds along axis 0 (e^{2b s s'}) and each has a
    # self-bond along each other axis (e^{3b} per site for either spin), so
    # Z = sum_{s,s'} e^{6b} e^{2b s s'} = 2 e^{8b} + 2 e^{4b}.
    beta = 0.2
    _, recs = H.run(H.Model("ising", 4), beta, chi=4, steps=1)
    z = math.log(2 * math.exp(8 * beta) + 2 * math.exp(4 * beta))
    assert recs[0].lnz_per_site == pytest.approx(z / 2, rel=1e-15)


def test_ising_with_field_tori():
    _check_tori(H.Model("ising", 2, h=0.3), 0.5, chi=16, steps=4)
    _check_tori(H.Model("ising", 3, h=-0.2), 0.25, chi=16, steps=2)
    _check_tori(H.Model("ising", 4, h=0.1), 0.2, chi=4, steps=1)


def test_potts_tori():
    _check_tori(H.Model("potts", 2, q=3), 0.9, chi=9, steps=1)
    _check_tori(H.Model("potts", 3, q=3), 0.55, chi=9, steps=1)
    _check_tori(H.Model("potts", 2, q=3), 0.9, chi=81, steps=2)


def test_config3_dims_untruncated_for_three_steps():
    # 3D Ising, chi = 16: dims of (c, n1, n2) before each step, and exactness at 2x2x2
    seen = []
    H.run(H.Model("ising", 3), 0.2216544, 16, 3,
          on_step=lambda r: seen.append(r.dims_before))
    # T[n2, n1, n2', n1', c, c']
    assert [(s[4], s[1], s[0]) for s in seen] == [(2, 2, 2), (4, 4, 2), (16, 4, 4)]


# --------------------------------------------------------------------------
# Algebraic identities of the method on random tensors
# --------------------------------------------------------------------------

def _explicit_m(T):
    """M of Section 2 built literally (tiny dims): two stacked copies joined by rho,
    legs ordered (for d = 3) as T^hat n-legs, T^check n-legs, ... ."""
    d = T.ndim // 2
    if d == 2:
        # M[(n^ n~), (n'^ n'~), c, c'] = sum_rho T[n^, n'^, c, rho] T[n~, n'~, rho, c']
        M = np.einsum("aAcr,bBrC->abABcC", T, T)
        return M
    if d == 3:
        # T[n2, n1, n2', n1', c, c']
        return np.einsum("xyXYcr,uvUVrC->xuyvXUYVcC", T, T)
    # d = 4: T[n3, n2, n1, n3', n2', n1', c, c']
    return np.einsum("xyzXYZcr,uvwUVWrC->xuyvzwXUYVZWcC", T, T)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_gram_three_steps_equals_explicit_mmt(d):
    rng = np.random.default_rng(5)
    dims = {2: (3, 3, 2, 2), 3: (2, 3, 2, 3, 2, 2), 4: (2, 3, 2, 2, 3, 2, 2, 2)}[d]
    T = rng.standard_normal(dims)
    M = _explicit_m(T)
    for j in range(1, d):
        for prime in (False, True):
            ax = H.axis_np(d, j) if prime else H.axis_n(d, j)
            A = H.gram_matrix(T, ax)
            chi = T.shape[ax]
            # position of the (hat, check) pair of the side leg in M
            if d == 2:
                pair = (2, 3) if prime else (0, 1)
            elif d == 3:
                pair = {(2, False): (0, 1), (1, False): (2, 3),
                        (2, True): (4, 5), (1, True): (6, 7)}[(j, prime)]
            else:
                pair = {(3, False): (0, 1), (2, False): (2, 3), (1, False): (4, 5),
                        (3, True): (6, 7), (2, True): (8, 9), (1, True): (10, 11)}[(j, prime)]
            Mm = np.moveaxis(M, pair, (0, 1))            # [hat, check, rest...]
            # merged row index hat + chi*check -> check is the slow index
            Mm = np.swapaxes(Mm, 0, 1).reshape(chi * chi, -1)
            np.testing.assert_allclose(A, Mm @ Mm.T, rtol=1e-12, atol=1e-12)


def _naive_3d_einsum(T, W1, W2):
    # hat copy  T[h2, h1, h2p, h1p, c, r];  check copy T[k2, k1, k2p, k1p, r, C]
    # U2[(h2 k2), n2] = W2[k2, h2, n2], U1[(h1 k1), n1] = W1[k1, h1, n1], same for primes
    return np.einsum(
        "abefcr,ABEFrC,AaN,BbM,EeP,FfQ->NMPQcC",
        T, T, W2, W1, W2, W1, optimize=True)


def _naive_4d_einsum(T, W1, W2, W3):
    # hat copy T[h3, h2, h1, h3p, h2p, h1p, c, r]; check copy T[k3, k2, k1, k3p, k2p, k1p, r, C]
    # U_j[(h + chi k), n] = W_j[k, h, n]
    return np.einsum(
        "abgefhcr,ABGEFHrC,AaN,BbM,GgO,EeP,FfQ,HhS->NMOPQScC",
        T, T, W3, W2, W1, W3, W2, W1, optimize=True)


def _naive_2d_einsum(T, W1):
    # hat T[h1, h1p, c, r]; check T[k1, k1p, r, C]
    return np.einsum("aecr,AErC,AaN,EeP->NPcC", T, T, W1, W1, optimize=True)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_three_stage_order_equals_single_expression(d):
    rng = np.random.default_rng(11)
    if d == 2:
        T = rng.standard_normal((3, 3, 4, 4))
        U1 = SI.random_isometry(9, 5, seed=1)
        W1 = U1.reshape(3, 3, 5)
        ref = _naive_2d_einsum(T, W1)
        got = H.new_tensor(T, {1: U1})
    elif d == 3:
        T = rng.standard_normal((3, 2, 3, 2, 2, 2))  # n2=3, n1=2, c=2
        U1 = SI.random_isometry(4, 3, seed=1)
        U2 = SI.random_isometry(9, 4, seed=2)
        ref = _naive_3d_einsum(T, U1.reshape(2, 2, 3), U2.reshape(3, 3, 4))
        got = H.new_tensor(T, {1: U1, 2: U2})
    else:
        T = rng.standard_normal((2, 3, 2, 2, 3, 2, 2, 2))  # n3=2, n2=3, n1=2, c=2
        U1 = SI.random_isometry(4, 3, seed=1)
        U2 = SI.random_isometry(9, 5, seed=2)
        U3 = SI.random_isometry(4, 2, seed=3)
        ref = _naive_4d_einsum(T, U1.reshape(2, 2, 3), U2.reshape(3, 3, 5), U3.reshape(2, 2, 2))
        got = H.new_tensor(T, {1: U1, 2: U2, 3: U3})
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_rename_cycles_directions():
    # 3D: T^new[n2, n1, n2', n1', c, c'] -> T^next[c, n2, c', n2', n1, n1']
    rng = np.random.default_rng(3)
    T = rng.standard_normal((2, 3, 2, 3, 4, 4))
    R = H.rename(T)
    assert R.shape == (4, 2, 4, 2, 3, 3)
    assert R[1, 0, 2, 1, 2, 0] == T[0, 2, 1, 0, 1, 2]
    T2 = rng.standard_normal((3, 3, 5, 5))
    R2 = H.rename(T2)
    assert R2.shape == (5, 5, 3, 3) and R2[4, 1, 2, 0] == T2[2, 0, 4, 1]


# --------------------------------------------------------------------------
# Truncation rule
# --------------------------------------------------------------------------

def test_choice_rule_and_judgement_values():
    # A with discarded weight 0.1, A' with discarded weight 0.3 -> U is adopted;
    # swapped -> U'; equal -> U' (epsilon >= epsilon').
    Q = SI.random_isometry(4, 4, seed=7)
    A = Q @ np.diag([5.0, 2.0, 0.06, 0.04]) @ Q.T
    Ap = Q @ np.diag([5.0, 1.7, 0.2, 0.1]) @ Q.T
    t = H.choose_isometry(A, Ap, chi=2)
    assert t.eps == pytest.approx(0.1) and t.eps_p == pytest.approx(0.3)
    assert not t.chose_prime
    t2 = H.choose_isometry(Ap, A, chi=2)
    assert t2.chose_prime
    t3 = H.choose_isometry(A, A, chi=2)
    assert t3.chose_prime
    # kept columns span the top-2 eigenvectors of the adopted matrix
    P = t.U @ t.U.T
    np.testing.assert_allclose(P, Q[:, :2] @ Q[:, :2].T, atol=1e-12)
    # no truncation when chi_j^2 <= chi
    t4 = H.choose_isometry(A, Ap, chi=8)
    assert t4.chi_new == 4 and t4.eps == 0.0 and t4.eps_p == 0.0


def test_multiplet_rule():
    # a cut that splits a degenerate pair drops the pair; a clean cut keeps chi_new;
    # eigenvalues at rounding level (here exact zeros) are not examined
    assert H.multiplet_safe_cut(np.array([5.0, 2.0, 1.0, 1.0, 0.1]), 3) == 2
    assert H.multiplet_safe_cut(np.array([5.0, 1.0, 1.0, 1.0, 0.1]), 3) == 1
    assert H.multiplet_safe_cut(np.array([5.0, 2.0, 1.0, 0.5]), 3) == 3
    assert H.multiplet_safe_cut(np.array([1.0, 0.0, 0.0, 0.0]), 2) == 2
    assert H.multiplet_safe_cut(np.array([1.0, 0.5]), 2) == 2
    Q = SI.random_isometry(5, 5, seed=9)
    A = Q @ np.diag([5.0, 2.0, 1.0, 1.0, 0.1]) @ Q.T
    t = H.choose_isometry(A, A, chi=3)
    assert t.kept == 2 and t.U.shape == (5, 3)
    assert np.all(t.U[:, 2] == 0.0)
    # the kept columns span the top-2 eigenvectors exactly
    np.testing.assert_allclose(t.U[:, :2] @ t.U[:, :2].T, Q[:, :2] @ Q[:, :2].T, atol=1e-12)
    # the literal rule keeps chi_new columns
    assert H.choose_isometry(A, A, chi=3, multiplets=False).kept == 3


# --------------------------------------------------------------------------
# Truncated regime
# --------------------------------------------------------------------------

ONSAGER_CASES = [2.0, 2.269185, 2.5]


@pytest.mark.parametrize("T", ONSAGER_CASES)
def test_onsager_two_quadratures_agree(T):
    b = 1.0 / T
    assert E.onsager_lnz_per_site(b) == pytest.approx(E.onsager_lnz_per_site_double(b), abs=1e-11)


def test_onsager_at_critical_point_closed_form():
    # at exact T_c: lnZ/N = 2G/pi + (1/2) ln 2, G = Catalan's constant
    bc = 0.5 * math.log(1 + math.sqrt(2))
    G = 0.915965594177219015054603514932
    assert E.onsager_lnz_per_site(bc) == pytest.approx(2 * G / math.pi + 0.5 * math.log(2), abs=1e-12)


@pytest.mark.parametrize("T", ONSAGER_CASES)
def test_2d_ising_hotrg_converges_to_onsager(T):
    b = 1.0 / T
    exact = E.onsager_lnz_per_site(b)
    errs = {}
    for chi in (4, 8, 16):
        _, recs = H.run(H.Model("ising", 2), b, chi, 20)
        errs[chi] = abs(recs[-1].lnz_per_site - exact) / exact
    assert errs[8] < 1e-3
    assert errs[16] < errs[4]
    assert errs[16] < 2e-5


@pytest.mark.parametrize("d", [2, 3, 4])
def test_infinite_temperature_is_exact(d):
    # beta = 0: W has rank 1, Z = q^N exactly for any chi and any lattice
    _, recs = H.run(H.Model("ising", d), 0.0, 4, 8)
    for r in recs:
        assert r.lnz_per_site == pytest.approx(math.log(2), abs=1e-14)


def test_low_temperature_limit():
    # beta large: Z ~ q e^{d beta N}, lnZ/V -> d beta + ln(q)/V
    beta = 3.0
    _, recs = H.run(H.Model("ising", 3), beta, 4, 12)
    assert recs[-1].lnz_per_site == pytest.approx(3 * beta + math.log(2) / 2 ** 12, abs=1e-9)


def test_high_temperature_series_2d():
    # 2D Ising: lnZ/N = ln 2 + 2 ln cosh b + tanh^4 b + O(tanh^6 b)
    b = 0.08
    _, recs = H.run(H.Model("ising", 2), b, 8, 20)
    series = math.log(2) + 2 * math.log(math.cosh(b)) + math.tanh(b) ** 4
    assert recs[-1].lnz_per_site == pytest.approx(series, abs=5 * math.tanh(b) ** 6)


def _gauge_transform(T0, Os):
    """Insert O O^T on every bond: the same O acts on both legs of a direction."""
    d = T0.ndim // 2
    T = T0
    for mu in range(d):
        # direction 0 is Current (c, c'), direction j >= 1 is Next j (n_j, n'_j)
        legs = [H.axis_c(d), H.axis_cp(d)] if mu == 0 else [H.axis_n(d, mu), H.axis_np(d, mu)]
        for ax in legs:
            T = np.moveaxis(np.tensordot(T, Os[mu], axes=([ax], [0])), -1, ax)
    return T


@pytest.mark.parametrize("d,chi,steps", [(2, 6, 12), (3, 4, 9)])
def test_bond_gauge_invariance(d, chi, steps):
    beta = {2: 0.42, 3: 0.22}[d]
    W, V = H.boltzmann_weights("ising", beta)
    T0 = H.initial_tensor(W, V, d)
    _, ref = H.run(H.Model("ising", d), beta, chi, steps, T0=T0)
    for seed in (10, 11):
        Os = [SI.random_isometry(2, 2, seed=seed + 100 * mu) for mu in range(d)]
        _, got = H.run(H.Model("ising", d), beta, chi, steps, T0=_gauge_transform(T0, Os))
        for a, b in zip(ref, got):
            assert b.lnz_per_site == pytest.approx(a.lnz_per_site, rel=1e-12)


@pytest.mark.parametrize("d,chi", [(2, 6), (3, 4)])
def test_normalisation_choice_invariance(d, chi):
    beta = {2: 0.45, 3: 0.23}[d]
    _, a = H.run(H.Model("ising", d), beta, chi, 10, norm="trace")
    _, b = H.run(H.Model("ising", d), beta, chi, 10, norm="maxabs")
    for x, y in zip(a, b):
        assert y.lnz_per_site == pytest.approx(x.lnz_per_site, rel=1e-12)


def test_gu_wen_ratio_limits():
    # ordered phase (2 degenerate states) -> 2, disordered -> 1
    _, lo = H.run(H.Model("ising", 2), 1 / 1.5, 8, 24)
    _, hi = H.run(H.Model("ising", 2), 1 / 4.0, 8, 24)
    assert lo[-1].gu_wen == pytest.approx(2.0, abs=1e-3)
    assert hi[-1].gu_wen == pytest.approx(1.0, abs=1e-3)


# --------------------------------------------------------------------------
# Section 4.2.6: alternative choice criteria (any rational criterion is allowed)
# --------------------------------------------------------------------------

def test_choice_criteria_agree_for_a_reflection_symmetric_model():
    """Ising: A and A' agree up to a bond gauge (R3), so adopting U, U' or the epsilon winner gives
    the same gauge-invariant lnZ/V."""
    m = H.Model("ising", 3)
    runs = {c: [r.lnz_per_site for r in H.run(m, 1 / 4.5115, 6, 8, choice=c)[1]] for c in H.CHOICES}
    for c in ("U", "Uprime"):
        np.testing.assert_allclose(runs[c], runs["epsilon"], rtol=1e-12)


def test_choice_criteria_on_a_tensor_without_reflection_symmetry():
    """A random positive tensor: U and U' differ; the epsilon criterion adopts, at every step, the
    side with the smaller judgement value, so its first step equals the fixed choice of that side
    bitwise."""
    T0 = LYp.to_paper(SI.random_positive_tensor((3, 4, 2) * 2, seed=24))
    T = T0 / H.trace(T0)
    a, tr_a = H.coarse_grain(T, 6, choice="epsilon")
    side = "Uprime" if tr_a[1].chose_prime else "U"
    b, _ = H.coarse_grain(T, 6, choice=side)
    np.testing.assert_array_equal(a, b)
    assert tr_a[1].chose_prime == (not tr_a[1].eps < tr_a[1].eps_p)
    lu = [r.lnz_per_site for r in H.run(H.Model("ising", 3), 0.0, 6, 6, T0=T0, choice="U")[1]]
    lp = [r.lnz_per_site for r in H.run(H.Model("ising", 3), 0.0, 6, 6, T0=T0, choice="Uprime")[1]]
    assert max(abs(x - y) / abs(y) for x, y in zip(lu, lp)) > 1e-8
    with pytest.raises(ValueError):
        H.choose_isometry(np.eye(4), np.eye(4), 2, choice="best")
