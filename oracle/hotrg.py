"""FP64 HOTRG oracle: one coarse-graining step at a time, in the paper's order.

TEST INFRASTRUCTURE ONLY -- never imported by the product path.

This is a plain, slow, obviously-correct NumPy implementation of the Higher Order
Tensor Renormalization Group as described by Yamashita & Sakurai, "A Parallel
Computing Method for the Higher Order Tensor Renormalization Group" (arXiv
2110.03607).  The distribution over chi^2 processes is removed: every "process"
index is simply a free index here.  Library primitives used as single steps:
``numpy.einsum`` (contractions), ``numpy.linalg.eigh`` (symmetric eigensolver).

Index convention (Section 3.1.3): a local tensor of a d-dimensional lattice is
    T[n_{d-1}, ..., n_1, n'_{d-1}, ..., n'_1, c, c']
where (c, c') are the legs in the Current direction and (n_j, n'_j) those of the
direction Next j.  Merged indices follow Section 3.2: (a b) = a + b * chi_{n_j},
with a on the hat copy and b on the check copy.

Readings of points the paper leaves open:
  R1  Section 3.2 / 4.2.5 speak of an SVD of A and A'.  A = M M^T is symmetric
      positive semi-definite, so a symmetric eigendecomposition is used; the
      "singular values" are its eigenvalues, sorted in descending order.
  R2  The judgement values epsilon, epsilon' (Section 2) are sums of the
      discarded eigenvalues of A (not of their square roots); eigenvalues that
      are negative only through rounding count as zero.
  R3  Choice rule (Section 2): epsilon < epsilon' -> U, otherwise U'.
  R4  Normalisation (Section 3.1.3): f^(p) = 1 / Tr T at every step, p = 0 included.
  R5  Columns are never sign-flipped (Section 4.2.7 allows it, it is a gauge).
  R6  The Current direction starts at lattice axis 0 (x) and cycles x, y, z, ...
      through the renaming of Section 3.1.3.
  R7  After p steps the result is lnZ/V for a periodic torus of 2^p sites.
  R8  "The first chi columns" is not unique when the cut splits a multiplet of
      (numerically) equal eigenvalues.  Then the whole multiplet is dropped: its
      columns of the adopted isometry are set to zero, which is the same as keeping
      fewer columns.  Two eigenvalues belong to one multiplet when they differ by at
      most MULTIPLET_RTOL times the larger one; eigenvalues below MULTIPLET_ATOL
      times the largest are never examined (their weight is at rounding level).
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

# ----------------------------------------------------------------------------
# Section 2, eqs. (1)-(4): model, Boltzmann weights, initial tensor
# ----------------------------------------------------------------------------


def boltzmann_weights(model: str, beta: float, q: int = 2, J: float = 1.0, h: float = 0.0):
    """W[s, s'] = exp(f(s, s')) and V[s] = exp(g(s)) with -H/kT = sum f + sum g (eqs. 1-2).

    ising:  s = +-1 (state 0 -> +1, state 1 -> -1), f = beta J s s', g = beta h s.
    potts:  q states, f = beta J delta(s, s'), g = 0 (h must be 0).
    """
    if model == "ising":
        spins = np.array([1.0, -1.0])
        W = np.exp(beta * J * np.outer(spins, spins))
        V = np.exp(beta * h * spins)
    elif model == "potts":
        if h != 0.0:
            raise ValueError("potts oracle supports h = 0 only")
        W = np.exp(beta * J * np.eye(q))
        V = np.ones(q)
    else:
        raise ValueError(model)
    return W, V


def bond_factor(W: np.ndarray) -> np.ndarray:
    """X = U sqrt(Lambda) from the eigendecomposition W = U Lambda U^T (Section 2).

    W is real symmetric; a negative eigenvalue means no real X exists, which is an
    error (the conjugate in eq. (4) would then not reproduce W).
    """
    lam, U = np.linalg.eigh(W)
    if np.min(lam) < -1e-12 * np.max(np.abs(lam)):
        raise ValueError("W is not positive semi-definite")
    lam = np.clip(lam, 0.0, None)
    return U * np.sqrt(lam)[None, :]


def initial_tensor(W: np.ndarray, V: np.ndarray, d: int) -> np.ndarray:
    """eq. (4): T_{j1 j1' ... jd jd'} = sum_s X_{s j1} ... X_{s jd} X_{s j1'} ... X_{s jd'} V_s.

    Returned in the order of Section 3.1.3, T[n_{d-1}..n_1, n'_{d-1}..n'_1, c, c'].
    Because every leg carries the same factor X_{s .}, the tensor is symmetric in
    all of its legs and the assignment of lattice directions to legs only fixes
    which direction is Current (R6).
    """
    X = bond_factor(W)
    q = X.shape[0]
    T = np.zeros((q,) * (2 * d))
    for s in range(q):
        vec = X[s, :]
        term = V[s]
        for _ in range(2 * d):
            term = np.multiply.outer(term, vec)
        T += term
    return T


# ----------------------------------------------------------------------------
# Leg bookkeeping for T[n_{d-1}..n_1, n'_{d-1}..n'_1, c, c']
# ----------------------------------------------------------------------------


def axis_n(d: int, j: int) -> int:
    """Axis of leg n_j (j = 1..d-1)."""
    return d - 1 - j


def axis_np(d: int, j: int) -> int:
    """Axis of leg n'_j (j = 1..d-1)."""
    return 2 * d - 2 - j


def axis_c(d: int) -> int:
    return 2 * d - 2


def axis_cp(d: int) -> int:
    return 2 * d - 1


def _letters(k: int) -> list[str]:
    return [chr(ord("a") + i) for i in range(k)]


# ----------------------------------------------------------------------------
# eq. (Trace_LocalTensor) and the Gu-Wen matrix Y (eq. Matrix_Y)
# ----------------------------------------------------------------------------


def trace(T: np.ndarray) -> float:
    """Tr T = sum over n~_{d-1}..n~_1, c~ of T[n~.., n~.., c~, c~] (eq. Trace_LocalTensor)."""
    d = T.ndim // 2
    L = _letters(d)
    # non-primed legs and primed legs share letters; c and c' share a letter
    spec = "".join(L[: d - 1]) + "".join(L[: d - 1]) + L[d - 1] + L[d - 1]
    return float(np.einsum(spec + "->", T))


def gu_wen_ratio(T: np.ndarray) -> float:
    """X = (trace Y)^2 / trace(Y^2) with Y[c, c'] = sum_n T[n.., n.., c, c'] (eqs. ratio_X, Matrix_Y)."""
    d = T.ndim // 2
    L = _letters(d - 1)
    spec = "".join(L) + "".join(L) + "XY->XY"
    Y = np.einsum(spec, T)
    return float(np.trace(Y) ** 2 / np.trace(Y @ Y))


# ----------------------------------------------------------------------------
# Section 3.2 / 4.2.4: the matrices A^(j), A'^(j) in three steps
# ----------------------------------------------------------------------------


def s_hat(T: np.ndarray, side_axis: int, T2: np.ndarray | None = None) -> np.ndarray:
    """S^hat[f, g, rho, eta] = sum T[.. f .., c, rho] T[.. g .., c, eta] (eq. Aux_Tensor_hat_S).

    The sum runs over every leg except the side leg (n_j or n'_j) and c'; c is
    summed.  rho and eta are the c' legs of the two copies.  T2 (default T) is the
    second factor, for the bilinear form used by the derivative.
    """
    T2 = T if T2 is None else T2
    d = T.ndim // 2
    L = _letters(2 * d)
    a = list(L)
    b = list(L)
    a[side_axis], b[side_axis] = "F", "G"
    a[axis_cp(d)], b[axis_cp(d)] = "R", "E"
    return np.einsum("".join(a) + "," + "".join(b) + "->FGRE", T, T2, optimize=True)


def s_check(T: np.ndarray, side_axis: int, T2: np.ndarray | None = None) -> np.ndarray:
    """S^check[f, g, rho, eta] = sum T[.. f .., rho, c'] T[.. g .., eta, c'] (eq. Aux_Tensor_check_S).

    The sum runs over every leg except the side leg and c; c' is summed.
    """
    T2 = T if T2 is None else T2
    d = T.ndim // 2
    L = _letters(2 * d)
    a = list(L)
    b = list(L)
    a[side_axis], b[side_axis] = "F", "G"
    a[axis_c(d)], b[axis_c(d)] = "R", "E"
    return np.einsum("".join(a) + "," + "".join(b) + "->FGRE", T, T2, optimize=True)


def combine_gram(Sh: np.ndarray, Sc: np.ndarray) -> np.ndarray:
    """A[(f^ f~), (g^ g~)] = sum_{rho, eta} Sh[f^ g^ rho eta] Sc[f~ g~ rho eta] (third step)."""
    chi = Sh.shape[0]
    return np.einsum("PQRE,pqRE->pPqQ", Sh, Sc).reshape(chi * chi, chi * chi)


def gram_matrix(T: np.ndarray, side_axis: int) -> np.ndarray:
    """A[(f^ f~), (g^ g~)] = sum_{rho, eta} S^hat[f^ g^ rho eta] S^check[f~ g~ rho eta].

    Merged index (f^ f~) = f^ + f~ * chi_{n_j} (Section 3.2), so f~ is the slow
    index of the row.  For side_axis = axis of n_j this is A^(j); for the axis of
    n'_j it is A'^(j).
    """
    chi = T.shape[side_axis]
    Sh = s_hat(T, side_axis)
    Sc = s_check(T, side_axis)
    # A4[f~, f^, g~, g^]
    A4 = np.einsum("PQRE,pqRE->pPqQ", Sh, Sc)
    return A4.reshape(chi * chi, chi * chi)


# ----------------------------------------------------------------------------
# Sections 2 and 4.2.5-4.2.7: decomposition, judgement values, choice, truncation
# ----------------------------------------------------------------------------


def eig_descending(A: np.ndarray):
    """Symmetric eigendecomposition with eigenvalues in descending order (R1)."""
    lam, U = np.linalg.eigh(A)
    order = np.arange(lam.size)[::-1]
    return lam[order], U[:, order]


MULTIPLET_RTOL = 1e-10
MULTIPLET_ATOL = 1e-12


def multiplet_safe_cut(lam_desc: np.ndarray, chi_new: int) -> int:
    """Number of leading columns kept so that the cut splits no multiplet (R8)."""
    k = chi_new
    if k >= lam_desc.size:
        return k
    while (k > 1 and lam_desc[k - 1] >= MULTIPLET_ATOL * lam_desc[0]
           and lam_desc[k - 1] - lam_desc[k] <= MULTIPLET_RTOL * lam_desc[k - 1]):
        k -= 1
    return k


def judgement_value(lam_desc: np.ndarray, chi_new: int) -> float:
    """epsilon = sum of the eigenvalues beyond the first chi_new (Section 2, R2)."""
    return float(np.sum(np.clip(lam_desc[chi_new:], 0.0, None)))


@dataclass
class Truncation:
    U: np.ndarray                 # chosen isometry, chi_j^2 x chi_new
    eps: float                    # epsilon   (non-prime side)
    eps_p: float                  # epsilon'  (prime side)
    chose_prime: bool             # True when U' was adopted
    lam: np.ndarray               # eigenvalues of A  (descending)
    lam_p: np.ndarray             # eigenvalues of A' (descending)
    chi_new: int
    kept: int                     # columns not zeroed by the multiplet rule (R8)


CHOICES = ("epsilon", "U", "Uprime")


def choose_isometry(A: np.ndarray, Ap: np.ndarray, chi: int, multiplets: bool = True,
                    choice: str = "epsilon") -> Truncation:
    """Decompose A and A', compare epsilon and epsilon', keep the first chi_new columns.

    chi_new = min(chi_j^2, chi) (Section 2).  choice "epsilon" (the paper's criterion): if
    epsilon < epsilon' then U is adopted, otherwise U' (R3).  Section 4.2.6 allows any rational
    criterion; "U" and "Uprime" always adopt that side (epsilon and epsilon' are still
    recorded).  With `multiplets`, columns of a multiplet split by the cut are zeroed (R8).
    """
    if choice not in CHOICES:
        raise ValueError(choice)
    n = A.shape[0]
    chi_new = min(n, chi)
    lam, U = eig_descending(A)
    lam_p, U_p = eig_descending(Ap)
    eps = judgement_value(lam, chi_new)
    eps_p = judgement_value(lam_p, chi_new)
    prime = (not eps < eps_p) if choice == "epsilon" else (choice == "Uprime")
    if not prime:
        Ut, prime, lam_c = U[:, :chi_new].copy(), False, lam
    else:
        Ut, prime, lam_c = U_p[:, :chi_new].copy(), True, lam_p
    kept = multiplet_safe_cut(lam_c, chi_new) if multiplets else chi_new
    Ut[:, kept:] = 0.0
    return Truncation(Ut, eps, eps_p, prime, lam, lam_p, chi_new, kept)


# ----------------------------------------------------------------------------
# Section 4.2.9: the new local tensor in three stages (eq. Contraction_NewTensor)
# ----------------------------------------------------------------------------


def _contract_leg(X: np.ndarray, axis: int, W: np.ndarray) -> np.ndarray:
    """Contract leg `axis` of X with the first index of the matrix W; the result
    index takes the place of the contracted leg."""
    Y = np.tensordot(X, W, axes=([axis], [0]))
    return np.moveaxis(Y, -1, axis)


def new_tensor(T: np.ndarray, Ut: dict[int, np.ndarray], only=None, T_check: np.ndarray | None = None,
               U_prime: dict[int, np.ndarray] | None = None) -> np.ndarray:
    """T^new[n_{d-1}..n_1, n'_{d-1}..n'_1, c, c'] from two copies of T (hat and check)
    and the isometries Ut[j] (chi_{n_j}^2 x chi_new_j), in the order of Section 4.2.9:

      prime chain   eqs. (TU1)..(TUNCD): contract each n'^check_j with U^(j)
      bottleneck    eq. (BottleneckPart): sum over n'^hat_{d-1}..n'^hat_1 and rho
      non-prime     eqs. (AfterBNNCD)..(AfterBN1): contract (n^hat_j, n^check_j) with U^(j)

    The loops run over n'_1 (outermost) .. n'_{d-1} (innermost) as in the paper,
    which bounds the intermediate size.  The hat copy supplies c, the check copy
    supplies c', and rho joins the hat copy's c' to the check copy's c.

    only: optional list of tuples (n'_1, .., n'_{d-1}); when given, only those slices
    of T^new are computed (the others stay zero) -- used to sample large cases.
    T_check, U_prime: the check copy and the isometries of the prime legs when they
    differ from T and Ut (the terms of the derivative, which is multilinear in them).
    """
    Tc = T if T_check is None else T_check
    Up = Ut if U_prime is None else U_prime
    d = T.ndim // 2
    chi_c = T.shape[axis_c(d)]
    chi_n = {j: T.shape[axis_n(d, j)] for j in range(1, d)}
    k = {j: Ut[j].shape[1] for j in range(1, d)}
    # U[(a b), new] with (a b) = a + b chi  ->  Wj[b, a, new]: b = check index, a = hat index
    Wm = {j: Ut[j].reshape(chi_n[j], chi_n[j], k[j]) for j in range(1, d)}
    Wp = {j: Up[j].reshape(chi_n[j], chi_n[j], k[j]) for j in range(1, d)}

    out_shape = tuple(k[j] for j in range(d - 1, 0, -1)) * 2 + (chi_c, chi_c)
    Tnew = np.zeros(out_shape)

    def prime_chain(C: np.ndarray, j: int, fixed: dict[int, int]) -> None:
        if j == d:
            bottleneck_and_non_prime(C, fixed)
            return
        for nj in range(k[j]):
            if only is not None and not any(
                    t[j - 1] == nj and all(t[i - 1] == fixed[i] for i in fixed) for t in only):
                continue
            # C^check(j) = sum_{n'^check_j} U^(j)[(n'^hat_j n'^check_j), n'_j] C^check(j-1)
            # the leg n'^check_j of C is replaced by n'^hat_j
            Uslice = Wp[j][:, :, nj]                     # [n'^check_j, n'^hat_j]
            Cj = _contract_leg(C, axis_np(d, j), Uslice)
            prime_chain(Cj, j + 1, {**fixed, j: nj})

    def bottleneck_and_non_prime(Cck: np.ndarray, fixed: dict[int, int]) -> None:
        # Cck legs: (n^check_{d-1}..n^check_1, n'^hat_{d-1}..n'^hat_1, rho, c')
        # T^hat legs: (n^hat_{d-1}..n^hat_1, n'^hat_{d-1}..n'^hat_1, c, rho)
        hat_axes = [axis_np(d, j) for j in range(d - 1, 0, -1)] + [axis_cp(d)]
        chk_axes = [axis_np(d, j) for j in range(d - 1, 0, -1)] + [axis_c(d)]
        # eq. (BottleneckPart): C^hat(d-1)[n^hat.., c, n^check.., c']
        Ch = np.tensordot(T, Cck, axes=(hat_axes, chk_axes))
        # Ch legs: n^hat_{d-1}..n^hat_1 (0..d-2), c (d-1), n^check_{d-1}..n^check_1 (d..2d-2), c' (2d-1)
        # eqs. (AfterBNNCD)..(AfterBN1): contract (n^hat_j, n^check_j) with U^(j),
        # j = d-1 first; the hat leg becomes n_j, the check leg disappears.
        for j in range(d - 1, 0, -1):
            pos_hat = d - 1 - j
            # check legs of larger j were removed already, so n^check_j sits right after c
            pos_chk = d
            L = _letters(Ch.ndim)
            a = list(L)
            a[pos_hat], a[pos_chk] = "P", "Q"
            out = list(L)
            out[pos_hat] = "N"
            del out[pos_chk]
            Ch = np.einsum("".join(a) + ",QPN->" + "".join(out), Ch, Wm[j], optimize=True)
        # Ch legs now: n_{d-1}..n_1, c, c'
        idx = tuple(slice(None) for _ in range(d - 1))
        idx += tuple(fixed[j] for j in range(d - 1, 0, -1))
        Tnew[idx] = Ch

    prime_chain(Tc, 1, {})
    return Tnew


def rename(Tnew: np.ndarray) -> np.ndarray:
    """Renaming before the next step (eq. rename_indices): c^bar = n_1, c^bar' = n'_1,
    n^bar_j = n_{j+1}, n^bar'_j = n'_{j+1} (j = 1..d-2), n^bar_{d-1} = c, n^bar'_{d-1} = c'."""
    d = Tnew.ndim // 2
    order = []
    # non-primed block n^bar_{d-1}..n^bar_1
    order.append(axis_c(d))                           # n^bar_{d-1} = c
    for jb in range(d - 2, 0, -1):                    # n^bar_jb = n_{jb+1}
        order.append(axis_n(d, jb + 1))
    # primed block
    order.append(axis_cp(d))
    for jb in range(d - 2, 0, -1):
        order.append(axis_np(d, jb + 1))
    order.append(axis_n(d, 1))                        # c^bar = n_1
    order.append(axis_np(d, 1))                       # c^bar' = n'_1
    return np.ascontiguousarray(np.transpose(Tnew, order))


# ----------------------------------------------------------------------------
# One coarse-graining step and the lnZ bookkeeping of Section 4.1.1
# ----------------------------------------------------------------------------


@dataclass
class StepRecord:
    p: int
    trace: float                  # Tr T^(p) of the new (not yet normalised) tensor
    lnz_per_site: float           # ln Z^(p) / V^(p)
    gu_wen: float
    dims_before: tuple
    truncations: dict = field(default_factory=dict)


def coarse_grain(T: np.ndarray, chi: int, multiplets: bool = True, choice: str = "epsilon"):
    """One coarse-graining step along the Current direction of T (Sections 3-4).

    Returns (T^new before normalisation and before renaming, truncations).
    """
    d = T.ndim // 2
    tr = {}
    Ut = {}
    for j in range(1, d):
        A = gram_matrix(T, axis_n(d, j))              # non-prime side
        Ap = gram_matrix(T, axis_np(d, j))            # prime side
        tr[j] = choose_isometry(A, Ap, chi, multiplets, choice)
        Ut[j] = tr[j].U
    return new_tensor(T, Ut), tr


@dataclass
class Model:
    kind: str = "ising"           # "ising" or "potts"
    d: int = 2
    q: int = 2
    J: float = 1.0
    h: float = 0.0


def normalisation_factor(T: np.ndarray, norm: str) -> float:
    """f^(p) of Section 3.1.3.  "trace": 1/Tr T (the paper's example, R4);
    "maxabs": 1/max|T|, another admissible choice used to pin that lnZ/V does not
    depend on it."""
    if norm == "trace":
        return 1.0 / trace(T)
    if norm == "maxabs":
        return 1.0 / float(np.max(np.abs(T)))
    raise ValueError(norm)


def run(model: Model, beta: float, chi: int, steps: int, T0: np.ndarray | None = None,
        on_step=None, norm: str = "trace", multiplets: bool = True, choice: str = "epsilon"):
    """Full oracle run: initial tensor, normalisation, `steps` coarse-graining steps.

    lnZ bookkeeping follows eqs. (eq_lnZ) and (K_recurrence):
        K^(0) = 0,  K^(q) = 2 (K^(q-1) + ln(1/f^(q-1))),
        ln Z^(p) = K^(p) + ln Tr T^(p),  V^(p) = 2^p,
    with f^(p) = 1 / Tr T^(p) (R4).  Returns (lnz_per_site at p = 0, list of StepRecord).
    """
    if T0 is None:
        W, V = boltzmann_weights(model.kind, beta, model.q, model.J, model.h)
        T0 = initial_tensor(W, V, model.d)
    t0 = trace(T0)
    K = 0.0                                            # K^(0)
    lnz0 = K + math.log(t0)                            # ln Z^(0) / V^(0), V^(0) = 1
    f = normalisation_factor(T0, norm)                 # f^(0)
    T = f * T0
    K = 2.0 * (K + math.log(1.0 / f))                  # K^(1)
    records = []
    for p in range(1, steps + 1):
        dims = T.shape
        Tnew, tr = coarse_grain(T, chi, multiplets, choice)
        t = trace(Tnew)
        if not (t > 0.0 and math.isfinite(t)):
            raise FloatingPointError(f"non-positive trace at step {p}: {t}")
        lnz = K + math.log(t)                          # ln Z^(p)
        rec = StepRecord(p, t, lnz / 2.0 ** p, gu_wen_ratio(Tnew), dims, tr)
        records.append(rec)
        if on_step is not None:
            on_step(rec)
        f = normalisation_factor(Tnew, norm)           # f^(p)
        K = 2.0 * (K + math.log(1.0 / f))              # K^(p+1)
        T = rename(f * Tnew)
    return lnz0, records


def lattice_shape(d: int, steps: int) -> tuple:
    """Periodic torus represented after `steps` steps starting with axis 0 (R6, R7)."""
    L = [1] * d
    for p in range(steps):
        L[p % d] *= 2
    return tuple(L)


def free_energy_per_site(lnz_per_site: float, beta: float) -> float:
    """f = -(1/beta) lnZ/V."""
    return -lnz_per_site / beta
