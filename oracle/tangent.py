"""Forward-mode derivative d(lnZ/V)/d(beta) of the oracle run (TEST INFRASTRUCTURE ONLY).

Every quantity of oracle.hotrg.run is carried together with its derivative with
respect to beta, by the product rule through the same steps in the same order:

* bond factor X = U sqrt(Lambda): for the Ising and Potts weights the eigenvectors U
  of W do not depend on beta, so dX = U diag(dlambda / (2 sqrt(lambda))) with
  dlambda_i = u_i^T (dW/dbeta) u_i (checked at run time);
* initial tensor (eq. 4) and its trace;
* Gram matrices: A is a sum of products of two bilinear forms of T (Section 3.2);
* decomposition: for each kept column k of the adopted isometry,
      dU_k = sum_{l not kept} U_l (U_l^T dA U_k) / (lambda_k - lambda_l);
  rotations among kept columns are a bond gauge that leaves lnZ unchanged, so those
  terms are left out; the choice U / U' and the multiplet rule are held fixed;
* new tensor: multilinear in (hat copy, check copy, isometries of the non-prime legs,
  isometries of the prime legs), so its derivative is the sum of the terms with one
  factor differentiated;
* trace, lnZ/V (eqs. eq_lnZ, K_recurrence) and the normalisation by 1/Tr.
"""

from __future__ import annotations

import math

import numpy as np

from . import hotrg as H


def weight_derivatives(model: H.Model, beta: float):
    """dW/dbeta and dV/dbeta for the weights of oracle.hotrg.boltzmann_weights."""
    W, V = H.boltzmann_weights(model.kind, beta, model.q, model.J, model.h)
    if model.kind == "ising":
        s = np.array([1.0, -1.0])
        dW = model.J * np.outer(s, s) * W
        dV = model.h * s * V
    else:
        dW = model.J * np.eye(model.q) * W
        dV = np.zeros(model.q)
    return W, V, dW, dV


def bond_factor_tangent(W: np.ndarray, dW: np.ndarray):
    lam, U = np.linalg.eigh(W)
    if np.min(lam) < -1e-12 * np.max(np.abs(lam)):
        raise ValueError("W is not positive semi-definite")
    D = U.T @ dW @ U
    off = D - np.diag(np.diag(D))
    if np.max(np.abs(off)) > 1e-12 * max(1.0, np.max(np.abs(D))):
        raise ValueError("eigenvectors of W depend on beta; closed-form tangent does not apply")
    dlam = np.diag(D)
    sq = np.sqrt(np.clip(lam, 0.0, None))
    with np.errstate(divide="ignore", invalid="ignore"):
        dsq = np.where(sq > 0, dlam / (2.0 * sq), 0.0)
    return U * sq[None, :], U * dsq[None, :]


def initial_tensor_tangent(X, dX, V, dV, d):
    q = X.shape[0]
    T = np.zeros((q,) * (2 * d))
    dT = np.zeros_like(T)
    for s in range(q):
        vec, dvec = X[s], dX[s]
        # T_s = V_s (x)^{2d} vec; dT_s = dV_s (x) vec + V_s sum over legs of the product with dvec
        prod = np.array(1.0)
        for _ in range(2 * d):
            prod = np.multiply.outer(prod, vec)
        T += V[s] * prod
        dT += dV[s] * prod
        for leg in range(2 * d):
            term = np.array(1.0)
            for l2 in range(2 * d):
                term = np.multiply.outer(term, dvec if l2 == leg else vec)
            dT += V[s] * term
    return T, dT


def gram_tangent(T, dT, side_axis):
    Sh = H.s_hat(T, side_axis)
    Sc = H.s_check(T, side_axis)
    dSh = H.s_hat(dT, side_axis, T) + H.s_hat(T, side_axis, dT)
    dSc = H.s_check(dT, side_axis, T) + H.s_check(T, side_axis, dT)
    return H.combine_gram(Sh, Sc), H.combine_gram(dSh, Sc) + H.combine_gram(Sh, dSc)


def isometry_tangent(A, dA, Ap, dAp, chi):
    """Choice and truncation as in oracle.hotrg.choose_isometry, plus dU of the kept columns."""
    tr = H.choose_isometry(A, Ap, chi)
    Am, dAm = (Ap, dAp) if tr.chose_prime else (A, dA)
    lam, U = H.eig_descending(Am)
    kept = tr.kept
    Ut = np.zeros((U.shape[0], tr.chi_new))
    dUt = np.zeros_like(Ut)
    Ut[:, :kept] = U[:, :kept]
    Ud = U[:, kept:]
    M = Ud.T @ dAm @ U[:, :kept]                          # [discarded, kept]
    gap = lam[None, :kept] - lam[kept:, None]
    dUt[:, :kept] = Ud @ (M / gap)
    # the oracle's own isometry may differ from U[:, :kept] by column signs (same eigh):
    assert np.allclose(np.abs(np.sum(Ut[:, :kept] * tr.U[:, :kept], axis=0)), 1.0, atol=1e-8)
    return tr, Ut, dUt


def run_with_tangent(model: H.Model, beta: float, chi: int, steps: int, on_step=None):
    """Returns (lnz0, dlnz0, [(lnz_p, dlnz_p) for p = 1..steps]).  on_step(p, lnz_p, dlnz_p),
    when given, is called after every step (progress reports; no effect on the values)."""
    W, V, dW, dV = weight_derivatives(model, beta)
    X, dX = bond_factor_tangent(W, dW)
    T0, dT0 = initial_tensor_tangent(X, dX, V, dV, model.d)
    t0, dt0 = H.trace(T0), H.trace(dT0)
    lnz, dlnz = math.log(t0), dt0 / t0
    out0 = (lnz, dlnz)
    T, dT = T0 / t0, dT0 / t0 - T0 * dt0 / t0 ** 2
    d = model.d
    recs = []
    for p in range(1, steps + 1):
        Ut, dUt = {}, {}
        for j in range(1, d):
            A, dA = gram_tangent(T, dT, H.axis_n(d, j))
            Ap, dAp = gram_tangent(T, dT, H.axis_np(d, j))
            _, Ut[j], dUt[j] = isometry_tangent(A, dA, Ap, dAp, chi)
        Tnew = H.new_tensor(T, Ut)
        dTnew = H.new_tensor(dT, Ut, T_check=T) + H.new_tensor(T, Ut, T_check=dT)
        for j in range(1, d):
            Uj = {**Ut, j: dUt[j]}
            dTnew += H.new_tensor(T, Uj, U_prime=Ut) + H.new_tensor(T, Ut, U_prime=Uj)
        t, dt = H.trace(Tnew), H.trace(dTnew)
        lnz += math.log(t) / 2.0 ** p
        dlnz += (dt / t) / 2.0 ** p
        recs.append((lnz, dlnz))
        if on_step is not None:
            on_step(p, lnz, dlnz)
        T = H.rename(Tnew / t)
        dT = H.rename(dTnew / t - Tnew * dt / t ** 2)
    return out0[0], out0[1], recs
