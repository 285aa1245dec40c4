"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds none of the method's arithmetic: only random numbers with fixed seeds in
the shapes the method uses (dense local tensors, isometries with orthonormal
columns), and the physics configurations as plain parameter records.
"""

import numpy as np


def random_tensor(shape, seed=0, scale=1.0):
    """Dense FP64 tensor with i.i.d. N(0, scale^2) entries."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal(shape)


def random_isometry(n, k, seed=0):
    """n x k matrix with orthonormal columns: Q of the QR factorisation of an
    n x k Gaussian matrix (signs fixed so that diag(R) > 0)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, k))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))[None, :]


# Physics configurations (model, d, q, temperatures or betas, chi, steps).
CONFIG1 = dict(kind="ising", d=2, q=2, temps=(2.0, 2.269185, 2.5), chi=8, steps=20)
CONFIG2 = dict(kind="ising", d=3, q=2, temps=(4.0, 4.5115, 5.0), chi=8, steps=30)
CONFIG3 = dict(kind="ising", d=3, q=2, temps=(4.5115,), chi=16, steps=25)
CONFIG4_3D = dict(kind="ising", d=3, q=2, temps=tuple(np.linspace(4.0, 5.0, 64)), chi=12, steps=20)
CONFIG4_2D = dict(kind="ising", d=2, q=2, betas=tuple(np.linspace(0.3, 0.6, 48)),
                  chis=(16, 24, 32), steps=20)
CONFIG5 = dict(kind="potts", d=3, q=3, betas=(0.50, 0.55, 0.60), chi=16, steps=20)
# 4D Ising (the paper's own model, Section 5) at a bond dimension the oracle runs in seconds per
# step; T around the 4D critical temperature (about 6.68)
CONFIG6 = dict(kind="ising", d=4, q=2, temps=(6.0, 6.68, 7.5), chi=4, steps=12)
# ... and at chi = 5 (H = 625: no dimension a multiple of a GEMM tile), one temperature
CONFIG7 = dict(kind="ising", d=4, q=2, temps=(6.68,), chi=5, steps=8)


def rank_deficient_gram(n, m, sectors, seed):
    """Symmetric positive semidefinite n x n matrix shaped like the Gram matrix of an ordered
    phase: `sectors` blocks of m indices (scattered over n), each a rank-one term of weight
    1/sectors plus a tail of order 1e-20; every other entry exactly zero, so only `sectors`
    eigenvalues are non-negligible."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    idx = rng.permutation(n)
    for s in range(sectors):
        sec = idx[s * m:(s + 1) * m]
        v = rng.standard_normal(m)
        v /= np.linalg.norm(v)
        tail = rng.standard_normal((m, m)) * 1e-10
        A[np.ix_(sec, sec)] = np.outer(v, v) / sectors + tail @ tail.T
    return 0.5 * (A + A.T)


def random_positive_tensor(shape, seed=0, spread=0.5):
    """Dense FP64 tensor with i.i.d. entries exp(spread * N(0, 1)) (all positive, so every
    trace of a network of copies is positive)."""
    return np.exp(random_tensor(shape, seed=seed, scale=spread))
