"""Index bookkeeping between the oracle's order and the library's storage order.

Oracle (paper, Section 3.1.3): T[n_{d-1}..n_1, n'_{d-1}..n'_1, c, c'].
Library storage:               T[c][n_1]..[n_{d-1}][c'][n'_1]..[n'_{d-1}]  (an H x H matrix).
Pure transposes; no arithmetic of the method.
"""

import numpy as np


def paper_to_storage_axes(d):
    # storage slot 0 = c (paper axis 2d-2), slot j = n_j (paper axis d-1-j); primed likewise
    ax = [2 * d - 2] + [d - 1 - j for j in range(1, d)]
    ax += [2 * d - 1] + [2 * d - 2 - j for j in range(1, d)]
    return ax


def to_storage(T_paper):
    d = T_paper.ndim // 2
    return np.ascontiguousarray(np.transpose(T_paper, paper_to_storage_axes(d)))


def to_paper(T_storage):
    d = T_storage.ndim // 2
    inv = np.argsort(paper_to_storage_axes(d))
    return np.ascontiguousarray(np.transpose(T_storage, inv))


def storage_dims(T_paper):
    """(chi_c, chi_{n_1}, .., chi_{n_{d-1}}) of a tensor in paper order."""
    d = T_paper.ndim // 2
    return [T_paper.shape[2 * d - 2]] + [T_paper.shape[d - 1 - j] for j in range(1, d)]
