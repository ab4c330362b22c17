"""Dense matrices of a (small) problem, for brute-force evaluation.

Builds C and every A_i as dense symmetric n x n arrays straight from the
triplets: an off-diagonal triplet (j, k, a) sets both (j, k) and (k, j).
"""
from __future__ import annotations

import numpy as np


def dense_C(prob) -> np.ndarray:
    C = np.zeros((prob.n, prob.n))
    for j, k, v in zip(prob.c_row, prob.c_col, prob.c_val):
        C[j, k] += v
        if j != k:
            C[k, j] += v
    return C


def dense_A(prob) -> np.ndarray:
    A = np.zeros((prob.m, prob.n, prob.n))
    for i, j, k, v in zip(prob.a_con, prob.a_row, prob.a_col, prob.a_val):
        A[i, j, k] += v
        if j != k:
            A[i, k, j] += v
    return A
