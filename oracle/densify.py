"""Densify an H-matrix given as blocks (Section 2: dense sub-blocks plus
low-rank sub-blocks U V^T), in the permuted order of its cluster tree. Used
to split the H error into the approximation part and the arithmetic part.
"""
from __future__ import annotations

import numpy as np


def densify_lower(n: int, dense_blocks, lowrank_blocks, symmetric: bool = True) -> np.ndarray:
    """dense_blocks: iterable of (r0, c0, D) with D a 2-D array placed at
    [r0:r0+m, c0:c0+k]; lowrank_blocks: iterable of (r0, c0, U, V) placed as
    U V^T. Off-diagonal blocks are mirrored when ``symmetric``; diagonal
    blocks are taken from their lower triangle."""
    A = np.zeros((n, n))
    for r0, c0, D in dense_blocks:
        D = np.asarray(D, dtype=np.float64)
        m, k = D.shape
        if r0 == c0:
            Dl = np.tril(D)
            A[r0:r0 + m, c0:c0 + k] = Dl + (np.tril(D, -1).T if symmetric else 0.0)
        else:
            A[r0:r0 + m, c0:c0 + k] = D
            if symmetric:
                A[c0:c0 + k, r0:r0 + m] = D.T
    for r0, c0, U, V in lowrank_blocks:
        B = np.asarray(U, dtype=np.float64) @ np.asarray(V, dtype=np.float64).T
        m, k = B.shape
        A[r0:r0 + m, c0:c0 + k] = B
        if symmetric:
            A[c0:c0 + k, r0:r0 + m] = B.T
    return A
