"""Sylvester inertia of a dense symmetric matrix from a Bunch-Kaufman LDL^T.

Test infrastructure.  For a symmetric pencil (H, S) with S positive definite,
the number of eigenvalues below sigma equals the number of negative
eigenvalues of H - sigma S (Sylvester's law of inertia applied to the
congruence with the Cholesky factor of S), and that equals the number of
negative eigenvalues of the block-diagonal D of H - sigma S = L D L^T.  This
pins the spectrum of the path at sizes the oracle cannot reach: LAPACK's
symmetric indefinite factorization (through torch's CPU linalg) shares
nothing with the eigensolver under test.
"""
from __future__ import annotations

import numpy as np


def negative_count(A) -> int:
    """Number of negative eigenvalues of the symmetric matrix A (lower
    triangle read), from D of A = L D L^T (1 x 1 and 2 x 2 pivot blocks in
    LAPACK's sytrf convention: pivots[k] > 0 marks a 1 x 1 block, a pair of
    equal negative pivots a 2 x 2 block)."""
    import torch

    T = torch.as_tensor(np.asarray(A, dtype=np.float64))
    LD, piv = torch.linalg.ldl_factor(T)
    piv = piv.numpy()
    dg = torch.diagonal(LD).numpy().copy()
    sub = torch.diagonal(LD, -1).numpy().copy()
    del LD, T
    n = dg.shape[0]
    neg = 0
    k = 0
    while k < n:
        if piv[k] > 0:
            neg += int(dg[k] < 0.0)
            k += 1
        else:
            a, b, c = dg[k], sub[k], dg[k + 1]
            det = a * c - b * b
            if det < 0.0:
                neg += 1          # one eigenvalue of each sign
            elif a + c < 0.0:
                neg += 2          # both negative
            k += 2
    return neg
