"""The inertia counter used as the full-size spectrum pin agrees with the
eigenvalues of small symmetric matrices, including ones whose factorization
must take 2 x 2 pivots (zero diagonal), and with the generalized count of a
pencil (H, S) against the oracle's eigenvalues."""
import numpy as np
import pytest

from paper_1912_13403_amd import inputs
from tests.inertia import negative_count


@pytest.mark.parametrize("seed", range(6))
def test_negative_count_matches_eigenvalues(seed):
    rng = np.random.default_rng(seed)
    n = 40 + 7 * seed
    A = rng.standard_normal((n, n))
    A = A + A.T
    if seed % 2:
        A[np.diag_indices(n)] = 0.0   # forces 2 x 2 pivots
    shift = rng.uniform(-3, 3)
    A = A - shift * np.eye(n)
    assert negative_count(A) == int(np.sum(np.linalg.eigvalsh(A) < 0))


def test_pencil_count_matches_oracle(oracle):
    n = 120
    H, S = inputs.sized_problem(n, cfg=31)
    w, _ = oracle.solve_ev(H, S)
    for k in (1, 37, 60, 119):
        sigma = 0.5 * (w[k - 1] + w[k])
        assert negative_count(H - sigma * S) == k
