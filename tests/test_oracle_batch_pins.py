"""Pins for the oracle's shared chemical potential over several unit tasks
(Eq. (16)): the k-point x spin problems form one block-diagonal pencil
(Sec. 2.3), so a batch must equal the single solve of the block-diagonal
union; a task of weight 2 equals the same task listed twice; and a Fermi
level degenerate across tasks is shared as in the closed form of two chains."""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1912_13403_amd import inputs


def _blocks(X, sizes):
    out, o = [], 0
    for n in sizes:
        out.append(X[o:o + n, o:o + n])
        o += n
    return out


@pytest.mark.parametrize("kT", [0.0, 0.02])
def test_real_batch_equals_block_diagonal_union(oracle, kT):
    sizes = [23, 40, 31]
    probs = [inputs.sized_problem(n, cfg=60 + i) for i, n in enumerate(sizes)]
    Hs, Ss = [p[0] for p in probs], [p[1] for p in probs]
    ne = 41.0
    b = oracle.solve_dm_batch(Hs, Ss, ne, kT, f_max=2.0)
    Hu = sl.block_diag(*[np.tril(H) + np.tril(H, -1).T for H in Hs])
    Su = sl.block_diag(*[np.tril(S) + np.tril(S, -1).T for S in Ss])
    u = oracle.solve_dm(Hu, Su, ne, kT, f_max=2.0, deg_tol=1e-12 * max(oracle.norm1(H) for H in Hs))
    for D, Du in zip(b["D"], _blocks(u["D"], sizes)):
        assert np.max(np.abs(D - Du)) < 1e-12
    for E, Eu in zip(b["E"], _blocks(u["E"], sizes)):
        assert np.max(np.abs(E - Eu)) < 1e-12
    assert abs(b["mu"] - u["mu"]) < 1e-12
    assert abs(b["band_energy"] - u["band_energy"]) < 1e-11
    # the union's density matrix has no coupling between tasks
    o = sizes[0]
    assert np.max(np.abs(u["D"][o:, :o])) < 1e-12


def test_complex_batch_equals_block_diagonal_union(oracle):
    sizes = [17, 29]
    Hs, Ss = [], []
    for i, n in enumerate(sizes):
        Hu, Hd, S = inputs.kpoint_problem(10 + i, n=n)
        Hs += [Hu, Hd]
        Ss += [S, S]
    ne, kT = 19.0, 0.01
    b = oracle.solve_dm_batch(Hs, Ss, ne, kT, f_max=1.0)
    herm = lambda A: np.tril(A, -1) + np.tril(A, -1).conj().T + np.diag(np.real(np.diag(A)))
    u = oracle.solve_dm_complex(sl.block_diag(*[herm(H) for H in Hs]),
                                sl.block_diag(*[herm(S) for S in Ss]), ne, kT, f_max=1.0)
    bl = [n for n in sizes for _ in range(2)]
    for D, Du in zip(b["D"], _blocks(u["D"], bl)):
        assert np.max(np.abs(D - Du)) < 1e-12
    assert abs(b["mu"] - u["mu"]) < 1e-12
    assert abs(b["band_energy"] - u["band_energy"]) < 1e-11


@pytest.mark.parametrize("kT", [0.0, 0.03])
def test_weight_two_equals_task_listed_twice(oracle, kT):
    H1, S1 = inputs.sized_problem(30, cfg=70)
    H2, S2 = inputs.sized_problem(26, cfg=71)
    ne = 37.0
    a = oracle.solve_dm_batch([H1, H2, H2], [S1, S2, S2], ne, kT, f_max=1.0)
    b = oracle.solve_dm_batch([H1, H2], [S1, S2], ne, kT, weights=[1.0, 2.0], f_max=1.0)
    assert abs(a["mu"] - b["mu"]) < 1e-12
    assert np.max(np.abs(a["D"][0] - b["D"][0])) < 1e-12
    assert np.max(np.abs(a["D"][1] - b["D"][1])) < 1e-12
    assert abs(a["band_energy"] - b["band_energy"]) < 1e-11


def test_fermi_level_shared_across_tasks_closed_form(oracle):
    # two identical chains (f_max = 1) with 5 electrons: levels 1 and 2 of both
    # tasks are full and level 3, degenerate across the tasks, holds 1/2 each
    n = 10
    H, S = inputs.chain(n)
    b = oracle.solve_dm_batch([H, H], [S, S], 5.0, 0.0, f_max=1.0)
    k = np.arange(1, n + 1)
    eps = -2.0 * np.cos(k * np.pi / (n + 1))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(k, k) * np.pi / (n + 1))
    o = np.argsort(eps)
    V = V[:, o]
    D = V[:, :2] @ V[:, :2].T + 0.5 * np.outer(V[:, 2], V[:, 2])
    for Dp in b["D"]:
        assert np.max(np.abs(Dp - D)) < 1e-13
    assert abs(b["mu"] - eps[o][2]) < 1e-14
