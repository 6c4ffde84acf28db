"""Pins for the FP64 CPU oracle: checks against facts fixed by the paper's
definitions and by mathematics, never against the oracle itself.

References are to the ELSI 2.x paper (arXiv:1912.13403): the pencil H C = S C eps
(Eq. 3), the density matrix (Eq. 4), its conditions (Eq. 6, and the
non-orthogonal forms Tr(P S) = N_e, P = P S P of the extrapolation section),
the energy-weighted density matrix (Eq. 17), occupations from eigenvalues and
the electron count (Sec. 2.6).
"""
import numpy as np
import pytest
import scipy.linalg as sl

from paper_1912_13403_amd import inputs


def _chain_exact(n, t):
    k = np.arange(1, n + 1)
    eps = 2.0 * t * np.cos(k * np.pi / (n + 1))
    j = np.arange(1, n + 1)
    U = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, k) * np.pi / (n + 1))
    order = np.argsort(eps, kind="stable")
    return eps[order], U[:, order]


# --- closed forms -----------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 50, 129])
def test_chain_eigenvalues_closed_form(oracle, n):
    t = -1.0
    H, S = inputs.chain(n, t)
    w, C = oracle.solve_ev(H, S)
    eps, U = _chain_exact(n, t)
    scale = max(oracle.norm1(H), 1.0)
    assert np.max(np.abs(w - eps)) <= 1e-14 * scale * 4
    # eigenvalues are simple: each eigenvector is fixed up to sign
    for l in range(n):
        s = np.sign(C[:, l] @ U[:, l])
        assert np.max(np.abs(s * C[:, l] - U[:, l])) < 1e-12


@pytest.mark.parametrize("n,ne", [(50, 40), (129, 100), (64, 64)])
def test_chain_density_closed_form(oracle, n, ne):
    t = -1.0
    H, S = inputs.chain(n, t)
    r = oracle.solve_dm(H, S, ne, 0.0, f_max=2.0)
    eps, U = _chain_exact(n, t)
    nocc = ne // 2
    D = 2.0 * U[:, :nocc] @ U[:, :nocc].T
    E = 2.0 * (U[:, :nocc] * eps[:nocc]) @ U[:, :nocc].T
    assert np.max(np.abs(r["D"] - D)) < 1e-13
    assert np.max(np.abs(r["E"] - E)) < 1e-13
    assert abs(r["band_energy"] - 2.0 * eps[:nocc].sum()) < 1e-12
    assert abs(r["mu"] - 0.5 * (eps[nocc - 1] + eps[nocc])) < 1e-14


def test_generalized_chain_congruence(oracle):
    """(L H_c L^T, L L^T) has the chain's eigenvalues and D = L^-T D_c L^-1."""
    n, t = 96, -0.7
    Hc, _ = inputs.chain(n, t)
    _, S0 = inputs.sized_problem(n, cfg=5)
    L = np.linalg.cholesky(S0)
    H = L @ Hc @ L.T
    S = L @ L.T
    eps, U = _chain_exact(n, t)
    w, C = oracle.solve_ev(H, S)
    assert np.max(np.abs(w - eps)) <= 1e-13 * oracle.norm1(H)
    ne = 60
    r = oracle.solve_dm(H, S, ne, 0.0)
    Linv = np.linalg.inv(L)
    Dc = 2.0 * U[:, : ne // 2] @ U[:, : ne // 2].T
    D = Linv.T @ Dc @ Linv
    assert np.max(np.abs(r["D"] - D)) < 1e-12


def test_ring_degenerate_fermi_level_shares(oracle):
    """Periodic ring, no flux: eps_k = 2t cos(2 pi k / n) in degenerate pairs.
    With the Fermi level inside a pair, both states share the remaining
    electrons (the kT -> 0+ limit) and D is the rotation-invariant
    D_ij = (1/n) sum_k f_k cos(2 pi k (i-j)/n)."""
    n, t = 40, -1.0
    H, S = inputs.ring(n, t)
    k = np.arange(n)
    eps_k = 2 * t * np.cos(2 * np.pi * k / n)
    ne = 2 * 5 + 2  # k=0 (2 e), k=+-1, +-2 (8 e), then 2 e into the +-3 pair
    f_k = np.zeros(n)
    order = np.argsort(eps_k, kind="stable")
    f_k[order[:5]] = 2.0
    f_k[order[5:7]] = 1.0
    ij = np.subtract.outer(np.arange(n), np.arange(n))
    D = (f_k[None, None, :] * np.cos(2 * np.pi * np.multiply.outer(ij, k) / n)).sum(-1) / n
    r = oracle.solve_dm(H, S, ne, 0.0)
    assert np.max(np.abs(r["D"] - D)) < 1e-12
    assert np.sum(r["f"] == 1.0) == 2
    assert abs(r["mu"] - eps_k[order[5]]) < 1e-12


# --- brute force ------------------------------------------------------------

def _mp_pencil(H, S, dps=40):
    import mpmath as mp
    mp.mp.dps = dps
    n = H.shape[0]
    Hm = mp.matrix(n, n)
    Sm = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            a, b = (i, j) if i >= j else (j, i)
            Hm[i, j] = mp.mpf(float(H[a, b]))
            Sm[i, j] = mp.mpf(float(S[a, b]))
    L = mp.cholesky(Sm)
    Li = mp.inverse(L)
    A = Li * Hm * Li.T
    A = (A + A.T) / 2
    E, Q = mp.eigsy(A)
    C = Li.T * Q
    w = [E[i] for i in range(n)]
    order = sorted(range(n), key=lambda i: w[i])
    return mp, [w[i] for i in order], C, order


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_brute_force_mpmath(oracle, n):
    H, S = inputs.sized_problem(n, cfg=11 + n)
    mp, w_mp, C_mp, order = _mp_pencil(H, S)
    w, C = oracle.solve_ev(H, S)
    scale = oracle.norm1(H)
    assert np.max(np.abs(w - np.array([float(x) for x in w_mp]))) <= 1e-14 * scale * 4
    nocc = max(n // 2, 1)
    if n > 1:
        r = oracle.solve_dm(H, S, 2 * nocc, 0.0)
        D = np.zeros((n, n))
        for l in range(nocc):
            c = [C_mp[i, order[l]] for i in range(n)]
            for i in range(n):
                for j in range(n):
                    D[i, j] += float(2 * c[i] * c[j])
        assert np.max(np.abs(r["D"] - D)) < 1e-13


def _inertia_below(H, S, sigma):
    """#eigenvalues of (H,S) below sigma = #negative eigenvalues of H - sigma S
    (Sylvester), from a Bunch-Kaufman LDL^T (scipy/LAPACK)."""
    Hf = np.tril(H) + np.tril(H, -1).T
    Sf = np.tril(S) + np.tril(S, -1).T
    _, Dm, _ = sl.ldl(Hf - sigma * Sf, lower=True)
    return int(np.sum(np.linalg.eigvalsh(Dm) < 0))


def test_inertia_bisection_brute_force(oracle):
    n = 48
    H, S = inputs.sized_problem(n, cfg=21)
    w, _ = oracle.solve_ev(H, S)
    lo0, hi0 = -10.0, 10.0
    for l in range(n):
        lo, hi = lo0, hi0
        for _ in range(70):
            mid = 0.5 * (lo + hi)
            if _inertia_below(H, S, mid) > l:
                hi = mid
            else:
                lo = mid
        assert abs(0.5 * (lo + hi) - w[l]) <= 1e-13 * oracle.norm1(H)


# --- library cross-check ------------------------------------------------------

def _fd_mu(eps, ne, kT, fmax=2.0):
    from scipy.optimize import brentq

    def g(mu):
        x = (eps - mu) / kT
        return np.sum(fmax * 0.5 * (1 - np.tanh(0.5 * x))) - ne
    return brentq(g, eps[0] - 50 * kT - 1, eps[-1] + 50 * kT + 1, xtol=1e-15, rtol=1e-15)


@pytest.mark.parametrize("n,kT", [(300, 0.01), (257, 0.005)])
def test_scipy_eigh_cross_check(oracle, n, kT):
    H, S = inputs.sized_problem(n, cfg=31)
    w_ref, C_ref = sl.eigh(np.tril(H) + np.tril(H, -1).T, np.tril(S) + np.tril(S, -1).T)
    ne = n / 2.0
    r = oracle.solve_dm(H, S, ne, kT)
    scale = oracle.norm1(H)
    assert np.max(np.abs(r["eval"] - w_ref)) <= 1e-12 * scale
    mu = _fd_mu(w_ref, ne, kT)
    assert abs(r["mu"] - mu) < 1e-10 * scale
    f = 2.0 * 0.5 * (1 - np.tanh(0.5 * (w_ref - mu) / kT))
    D = (C_ref * f) @ C_ref.T
    E = (C_ref * (f * w_ref)) @ C_ref.T
    assert np.max(np.abs(r["D"] - D)) < 1e-11
    assert np.max(np.abs(r["E"] - E)) < 1e-11 * max(1.0, scale)


# --- invariants of D and E ----------------------------------------------------

def test_zero_temperature_invariants_cfg0(oracle):
    H, S, p = inputs.config_problem("cfg0_n512")
    Hf = np.tril(H) + np.tril(H, -1).T
    Sf = np.tril(S) + np.tril(S, -1).T
    r = oracle.solve_dm(H, S, p["n_electrons"], p["kT"], f_max=p["f_max"])
    D, E = r["D"], r["E"]
    ne = p["n_electrons"]
    assert abs(np.trace(D @ Sf) - ne) < 1e-12 * ne
    assert abs(np.trace(D @ Hf) - r["band_energy"]) < 1e-10
    assert abs(np.trace(E @ Sf) - r["band_energy"]) < 1e-10
    assert np.max(np.abs(Sf @ E - Hf @ D)) < 1e-11
    P = D / 2.0
    assert np.max(np.abs(P @ Sf @ P - P)) < 1e-12
    assert np.max(np.abs(D - D.T)) < 1e-13
    C = r["C"]
    assert np.max(np.abs(C.T @ Sf @ C - np.eye(p["n"]))) < 1e-12 * p["n"]
    res = Hf @ C - (Sf @ C) * r["eval"]
    assert np.max(np.abs(res).sum(axis=0)) / (p["n"] * oracle.norm1(H)) < 1e-15


def test_finite_temperature_invariants(oracle):
    n, kT, ne = 200, 0.02, 90.0
    H, S = inputs.sized_problem(n, cfg=41)
    Sf = np.tril(S) + np.tril(S, -1).T
    r = oracle.solve_dm(H, S, ne, kT)
    D = r["D"]
    assert abs(np.trace(D @ Sf) - ne) < 1e-11
    assert abs(np.trace(D @ Sf @ D @ Sf) - np.sum(r["f"] ** 2)) < 1e-10
    assert abs(np.sum(r["f"]) - ne) < 1e-11


# --- transformation laws ------------------------------------------------------

def test_shift_and_scale_laws(oracle):
    n, kT, ne = 120, 0.03, 50.0
    H, S = inputs.sized_problem(n, cfg=51)
    Sf = np.tril(S) + np.tril(S, -1).T
    r0 = oracle.solve_dm(H, S, ne, kT)
    sigma = 0.37
    r1 = oracle.solve_dm(H + sigma * Sf, S, ne, kT)
    assert np.max(np.abs(r1["eval"] - (r0["eval"] + sigma))) < 1e-13 * 10
    assert abs(r1["mu"] - (r0["mu"] + sigma)) < 1e-12
    assert np.max(np.abs(r1["D"] - r0["D"])) < 1e-11
    assert np.max(np.abs(r1["E"] - (r0["E"] + sigma * r0["D"]))) < 1e-11
    alpha = 2.5
    r2 = oracle.solve_dm(alpha * H, S, ne, alpha * kT)
    assert np.max(np.abs(r2["D"] - r0["D"])) < 1e-11
    assert np.max(np.abs(r2["E"] - alpha * r0["E"])) < 1e-11


def test_permutation_law(oracle):
    n, kT, ne = 90, 0.02, 40.0
    H, S = inputs.sized_problem(n, cfg=52)
    Hf = np.tril(H) + np.tril(H, -1).T
    Sf = np.tril(S) + np.tril(S, -1).T
    perm = np.random.default_rng(3).permutation(n)
    r0 = oracle.solve_dm(Hf, Sf, ne, kT)
    r1 = oracle.solve_dm(Hf[np.ix_(perm, perm)], Sf[np.ix_(perm, perm)], ne, kT)
    assert np.max(np.abs(r1["D"] - r0["D"][np.ix_(perm, perm)])) < 1e-11


def test_block_diagonal_union_equals_blocks(oracle):
    """Block-diagonal (H, S) of two problems solved whole, with a shared mu,
    equals the two blocks solved at that mu (the block structure of the
    multi-k matrices in the spin/k-point section)."""
    n1, n2, kT = 40, 30, 0.05
    H1, S1 = inputs.sized_problem(n1, cfg=61)
    H2, S2 = inputs.sized_problem(n2, cfg=62)
    sym = lambda X: np.tril(X) + np.tril(X, -1).T
    H = sl.block_diag(sym(H1), sym(H2))
    S = sl.block_diag(sym(S1), sym(S2))
    ne = 35.0
    r = oracle.solve_dm(H, S, ne, kT)
    mu = r["mu"]
    for (Hb, Sb, sl_) in ((H1, S1, slice(0, n1)), (H2, S2, slice(n1, n1 + n2))):
        w, C = oracle.solve_ev(Hb, Sb)
        f = 2.0 / (1.0 + np.exp((w - mu) / kT))
        D = (C * f) @ C.T
        assert np.max(np.abs(r["D"][sl_, sl_] - D)) < 1e-11
    assert np.max(np.abs(r["D"][:n1, n1:])) < 1e-13


# --- occupations ----------------------------------------------------------------

def test_occupation_limits(oracle):
    n = 64
    H, S = inputs.sized_problem(n, cfg=71)
    Sf = np.tril(S) + np.tril(S, -1).T
    r = oracle.solve_dm(H, S, 0.0, 0.0)
    assert np.max(np.abs(r["D"])) == 0.0
    r = oracle.solve_dm(H, S, 2.0 * n, 0.0)
    assert np.max(np.abs(r["D"] - 2.0 * np.linalg.inv(Sf))) < 1e-12
    # kT -> 0 with a gap >> kT reproduces the step occupations
    w, _ = oracle.solve_ev(H, S)
    gap = w[32] - w[31]
    f_fd, _ = oracle.occupations(w, 64.0, gap / 200.0)
    f_st, _ = oracle.occupations(w, 64.0, 0.0)
    assert np.max(np.abs(f_fd - f_st)) < 1e-12


def test_bisection_electron_count_and_monotone(oracle):
    rng = np.random.default_rng(5)
    eps = np.sort(rng.uniform(-2, 2, 1000))
    for kT in (1e-3, 0.01, 0.3):
        f, mu = oracle.occupations(eps, 700.0, kT)
        assert abs(f.sum() - 700.0) < 1e-10
        assert np.all(np.diff(f) <= 1e-300)
        f_lo, _ = oracle.occupations(eps, 500.0, kT)
        assert np.all(f_lo <= f + 1e-15)


# --- steps and failure --------------------------------------------------------

def test_cholesky_failure_reports_column(oracle):
    n = 12
    S = np.eye(n, order="F")
    S[6, 6] = -1.0
    H = np.eye(n, order="F")
    with pytest.raises(oracle.OracleError) as ei:
        oracle.solve_ev(H, S)
    assert ei.value.status == 1 and ei.value.column == 7
    L, info = oracle.cholesky(np.eye(5))
    assert info == 0 and np.array_equal(L, np.eye(5))


def test_tridiagonalization_is_orthogonal_similarity(oracle):
    n = 70
    H, _ = inputs.sized_problem(n, cfg=81)
    A = np.tril(H) + np.tril(H, -1).T
    d, e, Q = oracle.tridiagonalize(A)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    assert np.max(np.abs(Q.T @ Q - np.eye(n))) < 1e-14 * n
    assert np.max(np.abs(Q @ T @ Q.T - A)) < 1e-14 * n
    w, Z = oracle.tridiag_eigh(d, e)
    assert np.max(np.abs(w - np.linalg.eigvalsh(T))) < 1e-14 * n
    assert np.max(np.abs(T @ Z - Z * w)) < 1e-14 * n
