"""Parity at the benchmark configurations.

n = 4096 (the small configuration recipe with decay 64, and the n = 16384
recipe drawn at n = 4096): the oracle runs on the host in this session and
the GPU result is compared with it element by element: every eigenvalue,
mu, the band energy and EVERY entry of D and E.  The same sizes run the
eigenpair solve (all vectors and the lowest n_states), checked by the
residual, C^T S C = I and the eigenvalues against the oracle.  The stored
oracle values (tests/golden, written by make_golden.py from the oracle
alone) are checked against the live oracle run too.

The largest k-point task of the batched recipe (n = 2822, complex): the
single Hermitian solve against the oracle's Hermitian route, every entry of
D and E, in the FP64 form and in the refined form.

n = 16384: the oracle cannot run at this size.  The spectrum is pinned by
Sylvester inertia counts (an LDL^T of H - sigma S on the host for shifts
between GPU eigenvalues near mu and in both halves of the spectrum: exactly
k eigenvalues must lie below the k-th shift), and D, E by properties that
hold at any size: Tr(D S) = N_e, S E = H D on sampled rows, symmetry, and
the band energy Tr(D H) = sum f eps.

Tolerances: |d eps| <= 1e-10 ||H||_1, residual <= 1e-12, ||dD||_max <= 1e-9,
||dE||_max <= 1e-9 max(1, ||H||_1), |d mu| <= 1e-10 ||H||_1."""
import os

import numpy as np
import pytest

from paper_1912_13403_amd import inputs
from tests.inertia import negative_count

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda", 0)


@pytest.fixture(scope="module")
def h(torch_dev):
    from paper_1912_13403_amd import hsdm
    with hsdm.Handle(0) as handle:
        yield handle


def _oracle_cfg(oracle, oracle_run, name):
    H, S, p = inputs.config_problem(name)
    ref = oracle_run(name, lambda: oracle.solve_dm(H, S, p["n_electrons"], p["kT"],
                                                   f_max=p["f_max"]))
    return H, S, p, ref


@pytest.mark.parametrize("name", ["cfg1_n4096", "cfg2sub_n4096"])
def test_n4096_every_entry_against_oracle(oracle, oracle_run, torch_dev, h, name):
    torch, dev = torch_dev
    H, S, p, ref = _oracle_cfg(oracle, oracle_run, name)
    print(f"[cfg] {name}: GPU solve", flush=True)
    h.hsdm_reinit()
    out = h.hsdm_solve_dm_real(torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev),
                               p["n_electrons"], p["kT"])
    scale = oracle.norm1(H)
    w = out["eval"].cpu().numpy()
    assert np.max(np.abs(w - ref["eval"])) <= 1e-10 * scale
    assert abs(out["mu"] - ref["mu"]) <= 1e-10 * scale
    assert abs(out["band_energy"] - ref["band_energy"]) <= 1e-10 * scale * p["n_electrons"]
    D = out["D"].cpu().numpy()
    E = out["E"].cpu().numpy()
    dD = np.abs(D - ref["D"])
    dE = np.abs(E - ref["E"])
    i, j = np.unravel_index(int(np.argmax(dD)), dD.shape)
    print(f"[cfg] {name}: max|dD| {dD[i, j]:.3e} at ({i}, {j}), max|dE| {dE.max():.3e}",
          flush=True)
    assert dD.max() <= 1e-9
    assert dE.max() <= 1e-9 * max(1.0, scale)
    # the stored values came from the same oracle
    g = np.load(os.path.join(GOLDEN, f"oracle_{name}.npz"))
    assert np.max(np.abs(g["eval"] - ref["eval"])) <= 1e-12 * scale
    assert np.max(np.abs(g["D_samples"] - ref["D"][g["ii"], g["jj"]])) <= 1e-12


@pytest.mark.parametrize("n_states", [0, 1534])
def test_solve_ev_n4096(oracle, oracle_run, torch_dev, h, n_states):
    """Eigenpairs at n = 4096: all vectors, and the lowest 1534 (the occupied
    count of this configuration) through HSDM_KEY_N_STATES."""
    from paper_1912_13403_amd import hsdm
    torch, dev = torch_dev
    H, S, p, ref = _oracle_cfg(oracle, oracle_run, "cfg1_n4096")
    n = p["n"]
    Hd, Sd = torch.from_numpy(H).to(dev), torch.from_numpy(S).to(dev)
    h.hsdm_set_int(hsdm.HSDM_KEY_N_STATES, n_states)
    try:
        w, C = h.hsdm_solve_ev_real(Hd, Sd)
    finally:
        h.hsdm_set_int(hsdm.HSDM_KEY_N_STATES, 0)
    m = n_states if n_states else n
    assert tuple(C.shape) == (n, m)
    scale = oracle.norm1(H)
    assert np.max(np.abs(w.cpu().numpy() - ref["eval"])) <= 1e-10 * scale
    res = Hd @ C - (Sd @ C) * w[:m]
    r = torch.max(torch.sum(torch.abs(res), dim=0)).item() / (n * scale)
    orth = torch.max(torch.abs(C.T @ (Sd @ C) - torch.eye(m, dtype=torch.float64, device=dev)))
    print(f"[ev] n_states={n_states}: residual {r:.3e}, orthogonality {orth.item():.3e}",
          flush=True)
    assert r <= 1e-12
    assert orth.item() <= 1e-12 * n
    # the projector onto the formed vectors equals the oracle's (clusters
    # inside the set may rotate; the set's span may not)
    if n_states:
        Cr = torch.from_numpy(ref["C"][:, :m]).to(dev)
        P = C @ C.T
        Pr = Cr @ Cr.T
        assert torch.max(torch.abs(P - Pr)).item() <= 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_largest_kpoint_task_against_oracle(oracle, oracle_run, torch_dev, h, precision):
    """The largest unit task of the batched recipe (n_k = 2822, complex
    Hermitian, N_e = 0.2 n, kT = 0.01, one spin channel) through the single
    Hermitian solve, every entry of D and E against the oracle, in the FP64
    form and in the refined form (HSDM_KEY_PRECISION = 1)."""
    from paper_1912_13403_amd import hsdm
    torch, dev = torch_dev
    sizes = inputs.kpoint_sizes()
    k = int(np.argmax(sizes))
    n = sizes[k]
    Hu, _, S = inputs.kpoint_problem(k)
    ne, kT = 0.2 * n, 0.01
    ref = oracle_run(f"kpoint{k}_n{n}",
                     lambda: oracle.solve_dm_complex(Hu, S, ne, kT, f_max=1.0))
    h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, 1.0)
    h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, precision)
    try:
        h.hsdm_reinit()
        out = h.hsdm_solve_dm_complex(torch.from_numpy(Hu).to(dev), torch.from_numpy(S).to(dev),
                                      ne, kT)
        steps = len(h.refine_history()) if precision else 0
    finally:
        h.hsdm_set_real(hsdm.HSDM_KEY_FMAX, 2.0)
        h.hsdm_set_int(hsdm.HSDM_KEY_PRECISION, 0)
    if precision:
        assert 1 <= steps <= 8
    scale = float(np.abs(Hu).sum(axis=0).max())
    assert np.max(np.abs(out["eval"].cpu().numpy() - ref["eval"])) <= 1e-10 * scale
    assert abs(out["mu"] - ref["mu"]) <= 1e-10 * scale
    assert abs(out["band_energy"] - ref["band_energy"]) <= 1e-10 * scale * ne
    dD = np.abs(out["D"].cpu().numpy() - ref["D"]).max()
    dE = np.abs(out["E"].cpu().numpy() - ref["E"]).max()
    print(f"[kpoint] n={n} precision={precision}: max|dD| {dD:.3e}, max|dE| {dE:.3e}",
          flush=True)
    assert dD <= 1e-9
    assert dE <= 1e-9 * max(1.0, scale)


def _shift_index(w, target, window=64):
    """Index k near `target` whose gap w[k] - w[k-1] is the widest within
    the window: the shift (w[k-1] + w[k]) / 2 then has exactly k eigenvalues
    below it with the largest margin."""
    lo = max(1, target - window)
    hi = min(len(w) - 1, target + window)
    gaps = w[lo:hi + 1] - w[lo - 1:hi]
    return lo + int(np.argmax(gaps))


def test_n16384_inertia_and_properties(torch_dev, h):
    torch, dev = torch_dev
    name = "cfg2_n16384"

    def gram(B):
        Bt = torch.from_numpy(B).to(dev)
        G = (Bt @ Bt.T).cpu().numpy()
        del Bt
        return G

    H, S, p = inputs.config_problem(name, gram=gram)
    Hd = torch.from_numpy(H).to(dev)
    Sd = torch.from_numpy(S).to(dev)
    h.hsdm_reinit()
    out = h.hsdm_solve_dm_real(Hd, Sd, p["n_electrons"], p["kT"])
    D, E, w = out["D"], out["E"], out["eval"]
    n, ne = p["n"], p["n_electrons"]
    wh = w.cpu().numpy()
    assert np.all(np.diff(wh) >= 0)
    # spectrum: Sylvester inertia of H - sigma S at shifts between eigenvalues
    scale = float(np.abs(H).sum(axis=0).max())
    k_mu = int(np.searchsorted(wh, out["mu"]))
    for target in (n // 4, k_mu, (3 * n) // 4):
        k = _shift_index(wh, target)
        sigma = 0.5 * (wh[k - 1] + wh[k])
        assert wh[k] - wh[k - 1] > 2e-10 * scale  # the pin resolves the tolerance
        A = H - sigma * S
        cnt = negative_count(A)
        del A
        print(f"[inertia] sigma={sigma:.12f} (between eigenvalues {k - 1}, {k}): "
              f"{cnt} negative pivots", flush=True)
        assert cnt == k
    # Tr(D S) = N_e  (S, D symmetric: Tr(DS) = sum_ij D_ij S_ij)
    trDS = torch.sum(D * Sd).item()
    assert abs(trDS - ne) <= 1e-9 * ne
    # band energy = Tr(D H)
    trDH = torch.sum(D * Hd).item()
    assert abs(trDH - out["band_energy"]) <= 1e-9 * abs(out["band_energy"])
    # S E = H D on sampled rows (E = S^-1 H D in exact arithmetic)
    rows = torch.from_numpy(np.random.default_rng(3).integers(0, n, 48)).to(dev)
    lhs = Sd[rows] @ E
    rhs = Hd[rows] @ D
    assert torch.max(torch.abs(lhs - rhs)).item() <= 1e-9
    assert torch.equal(D[rows][:, rows], D[rows][:, rows].T)
    # occupations sum to N_e from the returned eigenvalues and mu
    x = (wh - out["mu"]) / p["kT"]
    f = p["f_max"] / (1.0 + np.exp(np.clip(x, -700, 700)))
    assert abs(np.sum(f) - ne) <= 1e-9 * ne
