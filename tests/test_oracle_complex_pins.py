"""Pins for the oracle's Hermitian route (unit tasks of Eq. (13) with complex
H_k, S_k): checks against closed forms, LAPACK and exact laws, never against
the oracle itself.

The oracle solves a Hermitian pencil through its real symmetric embedding; a
wrong sign or block in that embedding, or in reading D back out of it,
conjugates or scrambles D.  The ring threaded by a flux has a complex D that a
conjugation changes, the gauge-transformed chain has a D with phases on every
element, and LAPACK's Hermitian generalized solver and the congruence law see
every block.
"""
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.optimize import brentq

from paper_1912_13403_amd import inputs


def _herm(A):
    lo = np.tril(A, -1)
    return lo + lo.conj().T + np.diag(np.real(np.diag(A)))


def _fd(eps, mu, kT, fmax):
    return fmax * 0.5 * (1.0 - np.tanh(0.5 * (eps - mu) / kT))


def _fd_mu(eps, ne, kT, fmax):
    return brentq(lambda mu: np.sum(_fd(eps, mu, kT, fmax)) - ne,
                  eps.min() - 50 * kT - 1, eps.max() + 50 * kT + 1, xtol=1e-15, rtol=1e-15)


def _ring_exact(n, phi, t=-1.0):
    """Eigenpairs of the flux ring: u_k(j) = e^{i theta_k j}/sqrt(n),
    eps_k = 2 t cos(theta_k - phi), theta_k = 2 pi k / n."""
    th = 2.0 * np.pi * np.arange(n) / n
    eps = 2.0 * t * np.cos(th - phi)
    U = np.exp(1j * np.outer(np.arange(n), th)) / np.sqrt(n)
    o = np.argsort(eps, kind="stable")
    return eps[o], U[:, o]


@pytest.mark.parametrize("n,phi,ne", [(12, 0.37, 5), (31, 1.1, 9), (64, -0.23, 30)])
def test_flux_ring_zero_temperature_closed_form(oracle, n, phi, ne):
    H, S = inputs.ring_flux(n, phi)
    r = oracle.solve_dm_complex(H, S, ne, 0.0, f_max=1.0)
    eps, U = _ring_exact(n, phi)
    assert np.max(np.abs(r["eval"] - eps)) < 1e-13
    D = U[:, :ne] @ U[:, :ne].conj().T
    assert np.max(np.abs(r["D"] - D)) < 1e-12
    # the flux makes D genuinely complex: its conjugate is a different matrix
    assert np.max(np.abs(D.imag)) > 1e-3
    assert np.max(np.abs(r["E"] - (U[:, :ne] * eps[:ne]) @ U[:, :ne].conj().T)) < 1e-12
    assert abs(r["band_energy"] - eps[:ne].sum()) < 1e-12 * n


@pytest.mark.parametrize("kT", [0.05, 0.3])
def test_flux_ring_finite_temperature_closed_form(oracle, kT):
    n, phi, ne = 40, 0.61, 13.0
    H, S = inputs.ring_flux(n, phi)
    r = oracle.solve_dm_complex(H, S, ne, kT, f_max=1.0)
    eps, U = _ring_exact(n, phi)
    mu = _fd_mu(eps, ne, kT, 1.0)
    assert abs(r["mu"] - mu) < 1e-11
    f = _fd(eps, mu, kT, 1.0)
    assert np.max(np.abs(r["D"] - (U * f) @ U.conj().T)) < 1e-11


@pytest.mark.parametrize("n,ne", [(9, 4), (40, 17)])
def test_gauge_chain_closed_form(oracle, n, ne):
    H, S, theta = inputs.gauge_chain(n, seed=n)
    r = oracle.solve_dm_complex(H, S, ne, 0.0, f_max=1.0)
    k = np.arange(1, n + 1)
    eps = -2.0 * np.cos(k * np.pi / (n + 1))
    V = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(k, k) * np.pi / (n + 1))
    o = np.argsort(eps)
    eps, V = eps[o], V[:, o]
    assert np.max(np.abs(r["eval"] - eps)) < 1e-13
    u = np.exp(1j * theta)
    D = (u[:, None] * (V[:, :ne] @ V[:, :ne].T)) * np.conj(u)[None, :]
    assert np.max(np.abs(r["D"] - D)) < 1e-12


@pytest.mark.parametrize("n,kT", [(40, 0.01), (97, 0.0)])
def test_lapack_hermitian_cross_check(oracle, n, kT):
    Hu, Hd, S = inputs.kpoint_problem(7, n=n)
    ne = 0.2 * n if kT > 0 else float(n // 5)
    w_ref, C_ref = sl.eigh(_herm(Hd), _herm(S))
    r = oracle.solve_dm_complex(Hd, S, ne, kT, f_max=1.0)
    scale = np.abs(_herm(Hd)).sum(axis=0).max()
    assert np.max(np.abs(r["eval"] - w_ref)) < 1e-12 * scale
    if kT > 0:
        f = _fd(w_ref, _fd_mu(w_ref, ne, kT, 1.0), kT, 1.0)
    else:
        f = (np.arange(n) < int(ne)).astype(float)
    D = (C_ref * f) @ C_ref.conj().T
    E = (C_ref * (f * w_ref)) @ C_ref.conj().T
    assert np.max(np.abs(r["D"] - D)) < 1e-11
    assert np.max(np.abs(r["E"] - E)) < 1e-11 * scale


def test_real_valued_input_matches_real_route(oracle):
    H, S = inputs.sized_problem(50, cfg=7)
    ne = 24.0
    rr = oracle.solve_dm(H, S, ne, 0.02, f_max=2.0)
    rc = oracle.solve_dm_complex(H.astype(np.complex128), S.astype(np.complex128), ne, 0.02,
                                 f_max=2.0)
    assert np.max(np.abs(rc["eval"] - rr["eval"])) < 1e-13
    assert np.max(np.abs(rc["D"] - rr["D"])) < 1e-12
    assert np.max(np.abs(rc["D"].imag)) < 1e-13
    assert abs(rc["band_energy"] - rr["band_energy"]) < 1e-12 * abs(rr["band_energy"])


def test_hermitian_invariants_and_congruence(oracle):
    n, ne, kT = 60, 11.0, 0.02
    Hu, Hd, S = inputs.kpoint_problem(12, n=n)
    H, Sf = _herm(Hu), _herm(S)
    r = oracle.solve_dm_complex(Hu, S, ne, kT, f_max=1.0)
    D, E = r["D"], r["E"]
    assert np.max(np.abs(D - D.conj().T)) < 1e-13
    assert abs(np.trace(D @ Sf) - ne) < 1e-12 * ne
    assert np.max(np.abs(Sf @ E - H @ D)) < 1e-12 * np.abs(H).sum(axis=0).max()
    assert abs(np.trace(D @ H).real - r["band_energy"]) < 1e-11
    # congruence (H, S) -> (X^H H X, X^H S X): same spectrum, D -> X^-1 D X^-H
    rng = np.random.default_rng([5, 1912, 13403])
    X = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    r2 = oracle.solve_dm_complex(X.conj().T @ H @ X, X.conj().T @ Sf @ X, ne, kT, f_max=1.0)
    Xi = np.linalg.inv(X)
    assert np.max(np.abs(r2["eval"] - r["eval"])) < 1e-12
    assert np.max(np.abs(r2["D"] - Xi @ D @ Xi.conj().T)) < 1e-10


def test_zero_temperature_idempotency_spin_channel(oracle):
    n, ne = 48, 10.0
    Hu, Hd, S = inputs.kpoint_problem(20, n=n)
    r = oracle.solve_dm_complex(Hu, S, ne, 0.0, f_max=1.0)
    D, Sf = r["D"], _herm(S)
    assert np.max(np.abs(D @ Sf @ D - D)) < 1e-12
    assert abs(np.trace(D @ Sf).real - ne) < 1e-12 * ne
