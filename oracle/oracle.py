"""Python access to the FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE ONLY.  This module (and the C file it loads) may be
imported, called or executed only by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``.  The product library never uses
it, and it shares no code with the GPU path: it depends on numpy and ctypes
only, and the inputs it is given come from the seeded generators in
``paper_1912_13403_amd.inputs`` (a module that holds none of the method's
arithmetic).

Functions mirror the steps in ``oracle.c``; every matrix crosses the boundary
as a Fortran-ordered (column-major) float64 array.  Citations are to the ELSI
2.x paper (arXiv:1912.13403): Eq. (3) problem, Eq. (4) density matrix,
Eq. (17) energy-weighted density matrix, Sec. 2.6 occupations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build(force: bool = True) -> str:
    """Compile oracle.c into liborc.so with gcc (-O3, AVX2 code for any x86-64-v3
    host, OpenMP, IEEE FP64 without contraction into FMA)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               "-ffp-contract=off", "-o", _LIB, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_cholesky.argtypes = [ctypes.c_int, _dp, _dp]
        lib.orc_standard_form.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        lib.orc_tridiagonalize.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
        lib.orc_tql.argtypes = [ctypes.c_int, _dp, _dp, _dp]
        lib.orc_sort_pairs.argtypes = [ctypes.c_int, _dp, _dp]
        lib.orc_back_transform.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp]
        lib.orc_occupations.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.orc_density.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        lib.orc_band_energy.argtypes = [ctypes.c_int, _dp, _dp]
        lib.orc_band_energy.restype = ctypes.c_double
        lib.orc_solve_ev.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _ip]
        lib.orc_solve_dm.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, _dp, _dp, _dp, _dp, _dp,
                                     _dp, _dp, _ip]
        lib.orc_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _f(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


class OracleError(RuntimeError):
    def __init__(self, status, column=0):
        self.status = status
        self.column = column
        super().__init__(f"oracle status {status} (column {column})")


def num_threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().orc_num_threads())


def norm1(H) -> float:
    """||H||_1 (max column sum of |H|) of the symmetric matrix whose lower
    triangle is H's; the norm in which tolerances are stated."""
    L = np.tril(np.asarray(H, dtype=np.float64))
    full = L + np.tril(L, -1).T
    return float(np.abs(full).sum(axis=0).max())


def cholesky(S):
    S = _f(S)
    n = S.shape[0]
    L = np.zeros((n, n), order="F")
    info = _load().orc_cholesky(n, _p(S), _p(L))
    return L, int(info)


def standard_form(H, L):
    H, L = _f(H), _f(L)
    n = H.shape[0]
    A = np.zeros((n, n), order="F")
    _load().orc_standard_form(n, _p(H), _p(L), _p(A))
    return A


def tridiagonalize(A):
    A = _f(A)
    n = A.shape[0]
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 1))
    Q = np.zeros((n, n), order="F")
    _load().orc_tridiagonalize(n, _p(A), _p(d), _p(e), _p(Q))
    return d, e[: max(n - 1, 0)], Q


def tql(d, e, Z=None):
    """Eigenvalues (unsorted) and rotated Z of the tridiagonal (d, e)."""
    d = np.array(d, dtype=np.float64)
    n = d.shape[0]
    e = np.zeros(max(n, 1)) if len(e) == 0 else np.concatenate([np.asarray(e, np.float64), [0.0]])
    Z = np.eye(n, order="F") if Z is None else np.array(Z, dtype=np.float64, order="F")
    st = _load().orc_tql(n, _p(d), _p(e), _p(Z))
    if st:
        raise OracleError(st)
    return d, Z


def sort_pairs(d, Z):
    d = np.array(d, dtype=np.float64)
    Z = np.array(Z, dtype=np.float64, order="F")
    _load().orc_sort_pairs(d.shape[0], _p(d), _p(Z))
    return d, Z


def tridiag_eigh(d, e):
    """All eigenpairs of a symmetric tridiagonal, ascending."""
    w, Z = tql(d, e)
    return sort_pairs(w, Z)


def back_transform(L, Y):
    L, Y = _f(L), _f(Y)
    n, m = Y.shape
    C = np.zeros((n, m), order="F")
    _load().orc_back_transform(n, m, _p(L), _p(Y), _p(C))
    return C


def occupations(eps, n_electrons, kT, f_max=2.0, deg_tol=0.0):
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    n = eps.shape[0]
    f = np.zeros(n)
    mu = np.zeros(1)
    st = _load().orc_occupations(n, _p(eps), float(f_max), float(n_electrons), float(kT),
                                 float(deg_tol), _p(f), _p(mu))
    if st:
        raise OracleError(st)
    return f, float(mu[0])


def density(C, f, eps, with_e=True):
    C = _f(C)
    n, m = C.shape
    f = np.ascontiguousarray(f, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    D = np.zeros((n, n), order="F")
    E = np.zeros((n, n), order="F") if with_e else None
    _load().orc_density(n, m, _p(C), _p(f), _p(eps), _p(D), _p(E) if with_e else None)
    return D, E


def band_energy(f, eps):
    f = np.ascontiguousarray(f, dtype=np.float64)
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    return float(_load().orc_band_energy(f.shape[0], _p(f), _p(eps)))


def solve_ev(H, S):
    """All eigenpairs of the pencil (H, S), Eq. (3): (eval ascending, C)."""
    H, S = _f(H), _f(S)
    n = H.shape[0]
    w = np.zeros(n)
    C = np.zeros((n, n), order="F")
    col = ctypes.c_int(0)
    st = _load().orc_solve_ev(n, _p(H), _p(S), _p(w), _p(C), ctypes.byref(col))
    if st:
        raise OracleError(st, col.value)
    return w, C


def default_deg_tol(H) -> float:
    """Degeneracy window for kT = 0 sharing: 1e-12 * ||H||_1."""
    return 1e-12 * norm1(H)


def solve_dm(H, S, n_electrons, kT, f_max=2.0, deg_tol=None):
    """Density matrix route: returns dict(eval, C, f, D, E, mu, band_energy)."""
    H, S = _f(H), _f(S)
    n = H.shape[0]
    if deg_tol is None:
        deg_tol = default_deg_tol(H)
    w = np.zeros(n)
    C = np.zeros((n, n), order="F")
    f = np.zeros(n)
    D = np.zeros((n, n), order="F")
    E = np.zeros((n, n), order="F")
    mu = ctypes.c_double(0.0)
    eb = ctypes.c_double(0.0)
    col = ctypes.c_int(0)
    st = _load().orc_solve_dm(n, _p(H), _p(S), float(f_max), float(n_electrons), float(kT),
                              float(deg_tol), _p(w), _p(C), _p(f), _p(D), _p(E),
                              ctypes.byref(mu), ctypes.byref(eb), ctypes.byref(col))
    if st:
        raise OracleError(st, col.value)
    return dict(eval=w, C=C, f=f, D=D, E=E, mu=mu.value, band_energy=eb.value)


# ---- complex Hermitian problems (Eq. (13) unit tasks) ----------------------------
#
# A Hermitian pencil (H, S) is solved through its real symmetric embedding
# [[Re A, -Im A], [Im A, Re A]] (2n x 2n).  The embedded pencil has the same
# eigenvalues, each twice: u = x + i y with H u = eps S u maps to the two real
# eigenvectors [x; y] and [-y; x].  With one occupation per real eigenpair and
# twice the electron count, the real density matrix D_R holds
# D = D_R[:n, :n] + i D_R[n:, :n], because the pair contributes
# (x x^T + y y^T) = Re(u u^H) to the upper left block and (y x^T - x y^T) =
# Im(u u^H) to the lower left block.  No complex arithmetic is needed, so this
# route shares nothing with a complex eigensolver.  Parity pins: closed forms
# of a ring threaded by a flux and of a chain in a random gauge, LAPACK's
# Hermitian generalized solver, the congruence law and the density-matrix
# invariants (tests/test_oracle_pins.py).


def hermitian_embedding(A):
    """[[Re A, -Im A], [Im A, Re A]] of the Hermitian matrix whose lower
    triangle A holds (the imaginary parts of the diagonal are ignored)."""
    A = np.asarray(A)
    n = A.shape[0]
    lo = np.tril(A, -1)
    Ah = lo + lo.conj().T + np.diag(np.real(np.diag(A)))
    R = np.zeros((2 * n, 2 * n), order="F")
    R[:n, :n] = Ah.real
    R[n:, n:] = Ah.real
    R[n:, :n] = Ah.imag
    R[:n, n:] = -Ah.imag
    return R


def solve_dm_complex(H, S, n_electrons, kT, f_max=1.0, deg_tol=None):
    """Density matrix route for a Hermitian pencil (Eqs. (3), (4), (17)):
    dict(eval, f, D, E, mu, band_energy) with complex D and E."""
    n = np.asarray(H).shape[0]
    R, SR = hermitian_embedding(H), hermitian_embedding(S)
    if deg_tol is None:
        deg_tol = default_deg_tol(R)
    r = solve_dm(R, SR, 2.0 * n_electrons, kT, f_max=f_max, deg_tol=deg_tol)
    D = r["D"][:n, :n] + 1j * r["D"][n:, :n]
    E = r["E"][:n, :n] + 1j * r["E"][n:, :n]
    ev = 0.5 * (r["eval"][0::2] + r["eval"][1::2])
    f = 0.5 * (r["f"][0::2] + r["f"][1::2])
    return dict(eval=ev, f=f, D=D, E=E, mu=r["mu"], band_energy=0.5 * r["band_energy"])


# ---- unit tasks sharing one chemical potential (Eq. (16)) -----------------------
#
# The eigenvalues of all k-point x spin tasks are coupled by
# sum_p w_p sum_l f_pl = N_e.  kT > 0: bisection on that monotone sum, to
# adjacent doubles, with the same overflow-safe Fermi-Dirac form as the C
# oracle.  kT = 0: all (eps, w) pairs sorted by eps are filled in order; the
# Fermi level is the first at which the weighted count f_max sum w reaches N_e,
# and the states of all tasks within deg_tol of it share what is left equally
# per unit weight (the kT -> 0+ limit).


def _fermi(x, f_max):
    out = np.empty_like(x)
    pos = x >= 0
    t = np.exp(-x[pos])
    out[pos] = f_max * t / (1.0 + t)
    out[~pos] = f_max / (1.0 + np.exp(x[~pos]))
    return out


def occupations_shared(eps_list, weights, n_electrons, kT, f_max=2.0, deg_tol=0.0):
    """Occupations of several tasks with one mu: (list of f, mu)."""
    eps_all = np.concatenate([np.asarray(e, dtype=np.float64) for e in eps_list])
    w_all = np.concatenate([np.full(len(e), float(w)) for e, w in zip(eps_list, weights)])
    if kT > 0.0:
        lo, hi = eps_all.min() - 50.0 * kT - 1.0, eps_all.max() + 50.0 * kT + 1.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if mid <= lo or mid >= hi:
                break
            if np.sum(w_all * _fermi((eps_all - mid) / kT, f_max)) < n_electrons:
                lo = mid
            else:
                hi = mid
        mu = 0.5 * (lo + hi)
        return [_fermi((np.asarray(e) - mu) / kT, f_max) for e in eps_list], mu
    if n_electrons <= 0.0:
        return [np.zeros(len(e)) for e in eps_list], float(eps_all.min())
    order = np.argsort(eps_all, kind="stable")
    cum = f_max * np.cumsum(w_all[order])
    i = int(np.argmax(cum >= n_electrons - 1e-12 * f_max))
    ef = eps_all[order[i]]
    below = eps_all < ef - deg_tol
    group = (eps_all >= ef - deg_tol) & (eps_all <= ef + deg_tol)
    share = min((n_electrons - f_max * w_all[below].sum()) / w_all[group].sum(), f_max)
    above = eps_all[eps_all > ef + deg_tol]
    if share < f_max * (1.0 - 1e-15) or above.size == 0:
        mu = float(ef)
    else:
        mu = 0.5 * (eps_all[eps_all <= ef + deg_tol].max() + above.min())
    fl = []
    for e in eps_list:
        e = np.asarray(e)
        fl.append(np.where(e < ef - deg_tol, f_max, np.where(e <= ef + deg_tol, share, 0.0)))
    return fl, mu


def solve_dm_batch(Hs, Ss, n_electrons, kT, weights=None, f_max=2.0, deg_tol=None):
    """Tasks (real, or Hermitian through the embedding) with one chemical
    potential: dict(D, E, eval, f lists; mu; band_energy = sum_p w_p sum f eps)."""
    cplx = np.iscomplexobj(Hs[0])
    weights = [1.0] * len(Hs) if weights is None else list(weights)
    pencils = [(hermitian_embedding(H), hermitian_embedding(S)) if cplx else (_f(H), _f(S))
               for H, S in zip(Hs, Ss)]
    if deg_tol is None:
        deg_tol = max(default_deg_tol(R) for R, _ in pencils)
    pairs = [solve_ev(R, SR) for R, SR in pencils]
    ne = 2.0 * n_electrons if cplx else n_electrons
    fl, mu = occupations_shared([w for w, _ in pairs], weights, ne, kT, f_max, deg_tol)
    Ds, Es, evs, fs = [], [], [], []
    eb = 0.0
    for (w, C), f, wt in zip(pairs, fl, weights):
        D, E = density(C, f, w)
        eb += wt * float(np.sum(f * w))
        if cplx:
            n = C.shape[0] // 2
            D = D[:n, :n] + 1j * D[n:, :n]
            E = E[:n, :n] + 1j * E[n:, :n]
            w = 0.5 * (w[0::2] + w[1::2])
            f = 0.5 * (f[0::2] + f[1::2])
        Ds.append(D)
        Es.append(E)
        evs.append(w)
        fs.append(f)
    return dict(D=Ds, E=Es, eval=evs, f=fs, mu=mu, band_energy=(0.5 if cplx else 1.0) * eb)
