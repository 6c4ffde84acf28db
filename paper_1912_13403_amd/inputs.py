"""Seeded synthetic inputs for the dense H,S -> D path.

This module only draws random numbers and assembles matrices from them; it
holds none of the solver's arithmetic.  Both the GPU path (through the tests
and the benchmark) and the CPU oracle receive the very same arrays from here.

The paper's benchmark matrices (FHI-aims, SIESTA and DFTB+ Hamiltonians of the
benchmark section, Tables 2-4) are not available; these generators stand in
for them.  The exp(-|i-j|/l) envelope gives H the locality of a localized
basis, and S = I + a B B^T / n is a well-conditioned SPD overlap.

Recipe of a real symmetric problem (seed list [cfg, 1912, 13403]):
  B ~ N(0,1) n x n;  S = I + s_pert * B B^T / n  (symmetrized);
  G ~ N(0, 0.1^2) n x n;  H_ij = G_ij exp(-|i-j|/decay) for i < j, mirrored;
  H_ii = -1 + U(0, 2).
All arrays are float64, Fortran (column-major) order.
"""
from __future__ import annotations

import numpy as np

SEED_TAIL = (1912, 13403)

# name -> (n, decay, s_pert, n_electrons, kT, f_max, seed cfg index)
CONFIGS = {
    "cfg0_n512": dict(n=512, decay=32.0, s_pert=0.1, n_electrons=256.0, kT=0.0, f_max=2.0, cfg=0),
    "cfg1_n4096": dict(n=4096, decay=64.0, s_pert=0.1, n_electrons=2048.0, kT=0.01, f_max=2.0, cfg=1),
    "cfg2_n16384": dict(n=16384, decay=128.0, s_pert=0.05, n_electrons=8192.0, kT=0.005, f_max=2.0,
                        cfg=2),
    # the n=4096 stand-in drawn with the n=16384 problem's parameters
    "cfg2sub_n4096": dict(n=4096, decay=128.0, s_pert=0.05, n_electrons=2048.0, kT=0.005,
                          f_max=2.0, cfg=2),
}


def real_problem(n, decay, s_pert, cfg=0, gram=None, g_std=0.1):
    """(H, S) of the recipe above.  ``gram(B)`` may replace numpy's B @ B.T
    (the benchmark uses a device matmul for the n=16384 Gram product)."""
    rng = np.random.default_rng([int(cfg), *SEED_TAIL])
    B = rng.standard_normal((n, n))
    BBt = gram(B) if gram is not None else B @ B.T
    del B
    S = BBt
    S *= s_pert / n
    S = 0.5 * (S + S.T)
    S[np.diag_indices(n)] += 1.0
    G = rng.normal(0.0, g_std, (n, n))
    i = np.arange(n)
    env = np.exp(-np.abs(i[:, None] - i[None, :]) / float(decay))
    U = np.triu(G * env, 1)
    del G, env
    H = U + U.T
    del U
    H[np.diag_indices(n)] = -1.0 + 2.0 * rng.random(n)
    return np.asfortranarray(H), np.asfortranarray(S)


def config_problem(name, gram=None):
    """(H, S, params) of a named configuration."""
    p = dict(CONFIGS[name])
    H, S = real_problem(p["n"], p["decay"], p["s_pert"], cfg=p["cfg"], gram=gram)
    return H, S, p


def sized_problem(n, cfg=0, decay=32.0, s_pert=0.1):
    """A problem of any size with the small configuration's recipe; the
    electron count is n/2 (half filling of f_max = 2 states)."""
    H, S = real_problem(n, decay, s_pert, cfg=cfg)
    return H, S


def chain(n, t=-1.0):
    """Open tight-binding chain H = t * tridiag(1, 0, 1), S = I."""
    H = np.zeros((n, n), order="F")
    idx = np.arange(n - 1)
    H[idx + 1, idx] = t
    H[idx, idx + 1] = t
    return H, np.eye(n, order="F")


def ring(n, t=-1.0):
    """Periodic ring (uniform hopping t, no flux), S = I."""
    H, S = chain(n, t)
    if n > 2:
        H[0, n - 1] = t
        H[n - 1, 0] = t
    return H, S


# ---- complex Hermitian problems (periodic, spin-polarized systems) ---------------
#
# One unit task of Eq. (13): H_k^a C = S_k C eps for k-point k and spin a.
# Recipe of the batched periodic system (seed list [3, 1912, 13403, kindex]):
#   k on a Gamma-centred 4 x 4 x 2 grid (fractions of the reciprocal vectors),
#   lattice vectors R in {x, y, z};  size n_k ~ U{600..3000} per k-point;
#   H0 real symmetric as in the real recipe (decay 32);  three banded complex
#   H_R with Re, Im ~ N(0, 0.05^2) * exp(-|i-j|/32), zero beyond |i-j| > 64;
#   H_k = H0 + sum_R (e^{i k.R} H_R + e^{-i k.R} H_R^H) / 2  (Hermitian);
#   spin a = +-1:  H_k^a = H_k + a * 0.05 diag(m),  m_i ~ U(0, 1);
#   S0 = I + 0.1 B B^T / n;  S_R banded complex, scaled to ||S_R||_1 = ||S_R||_inf
#   = 0.1 so that lambda_min(S_k) >= 0.7;  S_k formed like H_k.
# The electron count of the whole system is 0.4 * sum_k n_k with f_max = 1,
# counted over all k-points and both spins; kT = 0.01.
# Arrays are complex128, Fortran order.

KGRID = (4, 4, 2)
NKPT = KGRID[0] * KGRID[1] * KGRID[2]


def kpoints():
    """The 32 k-points of the grid as fractions (kx, ky, kz) of the reciprocal vectors."""
    return [(i / KGRID[0], j / KGRID[1], l / KGRID[2])
            for i in range(KGRID[0]) for j in range(KGRID[1]) for l in range(KGRID[2])]


def kpoint_sizes(lo=600, hi=3000):
    rng = np.random.default_rng([3, *SEED_TAIL])
    return [int(v) for v in rng.integers(lo, hi + 1, NKPT)]


def _banded_complex(rng, n, std, decay, width):
    """Complex n x n matrix with Re, Im ~ N(0, std^2) * exp(-|i-j|/decay) on the
    diagonals |i-j| <= width (drawn diagonal by diagonal, -width first) and
    zero elsewhere."""
    A = np.zeros((n, n), dtype=np.complex128)
    for d in range(-width, width + 1):
        m = n - abs(d)
        if m <= 0:
            continue
        v = (rng.normal(0.0, std, m) + 1j * rng.normal(0.0, std, m)) * np.exp(-abs(d) / decay)
        i = np.arange(m)
        if d >= 0:
            A[i + d, i] = v
        else:
            A[i, i - d] = v
    return A


def kpoint_problem(kindex, n=None, gram=None):
    """(H_up, H_down, S) of k-point `kindex` of the recipe above (size n_k unless
    `n` is given, which keeps the recipe at another size).  ``gram(B)`` may
    replace numpy's B @ B.T."""
    k = kpoints()[kindex]
    n = kpoint_sizes()[kindex] if n is None else int(n)
    rng = np.random.default_rng([3, *SEED_TAIL, int(kindex)])
    B = rng.standard_normal((n, n))
    S0 = 0.1 * (gram(B) if gram is not None else B @ B.T) / n
    S0 = 0.5 * (S0 + S0.T) + np.eye(n)
    del B
    G = rng.normal(0.0, 0.1, (n, n))
    i = np.arange(n)
    U = np.triu(G * np.exp(-np.abs(i[:, None] - i[None, :]) / 32.0), 1)
    H0 = U + U.T
    H0[np.diag_indices(n)] = -1.0 + 2.0 * rng.random(n)
    del G, U
    H = H0.astype(np.complex128)
    S = S0.astype(np.complex128)
    for axis in range(3):
        ph = np.exp(2j * np.pi * k[axis])
        HR = _banded_complex(rng, n, 0.05, 32.0, 64)
        H += 0.5 * (ph * HR + np.conj(ph) * HR.conj().T)
        SR = _banded_complex(rng, n, 1.0, 8.0, 16)
        SR *= 0.1 / max(np.abs(SR).sum(axis=0).max(), np.abs(SR).sum(axis=1).max())
        S += 0.5 * (ph * SR + np.conj(ph) * SR.conj().T)
    m = rng.random(n)
    Hu = H + np.diag(0.05 * m)
    Hd = H - np.diag(0.05 * m)
    return np.asfortranarray(Hu), np.asfortranarray(Hd), np.asfortranarray(S)


def ring_flux(n, phi, t=-1.0):
    """Periodic ring threaded by a uniform flux: every bond j -> j+1 (mod n)
    carries the phase e^{i phi}, i.e. H[j+1, j] = t e^{i phi}; S = I."""
    H = np.zeros((n, n), dtype=np.complex128, order="F")
    for j in range(n):
        H[(j + 1) % n, j] += t * np.exp(1j * phi)
        H[j, (j + 1) % n] += t * np.exp(-1j * phi)
    return H, np.eye(n, dtype=np.complex128, order="F")


def gauge_chain(n, seed=0, t=-1.0):
    """Open chain in a random gauge: H = U H_chain U^H with U = diag(e^{i theta_j}),
    S = I.  Returns (H, S, theta)."""
    theta = np.random.default_rng([int(seed), *SEED_TAIL]).uniform(-np.pi, np.pi, n)
    Hc, _ = chain(n, t)
    u = np.exp(1j * theta)
    H = (u[:, None] * Hc) * np.conj(u)[None, :]
    return np.asfortranarray(H), np.eye(n, dtype=np.complex128, order="F"), theta


# ---- a stream of requests (serving) -----------------------------------------------
#
# Recipe (seed list [4, 1912, 13403]): Poisson arrivals at `rate` per second;
# sizes log-uniform on [lo, hi]; 60 % real problems (the real recipe, decay 32,
# S perturbation 0.1; N_e = n/2, kT = 0.01, f_max = 2), 40 % Hermitian (one
# k-point and spin of the k-point recipe at that size; N_e = 0.2 n, kT = 0.01,
# f_max = 1); 30 % SCF repeats of an earlier request of the same type: the same
# S (shared, not copied) and H + 1e-3 Z with Z symmetric (Hermitian) standard
# normal.  Problems are drawn by `make(spec)` so that a caller can draw them
# lazily; `gram(B)` may replace numpy's B @ B.T for the real recipe.


def request_specs(count, rate=40.0, lo=256, hi=8192, seed=0):
    """Arrival times and shapes of `count` requests (no matrices)."""
    rng = np.random.default_rng([4, *SEED_TAIL, int(seed)])
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    specs = []
    for i in range(count):
        u = rng.random()
        rep = None
        if i > 0 and rng.random() < 0.3:
            rep = int(rng.integers(0, i))
        if rep is not None:
            base = specs[rep]["base"]
            specs.append(dict(rid=i, arrival=float(t[i]), cplx=specs[base]["cplx"],
                              n=specs[base]["n"], base=base, repeat=True))
        else:
            n = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
            specs.append(dict(rid=i, arrival=float(t[i]), cplx=bool(u < 0.4), n=n, base=i,
                              repeat=False))
    for s in specs:
        s["n_electrons"] = 0.2 * s["n"] if s["cplx"] else 0.5 * s["n"]
        s["kT"] = 0.01
        s["f_max"] = 1.0 if s["cplx"] else 2.0
    return specs


def request_problem(spec, base_problem=None, gram=None):
    """(H, S) of a request.  A repeat passes its base request's (H, S) as
    base_problem and receives (H + 1e-3 Z, the same S object)."""
    rid, n = spec["rid"], spec["n"]
    if spec["repeat"]:
        H0, S0 = base_problem
        rng = np.random.default_rng([4, *SEED_TAIL, 7, int(rid)])
        Z = rng.standard_normal((n, n))
        if spec["cplx"]:
            Z = Z + 1j * rng.standard_normal((n, n))
            Z = np.tril(Z, -1) + np.tril(Z, -1).conj().T + np.diag(np.real(np.diag(Z)))
        else:
            Z = np.tril(Z) + np.tril(Z, -1).T
        return np.asfortranarray(H0 + 1e-3 * Z), S0
    if spec["cplx"]:
        Hu, _, S = kpoint_problem(rid % NKPT, n=n, gram=gram)
        return Hu, S
    return real_problem(n, 32.0, 0.1, cfg=1000 + rid, gram=gram)


# ---- the request recipe drawn on the device (serving benchmark) -------------------
#
# The serving benchmark replays thousands of requests; drawing each one's
# matrices on the host (an n^3 Gram product per overlap matrix) would take
# longer than the replay.  request_problem_device draws the same recipe with
# torch on the GPU, from a per-request seed (its own random streams, not the
# host generator's numbers), as device tensors in column-major layout.  It
# holds none of the solver's arithmetic.


def _device_seed(*key):
    return int(np.random.SeedSequence([4, *SEED_TAIL, *key]).generate_state(1, dtype=np.uint64)[0]
               & ((1 << 62) - 1))


def _device_banded(torch, gen, n, std, decay, width, dev, cplx=True):
    i = torch.arange(n, device=dev)
    d = (i[:, None] - i[None, :]).abs()
    env = torch.exp(-d.double() / decay) * (d <= width)
    re = torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
    im = torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
    return torch.complex(re, im) * (std * env) if cplx else re * (std * env)


def _device_s(torch, spec, dev):
    """Overlap matrix of a (non-repeat) request, drawn on the device."""
    n, rid = spec["n"], spec["rid"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(_device_seed(rid, 0))
    B = torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
    S = (0.1 / n) * (B @ B.T)
    del B
    S = 0.5 * (S + S.T) + torch.eye(n, device=dev, dtype=torch.float64)
    if not spec["cplx"]:
        return S
    k = kpoints()[rid % NKPT]
    Sc = S.to(torch.complex128)
    del S
    for axis in range(3):
        ph = complex(np.exp(2j * np.pi * k[axis]))
        SR = _device_banded(torch, gen, n, 1.0, 8.0, 16, dev)
        SR *= 0.1 / max(SR.abs().sum(dim=0).max().item(), SR.abs().sum(dim=1).max().item())
        Sc += 0.5 * (ph * SR + np.conj(ph) * SR.conj().T)
        del SR
    return Sc


def _device_h(torch, spec, dev):
    """Hamiltonian of a (non-repeat) request, drawn on the device."""
    n, rid = spec["n"], spec["rid"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(_device_seed(rid, 1))
    i = torch.arange(n, device=dev)
    env = torch.exp(-(i[:, None] - i[None, :]).abs().double() / 32.0)
    G = 0.1 * torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
    U = torch.triu(G * env, 1)
    del G, env
    H = U + U.T
    del U
    H.diagonal().copy_(-1.0 + 2.0 * torch.rand(n, generator=gen, device=dev, dtype=torch.float64))
    if not spec["cplx"]:
        return H
    k = kpoints()[rid % NKPT]
    Hc = H.to(torch.complex128)
    del H
    for axis in range(3):
        ph = complex(np.exp(2j * np.pi * k[axis]))
        HR = _device_banded(torch, gen, n, 0.05, 32.0, 64, dev)
        Hc += 0.5 * (ph * HR + np.conj(ph) * HR.conj().T)
        del HR
    Hc.diagonal().add_(0.05 * torch.rand(n, generator=gen, device=dev, dtype=torch.float64))
    return Hc


def _colmajor_view(torch, X):
    """The same (symmetric or Hermitian) matrix as a column-major tensor:
    for a Hermitian X stored row-major, its conjugate's transposed view is X."""
    if X.is_complex():
        return torch.conj_physical(X).t()
    return X.t()


def request_problem_device(spec, base_spec=None, S=None, dev=None):
    """(H, S) of a request as column-major device tensors drawn on the GPU by
    the recipe of request_problem (per-request seeds; a repeat draws its base
    request's H again and adds 1e-3 Z).  S: the base request's overlap matrix
    when it is still on the device (returned as is), else drawn."""
    import torch
    base = spec if not spec["repeat"] else base_spec
    if S is None:
        S = _colmajor_view(torch, _device_s(torch, base, dev))
    H = _device_h(torch, base, dev)
    if spec["repeat"]:
        n = spec["n"]
        gen = torch.Generator(device=dev)
        gen.manual_seed(_device_seed(spec["rid"], 2))
        Z = torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64)
        if spec["cplx"]:
            Z = torch.complex(Z, torch.randn(n, n, generator=gen, device=dev, dtype=torch.float64))
            Z = (torch.tril(Z, -1) + torch.tril(Z, -1).conj().T
                 + torch.diag(torch.diagonal(Z).real).to(Z.dtype))
        else:
            Z = torch.tril(Z) + torch.tril(Z, -1).T
        H = H + 1e-3 * Z
        del Z
    return _colmajor_view(torch, H), S
