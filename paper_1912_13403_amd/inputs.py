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
