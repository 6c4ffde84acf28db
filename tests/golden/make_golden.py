"""Write the oracle reference values for the n=4096 configurations.

Calls only the FP64 CPU oracle (oracle/) on inputs from the seeded generator
(paper_1912_13403_amd.inputs); nothing here touches the GPU path.  Stores, per
configuration: all eigenvalues, mu, band energy, sum of occupations, and the
values of D and E at 4096 seeded random positions (plus their diagonals).

    python tests/golden/make_golden.py [cfg1_n4096 cfg2sub_n4096]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1912_13403_amd import inputs  # noqa: E402


def main(names):
    for name in names:
        H, S, p = inputs.config_problem(name)
        n = p["n"]
        t0 = time.time()
        r = O.solve_dm(H, S, p["n_electrons"], p["kT"], f_max=p["f_max"])
        rng = np.random.default_rng([7, n])
        ii = rng.integers(0, n, 4096)
        jj = rng.integers(0, n, 4096)
        out = os.path.join(HERE, f"oracle_{name}.npz")
        np.savez_compressed(out, eval=r["eval"], mu=r["mu"], band_energy=r["band_energy"],
                            sum_f=float(np.sum(r["f"])), ii=ii, jj=jj,
                            D_samples=r["D"][ii, jj], E_samples=r["E"][ii, jj],
                            D_diag=np.diag(r["D"]).copy(), E_diag=np.diag(r["E"]).copy(),
                            norm1=O.norm1(H), n_electrons=p["n_electrons"], kT=p["kT"])
        print(f"{name}: n={n} oracle {time.time() - t0:.1f}s -> {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg1_n4096", "cfg2sub_n4096"])
