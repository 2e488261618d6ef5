"""Write tests/golden/d4_n32_uncapped_100steps.npz with the CPU oracle only.

Workload: d = 4 Fourier modes, n = 32 points on [-4, 4], nu = 0.05, Gaussian
initial condition from paper_2403_04946_amd.inputs.ic_params(4, seed=0),
plain classical RK4 on the full grid (oracle.fullgrid.rk4_step, no
truncation) with dt = 1e-3 for 100 steps.  The final 32^4 field is stored
compressed as its TT-SVD (oracle.fullgrid.tt_svd) at relative tolerance
STORE_EPS; the stored TT differs from the oracle's array by at most that
tolerance times its norm (the TT-SVD error bound), far below the 1e-10
parity target.  The exact norm of the oracle's array and the store error
are kept with it.

Run: python tests/golden/make_d4_n32_uncapped_golden.py   (about 3 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fullgrid, galerkin  # noqa: E402
from paper_2403_04946_amd import inputs  # noqa: E402

D, N, L, NU, DT, STEPS, SEED = 4, 32, 4.0, 0.05, 1e-3, 100, 0
STORE_EPS = 1e-13


def main():
    prob = fullgrid.Problem(galerkin.coefficient_B(D), galerkin.coefficient_D(D), NU, N, L)
    mu, sig = inputs.ic_params(D, SEED)
    f = fullgrid.gaussian_ic(mu, sig, N, L)
    for s in range(STEPS):
        f = fullgrid.rk4_step(f, DT, prob.apply)
        if (s + 1) % 10 == 0:
            print(f"step {s + 1}: norm {np.linalg.norm(f):.12e}", flush=True)
    cores, _ = fullgrid.tt_svd(f, STORE_EPS, None)
    store_err = np.linalg.norm(fullgrid.tt_to_full(cores) - f) / np.linalg.norm(f)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "d4_n32_uncapped_100steps.npz")
    arrays = {f"core{k}": c for k, c in enumerate(cores)}
    np.savez_compressed(out, mu=mu, sigma=sig, norm=np.linalg.norm(f), store_err=store_err, **arrays)
    print("wrote", out, "ranks", [c.shape[2] for c in cores], "store error", store_err)


if __name__ == "__main__":
    main()
