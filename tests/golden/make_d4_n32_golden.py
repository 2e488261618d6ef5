"""Write tests/golden/d4_n32_cap8_100steps.npz with the CPU oracle only.

Workload: d = 4 Fourier modes, n = 32 points on [-4, 4], nu = 0.05, Gaussian
initial condition from paper_2403_04946_amd.inputs.ic_params(4, seed=0),
RK4 step-truncation with dt = 1e-3 for 100 steps, truncation tolerance
1e-12 (relative) and rank cap 8 at every truncation point (placement as in
oracle.fullgrid.truncated_rk4_step).  The final field is stored as the
TT-SVD of the oracle's full array (its ranks are <= 8 because the last
operation of a step is the capped truncation), together with the smallest
ratio sigma_8/sigma_9 met at any truncation where sigma_9 exceeds the tolerance (a gap near 1 would
make the truncated tensor ill-determined).

Run: python tests/golden/make_d4_n32_golden.py   (about 5 minutes on 8 cores)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fullgrid, galerkin  # noqa: E402
from paper_2403_04946_amd import inputs  # noqa: E402

D, N, L, NU, DT, STEPS, EPS, CAP, SEED = 4, 32, 4.0, 0.05, 1e-3, 100, 1e-12, 8, 0


def main():
    prob = fullgrid.Problem(galerkin.coefficient_B(D), galerkin.coefficient_D(D), NU, N, L)
    mu, sig = inputs.ic_params(D, SEED)
    f = fullgrid.gaussian_ic(mu, sig, N, L)
    min_gap = [np.inf]

    def trunc(x):
        cores, sigmas = fullgrid.tt_svd(x, EPS, CAP)
        delta = EPS * np.linalg.norm(x) / np.sqrt(D - 1)
        for s in sigmas:
            # the cap decides the cut only where sigma_{CAP+1} is above the
            # tolerance; there a gap near 1 would make the result ill-determined
            if len(s) > CAP and s[CAP] > delta:
                min_gap[0] = min(min_gap[0], s[CAP - 1] / s[CAP])
        return fullgrid.tt_to_full(cores)

    def step(x):
        k1 = trunc(prob.apply(x))
        y2 = trunc(x + 0.5 * DT * k1)
        k2 = trunc(prob.apply(y2))
        y3 = trunc(x + 0.5 * DT * k2)
        k3 = trunc(prob.apply(y3))
        y4 = trunc(x + DT * k3)
        k4 = trunc(prob.apply(y4))
        return trunc(x + (DT / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4))

    for s in range(STEPS):
        f = step(f)
        if (s + 1) % 10 == 0:
            print(f"step {s + 1}: norm {np.linalg.norm(f):.12e} min gap {min_gap[0]:.6f}", flush=True)
    cores, _ = fullgrid.tt_svd(f, 0.0, None)
    ranks = [c.shape[2] for c in cores[:-1]]
    # the field is exactly rank <= CAP; drop numerically zero directions
    cores, _ = fullgrid.tt_svd(f, 1e-15, CAP)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "d4_n32_cap8_100steps.npz")
    arrays = {f"core{k}": c for k, c in enumerate(cores)}
    np.savez_compressed(out, mu=mu, sigma=sig, norm=np.linalg.norm(f), min_gap=min_gap[0],
                        full_ranks=np.array(ranks), **arrays)
    print("wrote", out, "ranks", [c.shape[2] for c in cores], "min gap", min_gap[0])


if __name__ == "__main__":
    main()
