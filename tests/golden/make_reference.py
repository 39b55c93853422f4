"""Write sampled FP64 oracle solutions for the GPU solve tests.

Calls only oracle/ (and the seeded generators in workloads/).  For a named
workload it runs the oracle's plain CG to a relative residual of ``tol``
(default 1e-13), estimates the extreme eigenvalues of A from the CG
coefficients (the Lanczos tridiagonal matrix they define), and stores: the
iteration count, lambda_min, lambda_max, kappa, |x|, and the solution at
``nsamples`` seeded sample positions (s, site, spin, colour).

    python tests/golden/make_reference.py c1
    python tests/golden/make_reference.py c2 --tol 1e-13 --samples 4096
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from workloads.configs import CONFIGS  # noqa: E402


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of the Lanczos matrix of CG: diagonal
    1/alpha_i + beta_{i-1}/alpha_{i-1}, off-diagonal sqrt(beta_i)/alpha_i."""
    n = len(alphas)
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = 1 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < n:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def main(name, tol, nsamples):
    c = CONFIGS[name]
    t0 = time.time()
    U = W.gauge_field(c.dims, c.eps, c.gauge_seed)
    op = oracle.MobiusDWF(U, c.Ls, c.b, c.c, c.M5, c.mf)
    b = W.gaussian_source(c.dims, c.Ls, c.src_seed)
    coeffs = []
    last = [time.time()]

    def progress(it, x, r):
        if time.time() - last[0] > 60:
            last[0] = time.time()
            print(f"{name}: iteration {it}, {time.time() - t0:.0f}s", flush=True)

    x, info = oracle.pcg(op, b, tol, 20000, precond=None, beta_rule="FR", callback=progress, coeffs=coeffs)
    alphas = [a for a, _ in coeffs]
    betas = [bb for _, bb in coeffs if bb is not None]
    lmin, lmax = lanczos_extremes(alphas, betas)
    rng = np.random.default_rng(12345)
    idx = [(int(rng.integers(c.Ls)), int(rng.integers(op.vh)), int(rng.integers(4)), int(rng.integers(3)))
           for _ in range(nsamples)]
    out = {
        "workload": name, "note": c.note,
        "solver": f"oracle plain CG (FR), FP64, rel. residual {tol:g}",
        "script": f"python tests/golden/make_reference.py {name} --tol {tol:g} --samples {nsamples}",
        "iters": info.iters, "true_rel_resid": info.true_rel_resid,
        "lambda_min": lmin, "lambda_max": lmax, "kappa": lmax / lmin,
        "x_norm": float(np.sqrt(oracle.norm2(x))),
        "history_first_20": [float(h) for h in info.history[:21]],
        "samples": [[*i, float(x[i].real), float(x[i].imag)] for i in idx],
    }
    with open(os.path.join(HERE, f"reference_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "iters", info.iters, "kappa", lmax / lmin, f"{time.time() - t0:.0f}s")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("name", nargs="?", default="c1")
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--samples", type=int, default=256)
    a = ap.parse_args()
    main(a.name, a.tol, a.samples)
