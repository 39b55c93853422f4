"""Write sampled FP64 oracle solutions for the GPU solve tests.

Calls only oracle/ (and the seeded generators in workloads/).  For a named
workload it runs the oracle's plain CG to a relative residual of 1e-12,
estimates the extreme eigenvalues of A from the CG (Lanczos) coefficients,
and stores: the iteration count, lambda_min, lambda_max, |x|, and the
solution at 256 seeded sample positions.

    python tests/golden/make_reference.py c1
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from workloads.configs import CONFIGS  # noqa: E402


def lanczos_extremes(alphas, betas):
    n = len(alphas)
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = 1 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < n:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def main(name):
    c = CONFIGS[name]
    U = W.gauge_field(c.dims, c.eps, c.gauge_seed)
    op = oracle.MobiusDWF(U, c.Ls, c.b, c.c, c.M5, c.mf)
    b = W.gaussian_source(c.dims, c.Ls, c.src_seed)
    alphas, betas = [], []
    x, info = oracle.cg(op, b, 1e-12, 20000)
    # the CG coefficients (alpha_k, beta_k) define the Lanczos tridiagonal of A;
    # rerun the recurrence for them
    r = b.copy()
    p = r.copy()
    rr = oracle.norm2(r)
    for _ in range(info.iters):
        q = op.A(p)
        a = rr / np.vdot(p, q).real
        r = r - a * q
        rn = oracle.norm2(r)
        alphas.append(a)
        betas.append(rn / rr)
        p = r + (rn / rr) * p
        rr = rn
    lmin, lmax = lanczos_extremes(alphas, betas)
    rng = np.random.default_rng(12345)
    idx = [(int(rng.integers(c.Ls)), int(rng.integers(op.vh)), int(rng.integers(4)), int(rng.integers(3)))
           for _ in range(256)]
    out = {
        "workload": name, "note": c.note, "solver": "oracle plain CG (FR), FP64, rel. residual 1e-12",
        "iters": info.iters, "true_rel_resid": info.true_rel_resid,
        "lambda_min": lmin, "lambda_max": lmax, "kappa": lmax / lmin,
        "x_norm": float(np.sqrt(oracle.norm2(x))),
        "samples": [[*i, float(x[i].real), float(x[i].imag)] for i in idx],
    }
    with open(os.path.join(HERE, f"reference_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "iters", info.iters, "kappa", lmax / lmin)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c1")
