"""GPU parity at the benchmark's full size: the 16^3x32 x Ls12 workload (mf
0.01, links exp(0.5 iH)), FP32 outer operator, FP16 preconditioner on 256
subdomains of 4^3x8 with 6 inner steps, in the launch configuration the
benchmark times (default schedules: chunked block order of the full-lattice
hops, XCD ranges).

The oracle applies the full A at this size in about a second on the host, so
A is compared whole; the local operator and the preconditioner are compared
on sampled subdomains (each oracle A_s embeds its subdomain into the full
lattice); the solve is checked by the oracle's residual of the returned
solution, a property that holds at any size.  Tolerances as in
test_gpu_parity: FP32 operator 1e-6, FP16 composite operator 3e-3, FP16
preconditioner 3e-2, solve tol 1e-10 (the oracle's own residual).
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

SAMPLE_SUBDOMAINS = [0, 137, 255]   # first, one in the bulk, last


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


_ctx = {}


def c2():
    if not _ctx:
        from paper_2104_05615_amd import MSPCG
        from workloads.configs import CONFIGS
        cfg = CONFIGS["c2"]
        U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
        s = MSPCG(cfg.dims)
        s.load_gauge(U)
        s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
        s.set_subdomains(cfg.sub)
        s.set_solver(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec="fp16", outer_prec="fp32")
        op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
        _ctx.update(cfg=cfg, s=s, op=op, til=oracle.Tiling(cfg.dims, cfg.sub))
    return _ctx["cfg"], _ctx["s"], _ctx["op"], _ctx["til"]


def test_c2_outer_operator_full_size():
    cfg, s, op, til = c2()
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 701)
    say(f"[gpu] c2 A fp32 on {cfg.dims} x Ls{cfg.Ls}")
    e = rel(s.apply("A", "fp32", psi), op.A(psi))
    say(f"      rel error {e:.2e}")
    assert e < 1e-6, e


def test_c2_local_operator_and_preconditioner_sampled_subdomains():
    cfg, s, op, til = c2()
    r = W.gaussian_source(cfg.dims, cfg.Ls, 702)
    say(f"[gpu] c2 A_sub fp16, subdomains {SAMPLE_SUBDOMAINS} of {til.nsub}")
    got = s.apply("A_sub", "fp16", r)
    rs = np.stack([r[:, til.index[k]] for k in SAMPLE_SUBDOMAINS])
    ref = oracle.local_operator(op, til, rs, subset=SAMPLE_SUBDOMAINS)
    for j, k in enumerate(SAMPLE_SUBDOMAINS):
        e = rel(got[:, til.index[k]], ref[j])
        say(f"      subdomain {k}: rel error {e:.2e}")
        assert e < 3e-3, (k, e)
    say(f"[gpu] c2 preconditioner fp16 (k={cfg.inner_iters}), subdomain 0")
    z = s.apply("precond", "fp16", r)
    zr = oracle.inner_cg(op, til, r, cfg.inner_iters, subset=[0])[0]
    e = rel(z[:, til.index[0]], zr)
    say(f"      rel error {e:.2e}")
    assert e < 3e-2, e


def test_c2_mspcg_solution_has_oracle_residual_below_tolerance():
    cfg, s, op, til = c2()
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    say("[gpu] c2 MSPCG solve (FP32 outer + FP64 reliable updates, FP16 inner)")
    x, st = s.solve(b)
    res = float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))
    say(f"      {st.outer_iters} outer iterations, library {st.true_rel_resid:.3e}, oracle {res:.3e}")
    assert st.status == 0 and res <= cfg.tol, (st, res)
    assert abs(res - st.true_rel_resid) <= 1e-3 * res
