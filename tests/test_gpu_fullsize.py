"""GPU parity at full size.  The benchmark's 16^3x32 x Ls12 workload (mf
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
preconditioner 3e-2, solve tol 1e-10 (the oracle's own residual).  The
other workloads at their sizes: 16^4 x Ls16 (A whole, a batched solve of two
point-smeared sources) and 32^3x64 x Ls12 (A whole, A_s on one subdomain).
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


def _handle(cfg, U):
    from paper_2104_05615_amd import MSPCG
    s = MSPCG(cfg.dims)
    s.load_gauge(U)
    s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    s.set_subdomains(cfg.sub)
    s.set_solver(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec="fp16", outer_prec="fp32")
    return s


def test_c3_batched_point_sources_full_size():
    """16^4 x Ls16, mf 0.005: A against the oracle whole, and a batched solve
    of two of the twelve point-smeared sources (one launch per operator for
    both, graph replay), each checked by the oracle's residual."""
    import torch
    from workloads.configs import CONFIGS
    cfg = CONFIGS["c3"]
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    s = _handle(cfg, U)
    op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 703)
    say(f"[gpu] c3 A fp32 on {cfg.dims} x Ls{cfg.Ls}")
    e = rel(s.apply("A", "fp32", psi), op.A(psi))
    say(f"      rel error {e:.2e}")
    assert e < 1e-6, e
    B = W.point_smeared_sources(cfg.dims, cfg.Ls, cfg.src_seed, cfg.nrhs)[:2]
    say("[gpu] c3 batched MSPCG solve, 2 point-smeared sources")
    bt = torch.from_numpy(np.ascontiguousarray(B).view(np.float64).ravel().copy()).cuda()
    xt = torch.empty_like(bt)
    st, stats = s.solve_batch_device(2, bt.data_ptr(), xt.data_ptr())
    torch.cuda.synchronize()
    xs = xt.cpu().numpy().view(np.complex128).reshape(B.shape)
    assert st == 0
    for i in range(2):
        res = float(np.linalg.norm(B[i] - op.A(xs[i])) / np.linalg.norm(B[i]))
        say(f"      RHS {i}: {stats[i].outer_iters} outer iterations, oracle residual {res:.3e}")
        assert stats[i].status == 0 and res <= cfg.tol, (i, res)
    s.close()


def test_c4_operators_full_size():
    """32^3x64 x Ls12 (one GPU's share at production shape): A against the
    oracle whole, and the FP16 local operator on one sampled subdomain of 8^3x16."""
    from workloads.configs import CONFIGS
    cfg = CONFIGS["c4"]
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    s = _handle(cfg, U)
    op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    til = oracle.Tiling(cfg.dims, cfg.sub)
    del U
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 704)
    say(f"[gpu] c4 A fp32 on {cfg.dims} x Ls{cfg.Ls}")
    e = rel(s.apply("A", "fp32", psi), op.A(psi))
    say(f"      rel error {e:.2e}")
    assert e < 1e-6, e
    k = 100
    say(f"[gpu] c4 A_sub fp16, subdomain {k} of {til.nsub}")
    got = s.apply("A_sub", "fp16", psi)[:, til.index[k]]
    ref = oracle.local_operator(op, til, psi[:, til.index[k]][None], subset=[k])[0]
    e = rel(got, ref)
    say(f"      rel error {e:.2e}")
    assert e < 3e-3, e
    s.close()
