"""GPU parity at full size.  The 16^3x32 x Ls12 workload (mf 0.01, links
exp(0.5 iH)), FP32 outer operator, FP16 preconditioner on 256 subdomains of
4^3x8 with 6 inner steps, and the benchmark's 32^3x64 x Ls12 workload (mf
0.00078, links exp(0.6 iH), 256 subdomains of 8^3x16, 3 inner steps), each
in the launch configuration the benchmark times (default schedules: chunked
block order of the full-lattice hops, XCD ranges).

The oracle applies the full A at these sizes in seconds on the host, so A is
compared whole; the local operator and the preconditioner are compared on
sampled subdomains (through each subdomain's padded field, which the oracle
pins equal to R_s A R_s^T); a solve is checked by the oracle's residual of
the returned solution, a property that holds at any size, and at 16^3x32 also
against the oracle's own solution (tests/golden/reference_c2.json, sampled
entries).  Every comparison checks the whole-field relative error and the
largest single-site error, with the bounds of test_gpu_parity (FP32
operator 1e-6, FP16 operator 3e-3, FP16 preconditioner 3e-2 against the
exact operator).  The 16^4 x Ls16 workload: A
whole and a batched solve of its twelve point-smeared sources with the FP16
and with the BF16 preconditioner.
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


def site_rel(a, b):
    d = np.linalg.norm((a - b).reshape(-1, 12), axis=1)
    return float(d.max() / np.linalg.norm(b.reshape(-1, 12), axis=1).max())


SITE = 4.0


def check(got, ref, tol, what):
    e, es = rel(got, ref), site_rel(got, ref)
    say(f"      {what}: rel error {e:.2e}, worst site {es:.2e}")
    assert e < tol and es < SITE * tol, (what, e, es, tol)


def sampled_local_checks(s, op, til, r, subs, k):
    """A_s and the k-step preconditioner on sampled subdomains against the
    exact oracle (through each subdomain's padded field)."""
    got = s.apply("A_sub", "fp16", r)
    rs = np.stack([r[:, til.index[j]] for j in subs])
    ref = oracle.local_operator(op, til, rs, subset=subs, padded=True)
    for i, j in enumerate(subs):
        check(got[:, til.index[j]], ref[i], 3e-3, f"A_sub subdomain {j}")
    z = s.apply("precond", "fp16", r)
    j = subs[0]
    zr = oracle.inner_cg(op, til, r, k, subset=[j], padded=True)[0]
    check(z[:, til.index[j]], zr, 3e-2, f"preconditioner (k={k}) subdomain {j}")


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
    check(s.apply("A", "fp32", psi), op.A(psi), 1e-6, "A fp32")


def test_c2_local_operator_and_preconditioner_sampled_subdomains():
    cfg, s, op, til = c2()
    r = W.gaussian_source(cfg.dims, cfg.Ls, 702)
    say(f"[gpu] c2 A_sub and preconditioner fp16, subdomains {SAMPLE_SUBDOMAINS} of {til.nsub}")
    sampled_local_checks(s, op, til, r, SAMPLE_SUBDOMAINS, cfg.inner_iters)


def test_c2_mspcg_solution_has_oracle_residual_below_tolerance():
    """The MSPCG solution: the oracle's residual meets the tolerance, and the
    solution agrees with the oracle's own CG solution to 1e-13
    (tests/golden/reference_c2.json, 4096 sampled entries) within
    kappa * tol, kappa(A) from the Lanczos matrix of that CG."""
    import json
    import os
    cfg, s, op, til = c2()
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_c2.json")))
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    say("[gpu] c2 MSPCG solve (FP32 outer + FP64 reliable updates, FP16 inner)")
    x, st = s.solve(b)
    res = float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))
    say(f"      {st.outer_iters} outer iterations, library {st.true_rel_resid:.3e}, oracle {res:.3e}")
    assert st.status == 0 and res <= cfg.tol, (st, res)
    assert abs(res - st.true_rel_resid) <= 1e-3 * res
    d = np.array([x[i0, i1, i2, i3] - complex(re, im) for i0, i1, i2, i3, re, im in ref["samples"]])
    rms_rel = float(np.sqrt(np.mean(np.abs(d) ** 2)) / (ref["x_norm"] / np.sqrt(x.size)))
    say(f"      solution against the oracle's: sampled relative error {rms_rel:.2e} "
        f"(kappa {ref['kappa']:.3g}, kappa * tol = {ref['kappa'] * cfg.tol:.2e})")
    assert rms_rel < 2 * ref["kappa"] * cfg.tol


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
    of all twelve point-smeared sources (one launch per operator for all of
    them, graph replay) with the FP16 and with the BF16 preconditioner, each
    solution checked by the oracle's residual."""
    import torch
    from workloads.configs import CONFIGS
    cfg = CONFIGS["c3"]
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    s = _handle(cfg, U)
    op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 703)
    say(f"[gpu] c3 A fp32 on {cfg.dims} x Ls{cfg.Ls}")
    check(s.apply("A", "fp32", psi), op.A(psi), 1e-6, "A fp32")
    B = W.point_smeared_sources(cfg.dims, cfg.Ls, cfg.src_seed, cfg.nrhs)
    n = len(B)
    assert n == 12
    bt = torch.from_numpy(np.ascontiguousarray(B).view(np.float64).ravel().copy()).cuda()
    for inner in ("fp16", "bf16"):
        say(f"[gpu] c3 batched MSPCG solve, {n} point-smeared sources, {inner} preconditioner")
        s.set_solver(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec=inner, outer_prec="fp32")
        xt = torch.empty_like(bt)
        st, stats = s.solve_batch_device(n, bt.data_ptr(), xt.data_ptr())
        torch.cuda.synchronize()
        xs = xt.cpu().numpy().view(np.complex128).reshape(B.shape)
        assert st == 0
        for i in range(n):
            res = float(np.linalg.norm(B[i] - op.A(xs[i])) / np.linalg.norm(B[i]))
            say(f"      RHS {i}: {stats[i].outer_iters} outer iterations, oracle residual {res:.3e}")
            assert stats[i].status == 0 and res <= cfg.tol, (inner, i, res)
    s.close()


_c4 = {}


def c4():
    if not _c4:
        from workloads.configs import CONFIGS
        cfg = CONFIGS["c4"]
        U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
        s = _handle(cfg, U)
        op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
        _c4.update(cfg=cfg, s=s, op=op, til=oracle.Tiling(cfg.dims, cfg.sub))
    return _c4["cfg"], _c4["s"], _c4["op"], _c4["til"]


def test_c4_operators_full_size():
    """32^3x64 x Ls12 (one GPU's share at production shape): A against the
    oracle whole; the FP16 local operator on sampled subdomains of 8^3x16 and
    the k-step FP16 preconditioner on one, against the exact oracle."""
    cfg, s, op, til = c4()
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 704)
    say(f"[gpu] c4 A fp32 on {cfg.dims} x Ls{cfg.Ls}")
    check(s.apply("A", "fp32", psi), op.A(psi), 1e-6, "A fp32")
    subs = [100, 0, 255]
    say(f"[gpu] c4 A_sub and preconditioner fp16, subdomains {subs} of {til.nsub}")
    sampled_local_checks(s, op, til, psi, subs, cfg.inner_iters)


def test_c4_fp64_outer_operator_and_region_limits():
    """32^3x64 x Ls12 with its 8^3x16 tiling set: the FP64 A (reliable
    updates, FP64 CG) against the oracle whole; the FP64 A_s, whose region
    field of 256 subdomains would pass 4 GiB, is refused with INVALID_ARG
    while the operators without region fields stay available."""
    from paper_2104_05615_amd import MSPCGError, MSPCG_ERR_INVALID_ARG
    cfg, s, op, til = c4()
    psi = W.gaussian_source(cfg.dims, cfg.Ls, 705)
    say("[gpu] c4 A fp64")
    check(s.apply("A", "fp64", psi), op.A(psi), 1e-12, "A fp64")
    with pytest.raises(MSPCGError) as e:
        s.apply("A_sub", "fp64", psi)
    assert e.value.status == MSPCG_ERR_INVALID_ARG and "4 GiB" in str(e.value)


def test_c4_mspcg_solution_has_oracle_residual_below_tolerance():
    """The benchmark's solve (FP32 outer + FP64 reliable updates, FP16 inner,
    k = 3) in the benchmark's launch configuration: the oracle's residual of
    the returned solution meets the tolerance and equals the library's."""
    cfg, s, op, til = c4()
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    say("[gpu] c4 MSPCG solve")
    x, st = s.solve(b)
    res = float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))
    say(f"      {st.outer_iters} outer iterations, {st.reliable_updates} reliable updates, "
        f"library {st.true_rel_resid:.3e}, oracle {res:.3e}")
    assert st.status == 0 and res <= cfg.tol, (st, res)
    assert abs(res - st.true_rel_resid) <= 1e-3 * res
    s.close()
    _c4.clear()
