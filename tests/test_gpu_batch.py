"""GPU: the batched multi-RHS solve (one launch per kernel for all RHS,
device-side decisions, graph replay) against single-RHS solves and the oracle.

The batched path runs the kernels of the single-RHS solve with the same
block partitions and reduction orders and takes the same decisions, so every
RHS must reproduce its single-RHS solve bit for bit: the same iteration and
reliable-update counts and the same solution.  The oracle then checks the
true residual of the batched solutions.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_resid(op, b, x):
    return float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))


def make(dims, Ls, mf, sub, seed=11, eps=0.5):
    from paper_2104_05615_amd import MSPCG
    U = W.gauge_field(dims, eps, seed)
    s = MSPCG(dims)
    s.load_gauge(U)
    s.set_mobius(Ls, 1.5, 0.5, 1.8, mf)
    s.set_subdomains(sub)
    return s, oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, mf)


def dev(arrs):
    import torch
    flat = np.concatenate([np.ascontiguousarray(a).view(np.float64).ravel() for a in arrs])
    return torch.from_numpy(flat).cuda()


def batch_solve(s, bs, x0s=None):
    import torch
    bt = dev(bs)
    xt = torch.empty_like(bt)
    x0 = dev(x0s) if x0s is not None else None
    st, stats = s.solve_batch_device(len(bs), bt.data_ptr(), xt.data_ptr(), x0.data_ptr() if x0 is not None else None)
    torch.cuda.synchronize()
    xs = xt.cpu().numpy().view(np.complex128).reshape((len(bs),) + bs[0].shape)
    return st, stats, xs


def single_solve(s, b):
    import torch
    bt = dev([b])
    xt = torch.empty_like(bt)
    st = s.solve_device(bt.data_ptr(), xt.data_ptr())
    torch.cuda.synchronize()
    return st, xt.cpu().numpy().view(np.complex128).reshape(b.shape)


CASES = [
    # outer, inner, precond, beta rule
    ("fp32", "fp16", True, "PR"),
    ("fp32", "bf16", True, "PR"),
    ("fp64", "fp64", True, "FR"),
    ("fp32", "fp32", False, "FR"),
    ("fp64", "fp64", False, "PR"),
]


@pytest.mark.parametrize("outer,inner,pre,beta", CASES)
def test_batch_reproduces_single_solves(outer, inner, pre, beta):
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub)
    s.set_solver(tol=1e-10, maxiter=3000, inner_iters=3, inner_prec=inner, outer_prec=outer,
                 use_precond=pre, beta_rule=beta)
    bs = [W.gaussian_source(dims, Ls, 300 + i) for i in range(3)]
    say(f"[gpu] batch 3 RHS outer={outer} inner={inner} precond={pre} beta={beta}")
    st, stats, xs = batch_solve(s, bs)
    assert st == 0, [x.status for x in stats]
    for i, b in enumerate(bs):
        say(f"[gpu]   single RHS {i}")
        s1, x1 = single_solve(s, b)
        say(f"      batch iters={stats[i].outer_iters} RU={stats[i].reliable_updates} "
            f"single iters={s1.outer_iters} RU={s1.reliable_updates}")
        assert stats[i].status == 0 and s1.status == 0
        assert stats[i].outer_iters == s1.outer_iters
        assert stats[i].reliable_updates == s1.reliable_updates
        assert stats[i].inner_iters_total == s1.inner_iters_total
        assert stats[i].true_rel_resid == s1.true_rel_resid
        assert np.array_equal(xs[i], x1)
    res = oracle_resid(op, bs[1], xs[1])
    say(f"      oracle residual of RHS 1: {res:.2e}")
    assert res < 2e-10


def test_batch_graph_replay_equals_eager_and_autotune_keeps_results():
    from paper_2104_05615_amd import KIND_INNER, KIND_OUTER
    dims, Ls, sub = (8, 8, 4, 4), 6, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub, seed=12)
    s.set_solver(tol=1e-9, maxiter=2000, inner_iters=4, inner_prec="fp16", outer_prec="fp32")
    bs = [W.gaussian_source(dims, Ls, 400 + i) for i in range(4)]
    say("[gpu] batch 4 RHS, graph replay")
    st, stats, xg = batch_solve(s, bs)
    assert st == 0
    say("[gpu] batch 4 RHS, eager (profiling on)")
    s.set_profiling(True)
    st2, stats2, xe = batch_solve(s, bs)
    n1, ms1 = s.kernel_time(1)
    s.set_profiling(False)
    assert st2 == 0 and np.array_equal(xg, xe)
    assert [a.outer_iters for a in stats] == [a.outer_iters for a in stats2]
    # profiled inner hops: 4 per inner iteration, once for all RHS per launch
    most = max(a.outer_iters for a in stats)
    assert n1 >= 4 * 4 * most and ms1 > 0
    say("[gpu] autotune 4 RHS")
    s.autotune(4)
    for kind in (KIND_OUTER, KIND_INNER):
        order, xcd, us = s.schedule(kind, 4)
        say(f"      kind {kind}: order={order} xcd={xcd} {us:.1f} us")
        assert order in (0, 1) and xcd in (0, 1) and us > 0
    st3, stats3, xt = batch_solve(s, bs)
    assert st3 == 0 and np.array_equal(xg, xt)


def test_batch_mixed_status_zero_nan_and_iteration_limit():
    from paper_2104_05615_amd import MSPCG_ERR_BREAKDOWN, MSPCG_NOT_CONVERGED
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub)
    s.set_solver(tol=1e-10, maxiter=500, inner_iters=2)
    good = W.gaussian_source(dims, Ls, 501)
    bad = W.gaussian_source(dims, Ls, 502)
    bad[0, 0, 0, 0] = np.nan
    zero = np.zeros_like(good)
    say("[gpu] batch with a zero and a NaN source")
    st, stats, xs = batch_solve(s, [good, zero, bad])
    assert st == MSPCG_ERR_BREAKDOWN
    assert stats[0].status == 0 and oracle_resid(op, good, xs[0]) < 2e-10
    assert stats[1].status == 0 and stats[1].outer_iters == 0 and np.all(xs[1] == 0)
    assert stats[2].status == MSPCG_ERR_BREAKDOWN
    s1, x1 = single_solve(s, good)
    assert np.array_equal(x1, xs[0])
    s.set_solver(tol=1e-10, maxiter=3, inner_iters=2)
    say("[gpu] batch with maxiter 3")
    b2 = [W.gaussian_source(dims, Ls, 510 + i) for i in range(2)]
    st, stats, xs = batch_solve(s, b2)
    assert st == MSPCG_NOT_CONVERGED
    for i in range(2):
        assert stats[i].status == MSPCG_NOT_CONVERGED and stats[i].outer_iters == 3
        assert abs(oracle_resid(op, b2[i], xs[i]) - stats[i].true_rel_resid) < 1e-9


def test_batch_warm_start_and_uneven_convergence():
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub)
    s.set_solver(tol=1e-10, maxiter=2000, inner_iters=3)
    b = [W.gaussian_source(dims, Ls, 600 + i) for i in range(3)]
    say("[gpu] batch cold")
    st, stats, xs = batch_solve(s, b)
    assert st == 0
    # RHS 0 starts at its solution and stops after one iteration while the
    # others (from zero, and from half of the solution) keep going
    x0 = [xs[0], np.zeros_like(xs[1]), 0.5 * xs[2]]
    say("[gpu] batch warm, uneven")
    st, st2, xw = batch_solve(s, b, x0)
    assert st == 0
    assert st2[0].outer_iters <= 1
    for i in range(3):
        say(f"[gpu]   single warm RHS {i}")
        x1, s1 = s.solve(b[i], x0=x0[i])
        assert s1.outer_iters == st2[i].outer_iters and np.array_equal(x1, xw[i])
        assert oracle_resid(op, b[i], xw[i]) < 2e-10


# ---------------------------------------------------------------- continuous batching

@pytest.mark.parametrize("outer,inner,pre,beta", [("fp32", "fp16", True, "PR"), ("fp64", "fp64", False, "FR")])
def test_continuous_batching_session_reproduces_each_source_alone(outer, inner, pre, beta):
    """A session of 3 slots: sources enter while others iterate (two at the
    start, a third after a few steps, two more as slots free up, one
    refused while every slot is taken) and each leaves with the solution and
    counts of its own one-RHS batched solve, bit for bit; a zero source
    finishes at once with x = 0.  The oracle checks two residuals."""
    import torch
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub)
    s.set_solver(tol=1e-10, maxiter=3000, inner_iters=3, inner_prec=inner, outer_prec=outer,
                 use_precond=pre, beta_rule=beta)
    bs = [W.gaussian_source(dims, Ls, 900 + k) for k in range(5)] + [np.zeros_like(W.gaussian_source(dims, Ls, 1))]
    ref = []
    for b in bs:
        st, stats, xs = batch_solve(s, [b])
        ref.append((stats[0], xs[0]))
    bt = [dev([b]) for b in bs]
    xt = [torch.full_like(b, float("nan")) for b in bt]
    torch.cuda.synchronize()
    say(f"[gpu] continuous batching outer={outer} inner={inner} precond={pre}")
    s.cb_open(3)
    try:
        slot_of, got = {}, {}
        queue = list(range(len(bs)))

        def submit_next():
            if not queue:
                return False
            i = queue[0]
            k = s.cb_submit(bt[i].data_ptr(), xt[i].data_ptr())
            if k is None:
                return False
            slot_of[k] = i
            queue.pop(0)
            return True

        submit_next()
        submit_next()
        steps, refused = 0, 0
        while len(got) < len(bs):
            if steps == 3 or (steps > 3 and steps % 2 == 0):
                while submit_next():
                    pass
                if queue and s.cb_submit(bt[queue[0]].data_ptr(), xt[queue[0]].data_ptr()) is None:
                    refused += 1
            running, pending = s.cb_step()
            steps += 1
            for k in list(slot_of):
                st = s.cb_poll(k)
                if st is not None:
                    got[slot_of.pop(k)] = st
            assert steps < 4000
        torch.cuda.synchronize()
    finally:
        s.cb_close()
    say(f"      {steps} steps, {refused} submissions refused while every slot was taken")
    assert refused >= 1
    for i, (rs, rx) in enumerate(ref):
        g = got[i]
        x = xt[i].cpu().numpy().view(np.complex128).reshape(bs[i].shape)
        assert g.status == rs.status == 0, (i, g, rs)
        assert (g.outer_iters, g.reliable_updates) == (rs.outer_iters, rs.reliable_updates), (i, g, rs)
        assert np.array_equal(x, rx), i
    assert got[5].outer_iters == 0 and np.all(xt[5].cpu().numpy() == 0)
    for i in (0, 3):
        x = xt[i].cpu().numpy().view(np.complex128).reshape(bs[i].shape)
        assert oracle_resid(op, bs[i], x) < 2e-10


def test_continuous_batching_session_refuses_other_calls():
    from paper_2104_05615_amd import MSPCGError
    import paper_2104_05615_amd as M
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op = make(dims, Ls, 0.05, sub)
    s.set_solver(tol=1e-10, maxiter=100, inner_iters=2)
    s.cb_open(2)
    try:
        for call in (lambda: s.set_solver(tol=1e-8), lambda: s.solve(W.gaussian_source(dims, Ls, 3)),
                     lambda: s.apply("A", "fp32", W.gaussian_source(dims, Ls, 4)), lambda: s.cb_open(2),
                     lambda: M._check(M.mspcg_set_mfma(0))):
            with pytest.raises(MSPCGError) as e:
                call()
            assert e.value.status == -1
    finally:
        s.cb_close()
    s.set_solver(tol=1e-10, maxiter=2000, inner_iters=2)   # usable again after the session
    x, st = s.solve(W.gaussian_source(dims, Ls, 5))
    assert st.status == 0
