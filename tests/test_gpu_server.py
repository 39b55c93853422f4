"""GPU: the request loop (mspcg_server_*) -- resident fields, admission by
device footprint, and its two ways of running requests: continuous batching
(the right-hand sides of one shape share the slots of one running batched
solve and enter it while others iterate; shapes run concurrently) and one
batched solve per request on its own stream.

A right-hand side's arithmetic does not depend on what runs beside it, so
every result must be the same alone (one request at a time, one batched
solve per request) and in the mix (all requests at once, continuously
batched, and as concurrent per-request solves): same iteration counts and
the same solution, bit for bit -- inside the stated tolerance by a wide
margin.  The oracle checks the residuals.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

MOB = (1.5, 0.5, 1.8)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_resid(op, b, x):
    return float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))


FIELDS = {"A": ((8, 4, 4, 4), 0.5, 21), "B": ((8, 8, 4, 4), 0.4, 22)}

# field, Ls, mf, sub, nrhs, solver
REQUESTS = [
    ("A", 4, 0.05, (4, 4, 4, 4), 2, dict(inner_iters=3)),
    ("B", 6, 0.1, (4, 4, 4, 4), 1, dict(inner_iters=4)),
    ("A", 4, 0.1, (4, 4, 4, 4), 3, dict(inner_iters=3, inner_prec="bf16")),
    ("B", 6, 0.05, (4, 4, 4, 4), 2, dict(inner_iters=4)),
    ("A", 5, 0.05, None, 1, dict(use_precond=False, beta_rule="FR")),
    ("A", 4, 0.05, (4, 4, 4, 4), 2, dict(inner_iters=3)),     # same shape as the first: context reuse
]


def sources(i, dims, Ls, nrhs):
    return [W.gaussian_source(dims, Ls, 700 + 10 * i + k) for k in range(nrhs)]


def run(max_inflight, budget=64 << 30, order=None, mode="batching", slots=3):
    import torch
    from paper_2104_05615_amd import Server
    srv = Server(0, budget, max_inflight)
    srv.set_mode(mode, slots)
    ids = {k: srv.add_field(d, W.gauge_field(d, eps, seed)) for k, (d, eps, seed) in FIELDS.items()}
    bufs, out = [], {}
    tickets = []
    idx = order if order is not None else range(len(REQUESTS))
    for i in idx:
        f, Ls, mf, sub, nrhs, solver = REQUESTS[i]
        dims = FIELDS[f][0]
        bs = sources(i, dims, Ls, nrhs)
        bt = torch.from_numpy(np.concatenate([b.view(np.float64).ravel() for b in bs])).cuda()
        xt = torch.empty_like(bt)
        torch.cuda.synchronize()
        t = srv.submit(ids[f], Ls, *MOB, mf, sub, nrhs, bt.data_ptr(), xt.data_ptr(), tol=1e-10, maxiter=4000,
                       **solver)
        bufs.append((i, bt, xt, bs))
        tickets.append((i, t))
        if max_inflight == 1:   # alone: finish each before the next arrives
            out[i] = srv.wait(t)
    for i, t in tickets:
        if i not in out:
            out[i] = srv.wait(t)
    info = srv.info()
    res = {}
    for i, bt, xt, bs in bufs:
        st, stats, lat = out[i]
        x = xt.cpu().numpy().view(np.complex128).reshape((len(bs),) + bs[0].shape)
        res[i] = (st, stats, lat, x, bs)
    srv.close()
    return res, info


def test_server_results_same_alone_and_in_the_mix():
    say("[gpu] server: requests one at a time, one batched solve each")
    alone, info1 = run(1, mode="contexts")
    say(f"      {info1}")
    assert info1["peak_inflight"] == 1
    assert info1["contexts"] < len(REQUESTS)           # the repeated shape reused its context
    say("[gpu] server: all requests at once, continuous batching (3 slots), reversed arrival")
    mix, info4 = run(4, order=list(reversed(range(len(REQUESTS)))))
    say(f"      {info4}")
    assert info4["peak_inflight"] >= 2
    assert info4["contexts"] < len(REQUESTS)           # one engine per shape
    say("[gpu] server: all requests at once, one batched solve each, 4 in flight")
    con, infoc = run(4, order=list(reversed(range(len(REQUESTS)))), mode="contexts")
    assert infoc["peak_inflight"] >= 2
    say("[gpu] server: requests one at a time, continuous batching")
    cb1, _ = run(1)
    for i in range(len(REQUESTS)):
        st1, s1, lat1, x1, bs = alone[i]
        for name, other in (("batching mix", mix), ("contexts mix", con), ("batching alone", cb1)):
            st4, s4, lat4, x4, _ = other[i]
            say(f"      request {i} {name}: status {st1}/{st4} iters {[a.outer_iters for a in s1]} "
                f"latency alone {lat1:.1f} ms, here {lat4:.1f} ms")
            assert st1 == 0 and st4 == 0
            assert [a.outer_iters for a in s1] == [a.outer_iters for a in s4]
            assert np.array_equal(x1, x4)
    # residuals of two of them against the oracle
    for i in (1, 2):
        f, Ls, mf, sub, nrhs, solver = REQUESTS[i]
        d, eps, seed = FIELDS[f]
        op = oracle.MobiusDWF(W.gauge_field(d, eps, seed), Ls, *MOB, mf)
        _, _, _, x, bs = mix[i]
        for k in range(nrhs):
            assert oracle_resid(op, bs[k], x[k]) < 2e-10


def test_server_admission_by_budget_and_oom():
    from paper_2104_05615_amd import MSPCG, MSPCG_ERR_OOM
    # footprint of the largest request shape, from a handle of the same shape
    d, eps, seed = FIELDS["B"]
    h = MSPCG(d)
    h.load_gauge(W.gauge_field(d, eps, seed))
    h.set_mobius(6, *MOB, 0.1)
    h.set_subdomains((4, 4, 4, 4))
    h.set_solver(tol=1e-10, inner_iters=4)
    est, _ = h.footprint(3)
    h.close()
    fields = sum(int(np.prod(v[0])) * 4 * 10 * 28 for v in FIELDS.values())
    budget = fields + int(1.3 * est)
    for mode in ("batching", "contexts"):
        say(f"[gpu] server ({mode}): budget {budget} B = fields {fields} + 1.3 x {est}")
        res, info = run(4, budget=budget, mode=mode, slots=3)
        say(f"      {info}")
        assert info["bytes_peak"] <= budget
        assert info["peak_inflight"] >= 1
        for i, (st, stats, lat, x, bs) in res.items():
            assert st == 0, (i, st)
        # a budget below any request (every solve needs more than 1 MB of
        # workspace here): each request fails with OOM, the server keeps running
        say(f"[gpu] server ({mode}): budget below one request")
        res, info = run(2, budget=fields + (256 << 10), mode=mode)
        assert all(v[0] == MSPCG_ERR_OOM for v in res.values())
        assert info["completed"] == len(REQUESTS) and info["inflight"] == 0


def test_engine_opens_with_the_slots_the_budget_holds():
    """A budget that holds one slot of the largest shape but not three:
    continuous batching still runs every request (that shape's engine opens
    with fewer slots and its right-hand sides take turns), inside the
    budget, and every solution meets the oracle's residual."""
    from paper_2104_05615_amd import MSPCG
    d, eps, seed = FIELDS["B"]
    h = MSPCG(d)
    h.load_gauge(W.gauge_field(d, eps, seed))
    h.set_mobius(6, *MOB, 0.1)
    h.set_subdomains((4, 4, 4, 4))
    h.set_solver(tol=1e-10, inner_iters=4)
    est1, _ = h.footprint(1)
    est3, _ = h.footprint(3)
    h.close()
    assert est3 > est1
    fields = sum(int(np.prod(v[0])) * 4 * 10 * 28 for v in FIELDS.values())
    budget = fields + (est1 + est3) // 2
    say(f"[gpu] server (batching, 3 slots): budget {budget} B = fields + (one slot {est1} + three {est3}) / 2")
    res, info = run(4, budget=budget, mode="batching", slots=3)
    say(f"      {info}")
    assert info["bytes_peak"] <= budget
    ops = {}
    for i, (st, stats, lat, x, bs) in res.items():
        assert st == 0, (i, st)
        f, Ls, mf, sub, nrhs, solver = REQUESTS[i]
        key = (f, Ls, mf)
        if key not in ops:
            dims, e, sd = FIELDS[f]
            ops[key] = oracle.MobiusDWF(W.gauge_field(dims, e, sd), Ls, *MOB, mf)
        for k in range(nrhs):
            assert oracle_resid(ops[key], bs[k], x[k]) < 2e-10


def test_footprint_estimate_covers_the_allocation():
    import torch
    from paper_2104_05615_amd import MSPCG
    d, eps, seed = FIELDS["B"]
    for solver, nrhs in ((dict(inner_iters=3), 3), (dict(use_precond=False, outer_prec="fp64"), 2),
                         (dict(inner_iters=2, inner_prec="fp32"), 1)):
        h = MSPCG(d)
        h.load_gauge(W.gauge_field(d, eps, seed))
        h.set_mobius(6, *MOB, 0.1)
        h.set_subdomains((4, 4, 4, 4))
        h.set_solver(tol=1e-8, maxiter=500, **solver)
        est, _ = h.footprint(nrhs)
        bs = [W.gaussian_source(d, 6, 800 + k) for k in range(nrhs)]
        bt = torch.from_numpy(np.concatenate([b.view(np.float64).ravel() for b in bs])).cuda()
        xt = torch.empty_like(bt)
        say(f"[gpu] footprint {solver} nrhs={nrhs}")
        st, stats = h.solve_batch_device(nrhs, bt.data_ptr(), xt.data_ptr())
        _, alloc = h.footprint(nrhs)
        say(f"      estimate {est} allocated {alloc}")
        assert st == 0
        assert alloc <= est and alloc >= 0.9 * est
        h.close()
