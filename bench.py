"""Benchmark: MSPCG vs CG time-to-solution on one MI355X.

A step is one complete solve A x = b (A = D^dag D of the even-odd Mobius
domain-wall operator) to a true relative residual of 1e-10, with the source
and gauge field already resident in HBM.  The default workload is one GPU's
share at production shape: a 32^3x64 lattice, Ls = 12, mf = 0.00078, links
exp(i 0.6 H); outer PCG in FP32 with FP64 reliable updates, inner CG in FP16
storage (FP32 arithmetic, MFMA fifth-dimension products) on 256 subdomains
of 8^3x16 with the snake terms kept.  Plain CG (FP32 + FP64 reliable
updates, and FP64) is timed beside it on the same GPU.

The legs after the timed steps (plain CG baselines, the serving sample, the
CPU oracle baseline) run only while the whole run stays inside --budget-s,
so that a long step count never pushes the run past its time limit; a
skipped leg says so in the JSON line.

Prints one JSON line.  `value` is the MSPCG time-to-solution in seconds.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MFMA_F16_PEAK_TFLOPS = 2500.0   # dense FP16 MFMA, MI355X
HBM_PEAK_GBS = 8000.0
METRIC = "MSPCG vs CG time-to-solution @ rel resid 1e-10; Dslash GB/s; p50/p99"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def region_counts(sub, dims):
    """Sites of the subdomain centre C (even), its L1 distance-1 shell N1 (odd)
    and distance-2 shell N2 (even), in the subdomain's local frame."""
    part = [s < d for s, d in zip(sub, dims)]
    rng = [range(-2, s + 2) if p else range(0, d) for s, d, p in zip(sub, dims, part)]
    nC = nN1 = nN2 = 0
    for t in rng[3]:
        for z in rng[2]:
            for y in rng[1]:
                for x in rng[0]:
                    c = (x, y, z, t)
                    dist = sum(max(0, -c[m], c[m] - (sub[m] - 1)) for m in range(4) if part[m])
                    par = (x + y + z + t) & 1
                    nC += dist == 0 and par == 0
                    nN1 += dist <= 1 and par == 1
                    nN2 += dist <= 2 and par == 0
    return nC, nN1, nN2


def stage_bytes(cfg, inner_prec):
    """Algorithmic bytes of one launch of each hop stage: every input site
    read once, every output written once, the epilogue's second field (w) and,
    in the last hop, the field of the fused <p, A p> partial read once where
    they are nonzero, and the 8 links of each output 4D site once (shared
    over Ls; FP32 for the outer hops, FP16 for the subdomain hops of the 16-
    and 8-bit formats).  Subdomain regions overlap their neighbours, so a
    subdomain hop counts a link once for every output site that needs it,
    whichever subdomain the site belongs to.  Keys: profiling kinds of the
    library (21..24 outer FP32 hops of A, 11..14 subdomain hops h1..h4)."""
    X, Y, Z, T = cfg.dims
    vh = X * Y * Z * T // 2
    Ls = cfg.Ls
    sp32 = 96
    sp16 = {"int8": 28, "fp16": 52, "bf16": 52, "fp32": 96, "fp64": 192}[inner_prec]
    link = 8 * 18 * 4                    # the 8 FP32 links of an output 4D site
    # subdomain hops of the 16- and 8-bit formats read FP16 links
    link_in = 8 * 18 * {"int8": 2, "fp16": 2, "bf16": 2, "fp32": 4, "fp64": 8}[inner_prec]
    n5 = vh * Ls
    out = {21: 2 * sp32 * n5 + link * vh, 22: 3 * sp32 * n5 + link * vh,
           23: 2 * sp32 * n5 + link * vh, 24: 4 * sp32 * n5 + link * vh}
    nC, nN1, nN2 = region_counts(cfg.sub, cfg.dims)
    ns = cfg.n_subdomains
    for k, (sin, sout) in {11: (nC, nN1), 12: (nN1 + nC, nN2), 13: (nN2, nN1), 14: (nN1 + 2 * nC, nC)}.items():
        out[k] = ns * Ls * sp16 * (sin + sout) + ns * link_in * sout
    return out, (nC, nN1, nN2)


STAGE_NAMES = {
    21: "k_hop<FullGeo,float,dag=0,w=0>: a = Q D^w_oe t0 (outer A, hop 1)",
    22: "k_hop<FullGeo,float,dag=0,w=1>: c = M5^-dag(p - M5^-1 D^w_eo a) (outer A, hop 2)",
    23: "k_hop<FullGeo,float,dag=1,w=0>: e = Q^dag D^w^dag_oe c (outer A, hop 3)",
    24: "k_hop<FullGeo,float,dag=1,w=1>: q = M5^dag c - M_phi^dag D^w^dag_eo e, <p,q> (outer A, hop 4)",
    11: "k_hop<SubGeo,half,dag=0,w=0>: h1 N1 <- C (inner A_s)",
    12: "k_hop<SubGeo,half,dag=0,w=1>: h2 N2 <- N1 (inner A_s)",
    13: "k_hop<SubGeo,half,dag=1,w=0>: h3 N1 <- N2 (inner A_s)",
    14: "k_hop<SubGeo,half,dag=1,w=1>: h4 C <- N1, <p_s,q_s> (inner A_s)",
}


# ---------------------------------------------------------------- serving stream

# request volumes of the serving stream: name -> (dims, Ls, subdomain tiling)
SERVE_VOLUMES = {
    "8^4x8": ((8, 8, 8, 8), 8, (4, 4, 4, 4)),
    "16^3x32x12": ((16, 16, 16, 32), 12, (4, 4, 4, 8)),
    "24^3x48x16": ((24, 24, 24, 48), 16, (6, 6, 6, 12)),
    "32^3x64x12": ((32, 32, 32, 64), 12, (8, 8, 8, 16)),
}
SERVE_FULL = dict(volumes=list(SERVE_VOLUMES), masses=[0.1, 0.01, 0.001], max_rhs=8)
SERVE_SAMPLE = dict(volumes=["8^4x8"], masses=[0.1, 0.01], max_rhs=3)


def serve_stream(volumes, masses, max_rhs, nreq=None, seed=105, load=0.75, budget_gb=140, max_inflight=4,
                 inner_iters=6, mode="batching", slots=8, work_s=None, svc=None):
    """Poisson stream of batched solves through the library's request server.

    Requests draw a volume, a mass and 1..max_rhs Gaussian sources (seeded,
    generated on the device); the gauge fields (one per volume, links
    exp(i 0.5 H), seeds 105, 106, ...) are resident.  The service time of each
    (volume, mass) is measured once, alone, with one RHS (or taken from
    `svc`); the stream is the first `nreq` requests of the seeded sequence,
    or as many as fit `work_s` seconds of sequential work; the arrival rate
    is `load` times the capacity those times imply for serving the drawn
    requests one after another.  Latency is submit -> completion, measured
    by the server.  `mode`: 'batching' (continuous batching, `slots` RHS
    slots per request shape) or 'contexts' (one batched solve per request).
    A progress line goes to stderr at least every 30 s."""
    import threading
    import torch
    import workloads as W
    from paper_2104_05615_amd import Server
    rng = np.random.default_rng(seed)
    cap = nreq if nreq is not None else 100000
    reqs = []
    for i in range(cap if nreq is not None else 1000):
        reqs.append((volumes[int(rng.integers(len(volumes)))], float(masses[int(rng.integers(len(masses)))]),
                     int(rng.integers(1, max_rhs + 1))))
    gaps = rng.exponential(1.0, size=len(reqs))
    srv = Server(0, int(budget_gb) << 30, max_inflight)
    srv.set_mode(mode, slots)
    fid = {}
    for k, name in enumerate(volumes):
        dims, Ls, sub = SERVE_VOLUMES[name]
        fid[name] = srv.add_field(dims, W.gauge_field(dims, 0.5, seed + k))
    solver = dict(tol=1e-10, maxiter=100000, inner_iters=inner_iters, inner_prec="fp16", outer_prec="fp32")
    stream = torch.cuda.current_stream()

    def make(name, nrhs, s):
        dims, Ls, sub = SERVE_VOLUMES[name]
        n = nrhs * Ls * int(np.prod(dims)) // 2 * 24
        g = torch.Generator(device="cuda")
        g.manual_seed(s)
        b = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
        return b, torch.empty_like(b)

    def submit(name, mf, nrhs, b, x):
        dims, Ls, sub = SERVE_VOLUMES[name]
        stream.synchronize()
        return srv.submit(fid[name], Ls, 1.5, 0.5, 1.8, mf, sub, nrhs, b.data_ptr(), x.data_ptr(), **solver)

    # service time per (volume, mass), one RHS, alone (also creates the
    # contexts), measured for the (volume, mass) pairs the stream reaches
    svc = dict(svc or {})
    total, n = 0.0, 0
    for name, mf, k in reqs:
        if (name, mf) not in svc:
            b, x = make(name, 1, 1)
            log(f"[serve] measuring {name} mf={mf} alone")
            st, stats, lat = srv.wait(submit(name, mf, 1, b, x))
            assert st == 0, (name, mf, st)
            svc[(name, mf)] = lat / 1e3
            log(f"[serve] alone {name} mf={mf}: {lat / 1e3:.3f}s, {stats[0].outer_iters} iters")
        if nreq is None and n > 0 and total + svc[(name, mf)] * k > work_s:
            break
        total += svc[(name, mf)] * k
        n += 1
    reqs = reqs[:n]
    gaps = gaps[:n]
    nreq = len(reqs)
    work = sum(svc[(n, m)] * k for n, m, k in reqs)
    capacity = nreq / work
    lam = load * capacity
    log(f"[serve] {mode}: {nreq} requests, sequential work {work:.1f}s, capacity {capacity:.3f}/s, "
        f"arrival rate {lam:.3f}/s")
    results = [None] * nreq
    pending = []
    cv = threading.Condition()
    done_submitting = [False]
    ndone = [0]
    t0 = time.perf_counter()

    def waiter():
        last = time.perf_counter()
        while True:
            with cv:
                while not pending and not done_submitting[0]:
                    cv.wait()
                if not pending:
                    return
                i, t, bufs = pending.pop(0)
            while not srv.poll(t):
                time.sleep(0.05)
                if time.perf_counter() - last > 30:
                    last = time.perf_counter()
                    inf = srv.info()
                    r = reqs[i]
                    log(f"[serve] {time.perf_counter() - t0:.0f}s: {ndone[0]} of {nreq} done, waiting on request "
                        f"{i} ({r[0]}, mf={r[1]}, {r[2]} RHS), {inf['inflight']} in flight, "
                        f"{inf['waiting']} queued")
            results[i] = srv.wait(t)
            del bufs
            # the request's buffers go back to the device, not to torch's
            # cache, so that the server's own allocations find the memory
            torch.cuda.empty_cache()
            ndone[0] += 1
            last = time.perf_counter()
            r = reqs[i]
            log(f"[serve] request {i} ({r[0]}, mf={r[1]}, {r[2]} RHS) done: status {results[i][0]}, "
                f"latency {results[i][2] / 1e3:.2f}s")

    th = threading.Thread(target=waiter, daemon=True)
    th.start()
    t0 = time.perf_counter()
    t_next = 0.0
    try:
        for i, (name, mf, nrhs) in enumerate(reqs):
            t_next += gaps[i] / lam
            b, x = make(name, nrhs, 1000 + i)
            delay = t0 + t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            t = submit(name, mf, nrhs, b, x)
            with cv:
                pending.append((i, t, (b, x)))
                cv.notify()
    finally:
        # the requests already submitted finish (the waiter drains them)
        # even when this loop fails, so the run ends instead of waiting
        with cv:
            done_submitting[0] = True
            cv.notify()
        th.join()
    makespan = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    lats = np.array([r[2] for r in results]) / 1e3
    ok = all(r[0] == 0 for r in results)
    nrhs_tot = sum(r[2] for r in reqs)
    out = {"design": mode, "slots": slots if mode == "batching" else None,
           "requests": nreq, "rhs": nrhs_tot, "all_converged": ok,
           "p50_s": float(np.percentile(lats, 50)), "p99_s": float(np.percentile(lats, 99)),
           "mean_s": float(lats.mean()), "max_s": float(lats.max()),
           "solves_per_s": nreq / makespan, "rhs_per_s": nrhs_tot / makespan, "makespan_s": makespan,
           "arrival_rate_per_s": lam, "capacity_sequential_per_s": capacity, "load": load,
           "sequential_work_s": work,
           "max_inflight": max_inflight, "budget_bytes": info["budget"], "peak_bytes": info["bytes_peak"],
           "peak_inflight": info["peak_inflight"], "contexts": info["contexts"], "evictions": info["evictions"],
           "mix": {"volumes": volumes, "masses": masses, "rhs": [1, max_rhs], "seed": seed,
                   "service_alone_s": {f"{n} mf={m}": v for (n, m), v in svc.items()}}}
    log(f"[serve] {mode}: p50 {out['p50_s']:.3f}s p99 {out['p99_s']:.3f}s, {out['solves_per_s']:.3f} solves/s, "
        f"peak in flight {info['peak_inflight']}")
    out["_svc"] = svc
    return out


# ---------------------------------------------------------------- batched multi-RHS (16^4 x Ls16, 12 sources)

def batch_bench(args):
    import torch
    import workloads as W
    from workloads.configs import CONFIGS
    from paper_2104_05615_amd import MSPCG, KIND_FP64, KIND_INNER, KIND_OUTER
    cfg = CONFIGS["c3"]
    log(f"[batch] workload {cfg.name}: {cfg.note}")
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    B = W.point_smeared_sources(cfg.dims, cfg.Ls, cfg.src_seed, cfg.nrhs)
    s = MSPCG(cfg.dims)
    s.load_gauge(U)
    s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    s.set_subdomains(cfg.sub)
    n = cfg.nrhs
    bt = torch.from_numpy(B.view(np.float64).reshape(-1).copy()).cuda()
    xt = torch.empty_like(bt)
    per = bt.numel() // n
    out = {"metric": "batched multi-RHS time-to-solution @ rel resid 1e-10", "unit": "s", "config": {
        "workload": f"{cfg.name}: {cfg.note}", "lattice": list(cfg.dims), "Ls": cfg.Ls, "mf": cfg.mf,
        "eps": cfg.eps, "subdomain": list(cfg.sub), "inner_iters": cfg.inner_iters, "nrhs": n,
        "sources": "point-smeared (Gaussian profile, sigma 2, spin-colour unit vectors)"}}
    for inner in ("fp16", "bf16"):
        s.set_solver(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec=inner, outer_prec="fp32")
        # one RHS after another
        torch.cuda.synchronize()
        t = time.perf_counter()
        seq = []
        for r in range(n):
            st = s.solve_device(bt[r * per:].data_ptr(), xt[r * per:].data_ptr())
            seq.append(st)
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t
        log(f"[batch] {inner}: {n} single solves {t_seq:.2f}s, iters {[a.outer_iters for a in seq]}")
        x_seq = xt.clone()
        s.autotune(n)
        sched = {k: s.schedule(kk, n) + (s.tchunk(kk, n),) for k, kk in (("outer", KIND_OUTER), ("fp64", KIND_FP64),
                                                                       ("inner", KIND_INNER))}
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, stats = s.solve_batch_device(n, bt.data_ptr(), xt.data_ptr())
        torch.cuda.synchronize()
        t_bat = time.perf_counter() - t
        same = bool(torch.equal(x_seq, xt))
        log(f"[batch] {inner}: batched {t_bat:.2f}s (status {st}), iters {[a.outer_iters for a in stats]}, "
            f"identical to single solves: {same}")
        out[inner] = {"sequential_s": t_seq, "batched_s": t_bat, "speedup": t_seq / t_bat, "status": st,
                      "outer_iters": [a.outer_iters for a in stats],
                      "true_rel_resid_max": max(a.true_rel_resid for a in stats),
                      "identical_to_single_solves": same,
                      "schedule": {k: {"order": v[0], "xcd": v[1], "tchunk": v[3], "four_hops_us": v[2]}
                                   for k, v in sched.items()}}
    out["value"] = out["fp16"]["batched_s"]
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- reduced-Ls preconditioner

def reduced_bench(args):
    """Reduced-Ls preconditioner (Sec. 3.3) on one workload: residual vectors
    r_k of a full-Ls MSPCG solve (after 25, 50, 100 and 200 outer iterations)
    train T (Lhat = Ls / 2, started from taking every second slice) for each
    mu of a small scan, and the full solve then runs with each trained
    preconditioner; reported beside the full-Ls MSPCG solve."""
    import torch
    import workloads as W
    from workloads.configs import CONFIGS
    from paper_2104_05615_amd import MSPCG
    cfg = CONFIGS[args.config]
    inner = args.inner_prec or cfg.inner_prec
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    s = MSPCG(cfg.dims)
    s.load_gauge(U)
    s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    s.set_subdomains(cfg.sub)
    s.set_log(args.log_every)
    bt = torch.from_numpy(b.view(np.float64).reshape(-1).copy()).cuda()
    xt = torch.empty_like(bt)
    n = bt.numel()
    params = dict(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec=inner,
                  outer_prec=cfg.outer_prec)

    def solve(**kw):
        s.set_solver(**dict(params, **kw))
        torch.cuda.synchronize()
        t = time.perf_counter()
        st = s.solve_device(bt.data_ptr(), xt.data_ptr())
        torch.cuda.synchronize()
        return time.perf_counter() - t, st

    solve()                                      # warm-up
    t_full, st_full = solve()
    log(f"[reduced] full Ls={cfg.Ls}: {t_full:.3f}s, {st_full.outer_iters} outer iterations")
    # training vectors: true residuals b - A x_k of the full-Ls solve
    vs = []
    ax = torch.empty_like(bt)
    for k in (25, 50, 100, 200):
        solve(maxiter=k)
        s.apply_device("A", "fp64", xt.data_ptr(), ax.data_ptr())
        torch.cuda.synchronize()
        vs.append(bt - ax)
    V = torch.cat([v / torch.linalg.vector_norm(v) for v in vs]).contiguous()
    Lh = cfg.Ls // 2
    T0 = np.zeros((Lh, 4, cfg.Ls, 4), dtype=np.complex128)
    for j in range(Lh):
        T0[j, :, 2 * j, :] = np.eye(4)
    out = {"metric": "reduced-Ls MSPCG time-to-solution @ rel resid 1e-10", "unit": "s", "config": cfg.name,
           "full": {"Ls": cfg.Ls, "time_s": t_full, "outer_iters": st_full.outer_iters}, "reduced": []}
    # Mobius parameters of the reduced operator: those of the full one, and
    # the same b - c with b + c scaled by Ls / Lhat (the Mobius scale that keeps
    # b + c times the number of slices)
    bc = [(cfg.b, cfg.c)]
    if args.alpha_match:
        a = (cfg.b + cfg.c) * cfg.Ls / Lh
        bc.append(((a + cfg.b - cfg.c) / 2, (a - cfg.b + cfg.c) / 2))
    for (bh, ch), mu in [(x, m) for x in bc for m in args.mu]:
        s.set_reduced(Lh, bh, ch, mu=mu, T=T0)
        s.set_solver(**params)
        t = time.perf_counter()
        hist = s.train_reduced(len(vs), V.data_ptr(), args.train_iters, momentum=0.5)
        t_train = time.perf_counter() - t
        log(f"[reduced] mu={mu}: trained in {t_train:.1f}s, chi2 {hist[0]:.3e} -> {hist[-1]:.3e}")
        t_red, st_red = solve(maxiter=5000)
        s.set_reduced(Lh, bh, ch, mu=mu, T=T0)
        t_dec, st_dec = solve(maxiter=5000)
        log(f"[reduced] Lhat={Lh} b_hat={bh:g} c_hat={ch:g} mu={mu}: chi2 {hist[0]:.3e} -> {hist[-1]:.3e} in {t_train:.1f}s; solve "
            f"{t_red:.3f}s, {st_red.outer_iters} iters (status {st_red.status}); untrained T: {t_dec:.3f}s, "
            f"{st_dec.outer_iters} iters")
        out["reduced"].append({"Lhat": Lh, "b_hat": bh, "c_hat": ch, "mu": mu, "train_s": t_train, "chi2_first": hist[0], "chi2_last": hist[-1],
                               "time_s": t_red, "outer_iters": st_red.outer_iters, "status": st_red.status,
                               "true_rel_resid": st_red.true_rel_resid,
                               "untrained": {"time_s": t_dec, "outer_iters": st_dec.outer_iters}})
    s.set_reduced(0)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- kernels only (for counter runs)

def kernels_bench(args):
    """A few applications of the outer operator A (FP32) and of the local
    operator A_s (inner precision) on one workload, and a plain device copy
    of 1 GiB whose counters calibrate the HBM byte counters.  No solve: a
    short program for rocprofv3 counter passes."""
    import torch
    import workloads as W
    from workloads.configs import CONFIGS
    from paper_2104_05615_amd import MSPCG
    cfg = CONFIGS[args.config]
    inner = args.inner_prec or cfg.inner_prec
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    s = MSPCG(cfg.dims)
    s.load_gauge(U)
    s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    s.set_subdomains(cfg.sub)
    s.set_solver(tol=cfg.tol, inner_iters=cfg.inner_iters, inner_prec=inner, outer_prec="fp32")
    bt = torch.from_numpy(b.view(np.float64).reshape(-1).copy()).cuda()
    xt = torch.empty_like(bt)
    src = torch.ones(1 << 28, device="cuda", dtype=torch.float32)   # 1 GiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    out = {"mode": "kernels", "config": cfg.name, "copy_bytes": 2 * src.numel() * 4}
    t = time.perf_counter()
    dst.copy_(src)
    torch.cuda.synchronize()
    out["copy_ms"] = 1e3 * (time.perf_counter() - t)
    for op, prec in (("A", "fp32"), ("A_sub", inner)):
        s.set_profiling(True)
        for _ in range(args.steps):
            s.apply_device(op, prec, bt.data_ptr(), xt.data_ptr())
        torch.cuda.synchronize()
        n_o, ms_o = s.kernel_time(0)
        n_i, ms_i = s.kernel_time(1)
        s.set_profiling(False)
        out[f"{op}_{prec}"] = {"outer_hops": n_o, "outer_ms": ms_o, "inner_hops": n_i, "inner_ms": ms_i}
        log(f"[kernels] {op} {prec}: {args.steps} applications")
    # a few outer iterations of MSPCG and of plain FP32 CG (iteration limit,
    # not converged): the BLAS-1, restriction, inner update and
    # prolongation kernels of one solve, for their counters
    if args.solve_iters > 0:
        for label, kw in (("mspcg", dict(inner_iters=cfg.inner_iters, inner_prec=inner, outer_prec="fp32")),
                          ("cg_fp32", dict(outer_prec="fp32", use_precond=False, beta_rule="FR"))):
            s.set_solver(tol=cfg.tol, maxiter=args.solve_iters, reliable_delta=0.1, **kw)
            st = s.solve_device(bt.data_ptr(), xt.data_ptr())
            torch.cuda.synchronize()
            out[label] = {"outer_iters": st.outer_iters, "status": st.status}
            log(f"[kernels] {label}: {st.outer_iters} outer iterations (limit {args.solve_iters})")
    print(json.dumps(out), flush=True)


KERNEL_SOURCES = ["common.h", "sitekern.h", "kernels.h", "kernels.hip", "sub.hip"]
def traffic_summary(workload):
    return os.path.join(ROOT, "profiles", f"hop_kernels_{workload}_hbm_traffic.md")
PROF_STRIDE = 8   # hop launches per timed launch in the bench's timed region


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_05615_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, stage):
    """HBM bytes per launch of a hop stage from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE passes, scaled by a plain
    copy); None when the kernels changed since, or for another workload."""
    try:
        txt = open(traffic_summary(workload)).read()
        blob = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != kernel_source_hash() or blob.get("workload") != workload:
        return None
    k = blob.get("stages", {}).get(str(stage))
    return None if k is None else k["traffic_bytes"]


T_BEGIN = time.time()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--inner-prec", default=None)
    ap.add_argument("--cg-steps", type=int, default=1)
    ap.add_argument("--solve-iters", type=int, default=0,
                    help="kernels mode: also run MSPCG and FP32 CG to this many outer iterations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", default="solve", choices=["solve", "batch", "serve", "kernels", "reduced"])
    ap.add_argument("--mu", type=float, nargs="+", default=[0.05, 0.2], help="mu values of the reduced-Ls scan")
    ap.add_argument("--train-iters", type=int, default=10, help="training steps of the reduced-Ls transform")
    ap.add_argument("--alpha-match", action="store_true",
                    help="also scan the reduced operator with b + c scaled by Ls / Lhat")
    ap.add_argument("--log-every", type=int, default=0, help="solver progress line every N outer iterations")
    ap.add_argument("--no-cg64", action="store_true", help="skip the FP64 CG baseline")
    ap.add_argument("--prec-compare", action="store_true",
                    help="also solve with the other inner storage formats (outside the timed region)")
    ap.add_argument("--budget-s", type=float, default=480.0,
                    help="wall-clock budget of the whole run: legs after the timed steps are skipped "
                         "when they would not fit")
    ap.add_argument("--oracle-check", action="store_true",
                    help="relative residual of the MSPCG solution by the FP64 oracle on the host")
    ap.add_argument("--requests", type=int, default=None, help="serving stream length (default: --serve-work)")
    ap.add_argument("--serve-work", type=float, default=300.0,
                    help="serving stream: as many requests as fit this many seconds of sequential work")
    ap.add_argument("--serve-design", default="batching", choices=["batching", "contexts", "both"])
    ap.add_argument("--slots", type=int, default=8, help="RHS slots per shape (continuous batching)")
    ap.add_argument("--budget-gb", type=int, default=140,
                    help="HBM budget of the request server (GB); the clients' sources and solutions, up to "
                         "38 GB per 32^3x64 x Ls12 request of 8 RHS, live beside it")
    ap.add_argument("--serve-sample", type=int, default=10,
                    help="requests of the serving sample in solve mode (0: none)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "bench.py runs on one GPU: the solver has no multi-GPU halo exchange, "
                                   "so --gpus N > 1 is not supported"}))
        sys.exit(2)
    if args.mode == "batch":
        return batch_bench(args)
    if args.mode == "reduced":
        return reduced_bench(args)
    if args.mode == "kernels":
        return kernels_bench(args)
    if args.mode == "serve":
        import torch  # noqa: F401
        designs = ["batching", "contexts"] if args.serve_design == "both" else [args.serve_design]
        out, svc = {}, None
        for d in designs:
            r = serve_stream(nreq=args.requests, work_s=args.serve_work, budget_gb=args.budget_gb, mode=d,
                             slots=args.slots, svc=svc, **SERVE_FULL)
            svc = r.pop("_svc")
            out[d] = r
            print(json.dumps({"design": d, "serve": r}), file=sys.stderr, flush=True)
        print(json.dumps({"metric": "serving p50/p99 latency and solves/s", "unit": "s",
                          "value": out[designs[0]]["p99_s"], "serve": out}), flush=True)
        return

    import torch
    import workloads as W
    from workloads.configs import CONFIGS
    from paper_2104_05615_amd import MSPCG, KERNEL_INNER_HOP, KERNEL_OUTER_HOP, KERNEL_PRECOND

    cfg = CONFIGS[args.config]
    inner = args.inner_prec or cfg.inner_prec
    log(f"[bench] workload {cfg.name}: {cfg.note}")
    t0 = time.time()
    U = W.gauge_field(cfg.dims, cfg.eps, cfg.gauge_seed)
    b = W.gaussian_source(cfg.dims, cfg.Ls, cfg.src_seed)
    log(f"[bench] inputs generated in {time.time() - t0:.1f}s")

    s = MSPCG(cfg.dims, device=0)
    s.load_gauge(U)
    s.set_mobius(cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    s.set_subdomains(cfg.sub)
    s.set_log(args.log_every)
    dev = torch.device("cuda:0")
    bt = torch.from_numpy(b.view(np.float64).reshape(-1).copy()).to(dev)
    xt = torch.empty_like(bt)
    torch.cuda.synchronize()

    def run(n, label=None, **solver):
        s.set_solver(**solver)
        out = []
        for _ in range(n):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = s.solve_device(bt.data_ptr(), xt.data_ptr())
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t, st))
            if label:
                # one line per solve as it ends (a few microseconds against
                # seconds per solve): a long timed region stays visibly alive
                log(f"[bench] {label} {len(out) - 1}: {out[-1][0]:.3f}s, {st.outer_iters} outer, "
                    f"{st.reliable_updates} RU, true resid {st.true_rel_resid:.2e}")
        return out

    mspcg_params = dict(tol=cfg.tol, maxiter=20000, inner_iters=cfg.inner_iters, inner_prec=inner,
                        outer_prec=cfg.outer_prec, reliable_delta=0.1, beta_rule="PR", use_precond=True)
    # warmup
    # The oracle's bounded CPU sample runs on the host cores while the GPU
    # does its untimed warmup solves (it touches no device memory); it is
    # joined before the timed region starts.
    cpu = {}
    cpu_thread = None
    if not args.no_cpu_baseline:
        import threading

        def cpu_job():
            try:
                cpu["sample"] = cpu_sample(cfg, U, b)
            except Exception as e:   # reported in the line, never fatal to the GPU bench
                cpu["error"] = repr(e)
        cpu_thread = threading.Thread(target=cpu_job, name="oracle-cpu-sample")
        cpu_thread.start()
    run(args.warmup, label="warmup", **mspcg_params)
    if cpu_thread is not None:
        cpu_thread.join()
    # timed region: K solves; HIP events on the solver's stream time one
    # launch in PROF_STRIDE of every hop stage (all launches of a stage do
    # the same work, and timing every one of them would add ~5% to the solve)
    s.set_profiling(True, stride=PROF_STRIDE)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    res = run(args.steps, label="step", **mspcg_params)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    n_out, ms_out = s.kernel_time(KERNEL_OUTER_HOP)
    n_in, ms_in = s.kernel_time(KERNEL_INNER_HOP)
    n_pc, ms_pc = s.kernel_time(KERNEL_PRECOND)
    stage_t = {k: s.kernel_time(k) for k in STAGE_NAMES}
    s.set_profiling(False)
    times = [r[0] for r in res]
    sts = [r[1] for r in res]
    assert all(st.status == 0 and st.true_rel_resid <= cfg.tol for st in sts), "MSPCG did not converge"
    x_ms = xt.clone()

    # legs after the timed region run while the run stays inside the budget
    t_solve = statistics.median(times)
    skipped = []

    def fits(name, est_s):
        ok = time.time() - T_BEGIN + est_s <= args.budget_s
        if not ok:
            skipped.append(name)
            log(f"[bench] {name}: skipped (estimated {est_s:.0f}s would exceed the {args.budget_s:.0f}s budget)")
        return ok

    # baselines on the same GPU (outside the timed region)
    cg32 = cg64 = None
    x_cg = None
    if fits("cg_fp32", 0.6 * t_solve * args.cg_steps):
        cg32 = run(args.cg_steps, tol=cfg.tol, maxiter=100000, outer_prec="fp32", reliable_delta=0.1,
                   beta_rule="FR", use_precond=False)
        log(f"[bench] CG fp32: {cg32[-1][0]:.3f}s, {cg32[-1][1].outer_iters} iters, "
            f"true resid {cg32[-1][1].true_rel_resid:.2e}")
        x_cg = xt.clone()
    if not args.no_cg64 and fits("cg_fp64", 1.5 * t_solve * args.cg_steps):
        cg64 = run(args.cg_steps, tol=cfg.tol, maxiter=100000, outer_prec="fp64", reliable_delta=0.1,
                   beta_rule="FR", use_precond=False)
        log(f"[bench] CG fp64: {cg64[-1][0]:.3f}s, {cg64[-1][1].outer_iters} iters, "
            f"true resid {cg64[-1][1].true_rel_resid:.2e}")
        x_cg = xt.clone()
    sol_rel = (float(torch.linalg.vector_norm(x_ms - x_cg) / torch.linalg.vector_norm(x_cg))
               if x_cg is not None else None)

    # the preconditioner's storage format against the outer iteration count
    # (Sec. 3.2: 8-bit storage is cheaper per inner step, 16-bit a better
    # preconditioner); one solve each, outside the timed region
    storage = {}
    for p in ([q for q in ("fp16", "bf16", "int8") if q != inner] if args.prec_compare else []):
        if not fits(f"inner_{p}", 1.3 * t_solve):
            continue
        (dt, st), = run(1, **dict(mspcg_params, inner_prec=p))
        storage[p] = {"time_s": dt, "outer_iters": st.outer_iters, "status": st.status,
                      "true_rel_resid": st.true_rel_resid}
        log(f"[bench] MSPCG inner {p}: {dt:.3f}s, {st.outer_iters} outer iters, "
            f"true resid {st.true_rel_resid:.2e}")

    # roofline of the hop kernels (HIP events over the timed region)
    sbytes, regions = stage_bytes(cfg, inner)
    kernels = {}
    for k, (n, ms) in stage_t.items():
        if n:
            avg = ms / n
            kernels[str(k)] = {"name": STAGE_NAMES[k], "launches_timed": n, "sample_stride": PROF_STRIDE,
                               "total_ms_est": ms * PROF_STRIDE, "avg_ms": avg,
                               "algorithmic_bytes": sbytes[k], "GBps": sbytes[k] / (avg * 1e-3) / 1e9}
    dom_key, dom = max(kernels.items(), key=lambda kv: kv[1]["total_ms_est"])
    roof = {"kernel": dom["name"], "bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dom["GBps"] / HBM_PEAK_GBS, "traffic": measured_traffic(cfg.name, dom_key),
            "avg_launch_ms": dom["avg_ms"], "launches_timed": dom["launches_timed"],
            "sample": f"one launch in {PROF_STRIDE} of the stage timed with HIP events over the timed region",
            "algorithmic_bytes_per_launch": dom["algorithmic_bytes"]}
    # for scale, outside the timed region: what a plain device copy streams here
    src = torch.empty(1 << 28, device=dev, dtype=torch.float32)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    roof["copy_GBps"] = 5 * 2 * src.numel() * 4 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    roof["copy_sample"] = "torch device copy of 1 GiB (2 GiB moved), 5 times, events on the current stream"
    del src, dst
    # MFMA work of the fifth-dimension epilogue: useful dense flops (one real
    # Ls x Ls matrix per chirality on the 12 reals of that chirality: 48 Ls
    # flops per 5D site and matrix; the centre-field matrix of h2 only on the
    # centre region, where that field lives) against the FP16 MFMA peak
    nC, nN1, nN2 = regions
    mats = {11: nN1, 12: nN2 + nC, 13: nN1, 14: 2 * nC}
    mfma = {}
    for k, n4 in mats.items():
        if str(k) in kernels:
            fl = 48 * cfg.Ls * cfg.Ls * n4 * cfg.n_subdomains
            tf = fl / (kernels[str(k)]["avg_ms"] * 1e-3) / 1e12
            mfma[str(k)] = {"useful_flops_per_launch": fl, "TFLOPs": tf, "peak_TFLOPs": MFMA_F16_PEAK_TFLOPS,
                            "frac": tf / MFMA_F16_PEAK_TFLOPS}
    outer_b = sum(sbytes[k] for k in (21, 22, 23, 24)) / 4
    inner_b = sum(sbytes[k] for k in (11, 12, 13, 14)) / 4
    avg_out = ms_out / max(n_out, 1)
    avg_in = ms_in / max(n_in, 1)
    gbs_out = outer_b / (avg_out * 1e-3) / 1e9 if n_out else None
    gbs_in = inner_b / (avg_in * 1e-3) / 1e9 if n_in else None
    ms_per_step = 1000.0 * total / args.steps
    line = {
        "metric": METRIC,
        "value": ms_per_step / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name}: {cfg.note}", "lattice": list(cfg.dims), "Ls": cfg.Ls,
                   "mf": cfg.mf, "eps": cfg.eps, "subdomain": list(cfg.sub), "inner_iters": cfg.inner_iters,
                   "inner_prec": inner, "outer_prec": cfg.outer_prec, "tol": cfg.tol,
                   "parallelism": "single GPU, 256 virtual subdomains"},
        "mspcg": {"time_s_median": statistics.median(times), "outer_iters": sts[-1].outer_iters,
                  "inner_iters_total": sts[-1].inner_iters_total, "reliable_updates": sts[-1].reliable_updates,
                  "true_rel_resid": sts[-1].true_rel_resid,
                  "precond_ms_per_solve": ms_pc / args.steps},
        "cg_fp32": None if cg32 is None else {"time_s": cg32[-1][0], "outer_iters": cg32[-1][1].outer_iters,
                                              "true_rel_resid": cg32[-1][1].true_rel_resid},
        "cg_fp64": None if cg64 is None else {"time_s": cg64[-1][0], "outer_iters": cg64[-1][1].outer_iters,
                                              "true_rel_resid": cg64[-1][1].true_rel_resid},
        "inner_storage": storage,
        "speedup_vs_cg_fp32": None if cg32 is None else cg32[-1][0] / statistics.median(times),
        "speedup_vs_cg_fp64": None if cg64 is None else cg64[-1][0] / statistics.median(times),
        ("solution_rel_diff_mspcg_vs_cg64" if cg64 is not None else "solution_rel_diff_mspcg_vs_cg32"): sol_rel,
        "kernels": kernels,
        "dslash": {"outer_hop_GBps": gbs_out, "outer_hop_avg_ms": avg_out, "outer_launches_timed": n_out,
                   "inner_hop_GBps": gbs_in, "inner_hop_avg_ms": avg_in, "inner_launches_timed": n_in,
                   "outer_hop_ms_total_est": ms_out * PROF_STRIDE, "inner_hop_ms_total_est": ms_in * PROF_STRIDE,
                   "regions_C_N1_N2": regions},
        "roofline": roof,
        "mfma_epilogue": mfma,
        "p50_p99": None,
    }
    if args.oracle_check:
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        import oracle
        x = x_ms.cpu().numpy().view(np.complex128).reshape(b.shape)
        log("[bench] oracle residual of the MSPCG solution: applying A on the host")
        t = time.perf_counter()
        op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
        r = b - op.A(x)
        res = float(np.linalg.norm(r) / np.linalg.norm(b))
        log(f"[bench] oracle residual {res:.3e} ({time.perf_counter() - t:.1f}s)")
        line["mspcg"]["oracle_rel_resid"] = res
    if "sample" in cpu:
        line["cpu_baseline"] = cpu_baseline(cfg, cpu["sample"], sts[-1].outer_iters,
                                            None if cg32 is None else cg32[-1][1].outer_iters)
    elif "error" in cpu:
        line["cpu_baseline"] = {"error": cpu["error"]}
    if args.serve_sample > 0 and fits("serving_sample", 30.0):
        del s
        r = serve_stream(nreq=args.serve_sample, **SERVE_SAMPLE)
        r.pop("_svc")
        line["p50_p99"] = {"p50_s": r["p50_s"], "p99_s": r["p99_s"], "solves_per_s": r["solves_per_s"],
                           "sample": "serving sample, continuous batching: Poisson stream of %d requests over "
                                     "8^4x8, "
                                     "mf in {0.1, 0.01}, 1-3 RHS each, load %.2f of the measured sequential capacity"
                                     % (r["requests"], r["load"]),
                           "detail": r}

    line["skipped_for_time"] = skipped
    line["run_s"] = time.time() - T_BEGIN
    print(json.dumps(line), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(cfg, U, b):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    solve: one application of the full A and the k-step inner CG of one
    subdomain (its A_s through the padded field, Sec. 3.1.2), with all
    threads, and one A_s application again with one thread."""
    os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
    from threadpoolctl import threadpool_info, threadpool_limits
    import oracle
    op = oracle.MobiusDWF(U, cfg.Ls, cfg.b, cfg.c, cfg.M5, cfg.mf)
    til = oracle.Tiling(cfg.dims, cfg.sub)
    t = time.perf_counter()
    op.A(b)
    t_A = time.perf_counter() - t
    log(f"[bench] oracle: A in {t_A:.2f}s")
    t = time.perf_counter()
    oracle.inner_cg(op, til, b, cfg.inner_iters, subset=[0], padded=True)
    t_pc1 = time.perf_counter() - t
    log(f"[bench] oracle: inner CG (k={cfg.inner_iters}) on 1 subdomain in {t_pc1:.2f}s")
    pools = threadpool_info()
    threads = max([p.get("num_threads", 1) for p in pools] + [1])
    # one A_s application of the same subdomain, with all threads and with one
    vs = til.restrict(b)[:1]
    t = time.perf_counter()
    oracle.local_operator(op, til, vs, subset=[0], padded=True)
    t_as = time.perf_counter() - t
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        oracle.local_operator(op, til, vs, subset=[0], padded=True)
        t_as_1 = time.perf_counter() - t
    log(f"[bench] oracle: one A_s application {t_as:.3f}s, on 1 thread {t_as_1:.3f}s")
    return {"t_A": t_A, "t_pc1": t_pc1, "t_as": t_as, "t_as_1": t_as_1, "threads": threads, "nsub": til.nsub}


def cpu_baseline(cfg, smp, mspcg_iters, cg_iters):
    """The CPU sample scaled to a time-to-solution: the GPU's outer iteration
    count times (one A + the inner CG of every subdomain)."""
    t_A, t_pc1, t_as, t_as_1, threads = smp["t_A"], smp["t_pc1"], smp["t_as"], smp["t_as_1"], smp["threads"]
    nsub = smp["nsub"]
    per_iter = t_A + t_pc1 * nsub
    out = {"value": per_iter * mspcg_iters, "unit": "s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "cpu_count": os.cpu_count(),
           "sample": (f"one oracle A application ({t_A:.2f}s) and the k={cfg.inner_iters} inner CG of 1 of "
                      f"{nsub} subdomains through its padded field ({t_pc1:.2f}s), {threads} threads, timed "
                      f"while the GPU ran its untimed warmup solves; extrapolated to {nsub} subdomains and "
                      f"the GPU's {mspcg_iters} outer iterations"),
           "one_thread": {"A_s_one_subdomain_s": t_as_1, "A_s_one_subdomain_all_threads_s": t_as,
                          "threads_speedup": t_as_1 / t_as,
                          "value_extrapolated_s": per_iter * (t_as_1 / t_as) * mspcg_iters,
                          "sample": "one A_s application through the padded field on 1 thread against all "
                                    "threads; the whole solve scaled by that ratio"}}
    if cg_iters is not None:
        out["cg_fp64_extrapolated_s"] = t_A * cg_iters
    return out


if __name__ == "__main__":
    main()
