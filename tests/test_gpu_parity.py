"""GPU parity: every operator of the C ABI against the FP64 oracle.

Inputs are seeded (workloads/); the oracle computes the same operator from
its definition on the CPU.  Two measures are checked for every output: the
relative L2 error of the whole field, and the largest error of one 5D site
(its 24 reals) relative to the largest site of the reference, so that a
small wrong region (a face, a subdomain, one site block) cannot hide under a
whole-field norm.  Bounds against the exact operator: FP64 1e-12, FP32 1e-6,
FP16 3e-3 (a single hop 1.5e-3), BF16 3e-2, INT8 1e-1 -- the FP32 and FP16
bounds are the ones fixed for operator applications; BF16 has 3 fewer
mantissa bits than FP16 and gets 8x the FP16 bound; INT8 rounds each real to
a step of m/127 (m the site's largest magnitude), about 5e-3 per store of a
Gaussian field, and keeps the same multiple of its one-store error.

The local operator and the preconditioner in the 16- and 8-bit formats get
bounds from the error the format itself causes on the test's input: the
oracle's model of the format (``oracle.local_operator_stored`` /
``oracle.inner_cg_stored``: every field a kernel writes stored in the format,
FP16 links) against the exact operator, times 2.5, plus an allowance for the
fifth-dimension epilogue's FP16 operands (each value within 2^-12 of its site
column's largest, which the model leaves out).  Each test asserts that this
bound is well below the share of the snake terms (Sec. 2.3, eq. diri) in that
operator on that tiling, measured with the oracle's per-hop truncated
operator: an implementation that dropped them could not pass.  (The model is
not compared with the GPU directly: the epilogue's rounding, relative to a
site column's largest value, moves the small fifth-dimension slices of a
site by more than one step of the 8-bit and BF16 formats, so those
rounding decisions are independent of the model's.)
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

TOL_A = {"fp64": 1e-12, "fp32": 1e-6, "fp16": 3e-3, "bf16": 3e-2, "int8": 1e-1}
TOL_HOP = {"fp64": 1e-13, "fp32": 1e-6, "fp16": 1.5e-3, "bf16": 1.2e-2, "int8": 4.5e-2}

LATTICES = [
    # dims, Ls : covers a ragged last block (V/2 not a multiple of the block's
    # sites), odd Ls, the degenerate 2^4 lattice and unequal extents; the
    # MFMA epilogue's one-, two-, three- and four-wavefront schedules (Ls up
    # to 4, 5..8, 9..12, 13..16), each with an Ls that is not a multiple of 4
    ((4, 4, 4, 4), 4),
    ((6, 4, 2, 8), 5),
    ((2, 2, 2, 2), 3),
    ((8, 8, 8, 8), 8),
    ((4, 2, 6, 4), 12),
    ((2, 4, 2, 4), 11),
    ((4, 4, 2, 2), 16),
    ((2, 2, 4, 2), 14),
]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def site_rel(a, b):
    """max over 5D sites of |a - b| over the site, relative to the largest
    site norm of b (a site is the 4 x 3 complex components)"""
    d = np.linalg.norm((a - b).reshape(-1, 12), axis=1)
    return float(d.max() / np.linalg.norm(b.reshape(-1, 12), axis=1).max())


# the largest single-site error allowed, as a multiple of the field's L2 bound
SITE = 4.0
# allowance for the epilogue's FP16 operands (measured ~3e-4 for one A_s,
# ~5e-4 for the k = 3 preconditioner, FP16 storage)
EPI = {"A_sub": 1e-3, "precond": 2e-3}


def format_bound(kind, model_err):
    """2.5 x the format's own error on the input, plus the epilogue allowance."""
    return 2.5 * model_err + EPI[kind]


def check(got, ref, tol, what):
    e, es = rel(got, ref), site_rel(got, ref)
    assert e < tol and es < SITE * tol, (what, e, es, tol)
    return e, es


def rand_field(Ls, vh, seed):
    g = np.random.default_rng(seed).standard_normal((Ls, vh, 4, 3, 2))
    return g[..., 0] + 1j * g[..., 1]


_cache = {}


def setup(dims, Ls, mf=0.1, eps=0.5, seed=11, sub=None):
    from paper_2104_05615_amd import MSPCG
    key = (dims, Ls, mf, eps, seed, sub)
    if key not in _cache:
        U = W.gauge_field(dims, eps, seed)
        s = MSPCG(dims)
        s.load_gauge(U)
        s.set_mobius(Ls, 1.5, 0.5, 1.8, mf)
        if sub is not None:
            s.set_subdomains(sub)
        op = oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, mf)
        _cache[key] = (s, op, U)
    return _cache[key]


# ---------------------------------------------------------------- hopping term

@pytest.mark.parametrize("dims,Ls", LATTICES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "int8"])
def test_dslash_parity(dims, Ls, prec):
    s, op, U = setup(dims, Ls)
    psi = rand_field(Ls, op.vh, 3)
    for name, par, dag in (("dslash_eo", 0, False), ("dslash_oe", 1, False),
                           ("dslash_dag_eo", 0, True), ("dslash_dag_oe", 1, True)):
        say(f"[gpu] {name} {prec} dims={dims} Ls={Ls}")
        got = s.apply(name, prec, psi)
        ref = oracle.wilson_hop(U, psi, par, dagger=dag)
        check(got, ref, TOL_HOP[prec], (name, prec))


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 8), ((4, 2, 6, 4), 12), ((6, 4, 2, 8), 5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
def test_fifth_dimension_ops(dims, Ls, prec):
    s, op, U = setup(dims, Ls, mf=0.05)
    psi = rand_field(Ls, op.vh, 5)
    tol = {"fp64": 1e-13, "fp32": 1e-6, "fp16": 1.5e-3}[prec]
    for name, M in (("m5", op.M5op), ("m5inv", op.M5inv), ("mphi", op.Mphi)):
        say(f"[gpu] {name} {prec} dims={dims} Ls={Ls}")
        got = s.apply(name, prec, psi)
        check(got, oracle.apply5(M, psi), tol, (name, prec))


# ---------------------------------------------------------------- D, D^dag, A

@pytest.mark.parametrize("dims,Ls", LATTICES)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "int8"])
def test_schur_and_normal_operator(dims, Ls, prec):
    s, op, U = setup(dims, Ls)
    psi = rand_field(Ls, op.vh, 7)
    for name, f in (("D", op.D), ("Ddag", op.Ddag), ("A", op.A)):
        say(f"[gpu] {name} {prec} dims={dims} Ls={Ls}")
        got = s.apply(name, prec, psi)
        check(got, f(psi), TOL_A[prec], (name, prec))


@pytest.mark.parametrize("dims,Ls", [((4, 4, 4, 4), 4), ((6, 4, 2, 8), 5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "int8"])
def test_storage_round_trip(dims, Ls, prec):
    """A field stored in each format and read back against the oracle's
    definition of the format: FP64 and FP32 exact; the scaled formats take
    the same FP32 rounding decisions, so every real agrees up to the FP32
    rounding of the read-back product (a few ulp of the site's largest
    real; a different code would differ by a whole step).  Sites spanning
    16 orders of magnitude, and zero sites, are included."""
    s, op, U = setup(dims, Ls)
    psi = rand_field(Ls, op.vh, 17) * np.exp(np.random.default_rng(18).uniform(-18, 18, (Ls, op.vh, 1, 1)))
    psi[0, :3] = 0
    say(f"[gpu] store {prec} dims={dims} Ls={Ls}")
    got = s.apply("store", prec, psi)
    ref = oracle.stored(psi, prec)
    if prec in ("fp64", "fp32"):
        assert np.array_equal(got, ref)
        return
    g = np.stack([got.real, got.imag], -1).reshape(got.shape[:-2] + (24,))
    r = np.stack([ref.real, ref.imag], -1).reshape(ref.shape[:-2] + (24,))
    m = np.max(np.abs(r), axis=-1, keepdims=True)
    assert np.all(np.abs(g - r) <= 2.0 ** -21 * m)
    assert np.array_equal(g[0, :3], np.zeros_like(g[0, :3]))


def test_gpu_normal_operator_hermitian_positive():
    s, op, U = setup((8, 8, 8, 8), 8)
    x, y = rand_field(8, op.vh, 21), rand_field(8, op.vh, 23)
    say("[gpu] A hermiticity fp64")
    Ax, Ay = s.apply("A", "fp64", x), s.apply("A", "fp64", y)
    a, b = np.vdot(x, Ay), np.vdot(Ax, y)
    assert abs(a - b) < 1e-12 * abs(a)
    q = np.vdot(x, Ax)
    assert q.real > 0 and abs(q.imag) < 1e-12 * q.real


# ---------------------------------------------------------------- local operator and preconditioner

SUBS = [
    ((8, 4, 4, 4), 4, (4, 4, 4, 4)),
    ((8, 8, 4, 2), 6, (4, 4, 4, 2)),
    ((12, 4, 2, 2), 3, (4, 4, 2, 2)),
    ((8, 8, 8, 8), 8, (4, 4, 4, 4)),
    ((8, 4, 4, 8), 12, (4, 4, 4, 4)),   # the benchmark's Ls: 16-bit terms on 4 x 4 x 4 MFMA blocks
    ((8, 4, 2, 4), 16, (4, 4, 2, 4)),   # four-wavefront epilogue
]


_share = {}


def snake_share(dims, Ls, sub, what):
    """Share of the snake terms: the relative change of A_s r_s (or of the
    k = 3 preconditioner) when the Dirichlet cut is applied to every hop
    instead of to the whole operator (eq. diri), on the tests' inputs."""
    key = (dims, Ls, sub, what)
    if key not in _share:
        import oracle.dwf as D
        s, op, U = setup(dims, Ls, sub=sub)
        til = oracle.Tiling(dims, sub)
        if what == "A_sub":
            vs = til.restrict(rand_field(Ls, op.vh, 9))
            _share[key] = rel(oracle.truncated_local_operator(op, til, vs), oracle.local_operator(op, til, vs))
        else:
            r = rand_field(Ls, op.vh, 13)
            z = oracle.inner_cg(op, til, r, 3)
            real = D.local_operator
            D.local_operator = lambda o, t, v, subset=None, batch=8, padded=False: \
                D.truncated_local_operator(o, t, v, subset=subset)
            try:
                zt = oracle.inner_cg(op, til, r, 3)
            finally:
                D.local_operator = real
            _share[key] = rel(zt, z)
    return _share[key]


def model_op(op, prec):
    """The oracle operator on the links as the 16- and 8-bit kernels hold them."""
    return oracle.MobiusDWF(oracle.stored_links(op.U, prec), op.Ls, op.b, op.c, op.M5, op.mf)


@pytest.mark.parametrize("dims,Ls,sub", SUBS)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16", "bf16", "int8"])
def test_local_operator_parity(dims, Ls, sub, prec):
    s, op, U = setup(dims, Ls, sub=sub)
    til = oracle.Tiling(dims, sub)
    r = rand_field(Ls, op.vh, 9)
    say(f"[gpu] A_sub {prec} dims={dims} sub={sub} Ls={Ls}")
    got = s.apply("A_sub", prec, r)
    vs = til.restrict(r)
    ex = oracle.local_operator(op, til, vs)
    ref = til.prolong(ex, op.vh)
    tol = TOL_A[prec]
    if prec in ("fp16", "bf16", "int8"):
        share = snake_share(dims, Ls, sub, "A_sub")
        model_err = rel(oracle.local_operator_stored(model_op(op, prec), til, vs, prec), ex)
        tol = min(tol, format_bound("A_sub", model_err))
        assert tol < share / 2.5, (tol, share)
    e, es = check(got, ref, tol, prec)
    if prec in ("fp16", "bf16", "int8"):
        say(f"      {e:.2e} (worst site {es:.2e}), bound {tol:.2e} (format alone {model_err:.2e}), "
            f"snake share {share:.3f}")


@pytest.mark.parametrize("dims,Ls,sub", SUBS)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5), ("fp16", 3e-2), ("bf16", 2e-1),
                                      ("int8", 5e-1)])
def test_preconditioner_parity(dims, Ls, sub, prec, tol):
    """k = 3 inner CG steps per subdomain.  The inner CG is nonlinear in its
    input; against the exact preconditioner low-precision storage perturbs
    its scalars, so FP16/BF16/INT8 get a looser bound there than a single
    operator application; the 16- and 8-bit formats are held to 2.5x the
    error the format itself causes (the oracle's model), far below the
    snake terms' share of the preconditioner."""
    s, op, U = setup(dims, Ls, sub=sub)
    s.set_solver(inner_iters=3)
    til = oracle.Tiling(dims, sub)
    r = rand_field(Ls, op.vh, 13)
    say(f"[gpu] precond {prec} dims={dims} sub={sub} Ls={Ls}")
    got = s.apply("precond", prec, r)
    ref = oracle.precondition(op, til, r, 3)
    if prec in ("fp16", "bf16", "int8"):
        share = snake_share(dims, Ls, sub, "precond")
        model = til.prolong(oracle.inner_cg_stored(model_op(op, prec), til, r, 3, prec), op.vh)
        model_err = rel(model, ref)
        tol = min(tol, format_bound("precond", model_err))
        assert tol < share / 2.5, (tol, share)
    e, es = check(got, ref, tol, prec)
    if prec in ("fp16", "bf16", "int8"):
        say(f"      {e:.2e} (worst site {es:.2e}), bound {tol:.2e} (format alone {model_err:.2e}), "
            f"snake share {share:.3f}")


def test_preconditioner_locality():
    """Subdomains do not communicate: changing r outside subdomain 0 leaves z
    on subdomain 0 bit-identical (deterministic kernels)."""
    dims, Ls, sub = (8, 8, 8, 8), 8, (4, 4, 4, 4)
    s, op, U = setup(dims, Ls, sub=sub)
    s.set_solver(inner_iters=4)
    til = oracle.Tiling(dims, sub)
    r = rand_field(Ls, op.vh, 31)
    r2 = r.copy()
    r2[:, til.index[5]] *= -3.0
    for prec in ("fp32", "fp16"):
        say(f"[gpu] precond locality {prec}")
        z1 = s.apply("precond", prec, r)
        z2 = s.apply("precond", prec, r2)
        assert np.array_equal(z1[:, til.index[0]], z2[:, til.index[0]])
        assert not np.array_equal(z1[:, til.index[5]], z2[:, til.index[5]])
        z3 = s.apply("precond", prec, r)
        assert np.array_equal(z1, z3)


# ---------------------------------------------------------------- solves

def oracle_resid(op, b, x):
    return float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))


@pytest.mark.parametrize("outer,inner", [("fp64", "fp64"), ("fp32", "fp32"), ("fp32", "fp16"), ("fp32", "bf16"),
                                         ("fp32", "int8")])
def test_mspcg_solve_small(outer, inner):
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op, U = setup(dims, Ls, mf=0.05, sub=sub)
    b = W.gaussian_source(dims, Ls, 41)
    s.set_solver(tol=1e-10, maxiter=2000, inner_iters=4, inner_prec=inner, outer_prec=outer)
    say(f"[gpu] mspcg solve outer={outer} inner={inner}")
    x, st = s.solve(b)
    res = oracle_resid(op, b, x)
    say(f"      iters={st.outer_iters} RU={st.reliable_updates} lib={st.true_rel_resid:.2e} oracle={res:.2e}")
    assert st.status == 0
    assert res < 2e-10 and st.true_rel_resid <= 1e-10
    assert abs(res - st.true_rel_resid) < 1e-11
    if outer == "fp64" and inner == "fp64":
        til = oracle.Tiling(dims, sub)
        _, info = oracle.mspcg(op, til, b, 4, 1e-10, 2000)
        say(f"      oracle iters={info.iters}")
        assert abs(info.iters - st.outer_iters) <= 2


@pytest.mark.parametrize("outer", ["fp64", "fp32"])
def test_plain_cg_solve(outer):
    dims, Ls = (8, 4, 4, 4), 4
    s, op, U = setup(dims, Ls, mf=0.05, sub=(4, 4, 4, 4))
    b = W.gaussian_source(dims, Ls, 43)
    s.set_solver(tol=1e-10, maxiter=5000, outer_prec=outer, use_precond=False, beta_rule="FR")
    say(f"[gpu] cg solve {outer}")
    x, st = s.solve(b)
    res = oracle_resid(op, b, x)
    say(f"      iters={st.outer_iters} RU={st.reliable_updates} oracle={res:.2e}")
    assert st.status == 0 and res < 2e-10
    if outer == "fp64":
        _, info = oracle.cg(op, b, 1e-10, 5000)
        assert abs(info.iters - st.outer_iters) <= 2


def test_c1_fp64_mspcg_matches_oracle_solution():
    """8^4 x Ls8, 16 subdomains of 4^4, k = 5, FP64 throughout.  The oracle
    checks the residual of the GPU solution; the solution agrees with the
    oracle's CG solution (tests/golden/reference_c1.json, sampled entries) to
    the kappa * tol that the conditioning allows."""
    import json
    import os
    from workloads.configs import CONFIGS
    c = CONFIGS["c1"]
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_c1.json")))
    s, op, U = setup(c.dims, c.Ls, mf=c.mf, eps=c.eps, seed=c.gauge_seed, sub=c.sub)
    b = W.gaussian_source(c.dims, c.Ls, c.src_seed)
    tol = 1e-10
    s.set_solver(tol=tol, maxiter=2000, inner_iters=c.inner_iters, inner_prec="fp64", outer_prec="fp64")
    say("[gpu] c1 mspcg fp64")
    x, st = s.solve(b)
    say(f"      gpu iters={st.outer_iters}, oracle cg iters={ref['iters']}, kappa={ref['kappa']:.1f}")
    assert st.status == 0 and oracle_resid(op, b, x) < 2e-10
    n = x.size
    d = np.array([x[i0, i1, i2, i3] - complex(re, im) for i0, i1, i2, i3, re, im in ref["samples"]])
    rms_rel = np.sqrt(np.mean(np.abs(d) ** 2)) / (ref["x_norm"] / np.sqrt(n))
    say(f"      sampled relative error {rms_rel:.2e} (bound kappa*tol = {ref['kappa'] * tol:.2e})")
    assert rms_rel < 2 * ref["kappa"] * tol
    assert st.outer_iters < ref["iters"]


def test_c1_fp64_residual_history_matches_the_oracle():
    """The iterated relative residual |r_k| / |b| of the first 20 outer
    iterations (the quantity of Fig. residual-rbc and Fig. residual-cal) of
    the FP64 MSPCG solve on the 8^4 x Ls8 workload agrees with the oracle's
    MSPCG (same tiling, k = 5, PR beta) to 1e-8 relative; both start at 1."""
    from workloads.configs import CONFIGS
    c = CONFIGS["c1"]
    s, op, U = setup(c.dims, c.Ls, mf=c.mf, eps=c.eps, seed=c.gauge_seed, sub=c.sub)
    b = W.gaussian_source(c.dims, c.Ls, c.src_seed)
    s.set_solver(tol=1e-10, maxiter=2000, inner_iters=c.inner_iters, inner_prec="fp64", outer_prec="fp64")
    say("[gpu] c1 mspcg fp64: residual history")
    x, st = s.solve(b)
    h = s.history()
    assert st.status == 0 and len(h) == st.outer_iters + 1
    til = oracle.Tiling(c.dims, c.sub)
    _, info = oracle.mspcg(op, til, b, c.inner_iters, 1e-10, 20)
    ref = np.array(info.history[:21])
    got = h[:21]
    d = np.max(np.abs(got - ref) / ref)
    say(f"      first 21 residuals: max relative difference {d:.2e} (|r_20|/|b| = {ref[-1]:.3e})")
    assert got[0] == 1.0 and ref[0] == 1.0
    assert d < 1e-8, d


def lanczos_extremes(alphas, betas):
    """Extreme eigenvalues of the Lanczos matrix of CG (diagonal
    1/alpha_i + beta_{i-1}/alpha_{i-1}, off-diagonal sqrt(beta_i)/alpha_i)."""
    n = len(alphas)
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = 1 / alphas[i] + (betas[i - 1] / alphas[i - 1] if i > 0 else 0.0)
        if i + 1 < n:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(betas[i]) / alphas[i]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def test_c1_extreme_eigenvalues_from_the_cg_coefficients():
    """The FP64 plain CG solve to 1e-12 on the 8^4 x Ls8 workload gives,
    through the exported residuals and <p, A p>, the CG coefficients whose
    Lanczos matrix estimates the extreme eigenvalues of A; they agree with
    the oracle's estimate from its own CG (tests/golden/reference_c1.json)."""
    import json
    import os
    from workloads.configs import CONFIGS
    c = CONFIGS["c1"]
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "reference_c1.json")))
    s, op, U = setup(c.dims, c.Ls, mf=c.mf, eps=c.eps, seed=c.gauge_seed, sub=c.sub)
    b = W.gaussian_source(c.dims, c.Ls, c.src_seed)
    s.set_solver(tol=1e-12, maxiter=2000, outer_prec="fp64", use_precond=False, beta_rule="FR", reliable_delta=0.0)
    say("[gpu] c1 plain CG fp64 to 1e-12: Lanczos extremes")
    x, st = s.solve(b)
    h, pap = s.history(pap=True)
    rho = h ** 2
    alphas = rho[:-1] / pap
    betas = rho[1:-1] / rho[:-2]
    lmin, lmax = lanczos_extremes(alphas, betas)
    say(f"      {st.outer_iters} iterations (oracle {ref['iters']}), lambda_min {lmin:.6e} ({ref['lambda_min']:.6e}), "
        f"lambda_max {lmax:.6e} ({ref['lambda_max']:.6e})")
    assert st.status == 0 and abs(st.outer_iters - ref["iters"]) <= 2
    assert abs(lmin / ref["lambda_min"] - 1) < 1e-6 and abs(lmax / ref["lambda_max"] - 1) < 1e-6


def test_gauge_invariance_of_solve():
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    from paper_2104_05615_amd import MSPCG
    U = W.gauge_field(dims, 0.5, 61)
    Om = W.random_gauge_transform(dims, 62)
    b = W.gaussian_source(dims, Ls, 63)
    from workloads.fields import gauge_transform_field
    out = []
    for UU, bb in ((U, b), (W.gauge_transform_links(U, Om), gauge_transform_field(b, Om, 0))):
        s = MSPCG(dims)
        s.load_gauge(UU)
        s.set_mobius(Ls, 1.5, 0.5, 1.8, 0.05)
        s.set_subdomains(sub)
        s.set_solver(tol=1e-10, maxiter=1000, inner_iters=4, inner_prec="fp64", outer_prec="fp64")
        say("[gpu] gauge invariance solve")
        out.append(s.solve(bb))
    (x1, s1), (x2, s2) = out
    assert s1.outer_iters == s2.outer_iters
    assert rel(gauge_transform_field(x1, Om, 0), x2) < 1e-8


def test_zero_and_nonfinite_source_and_maxiter():
    from paper_2104_05615_amd import MSPCGError, MSPCG_ERR_BREAKDOWN, MSPCG_NOT_CONVERGED
    dims, Ls = (8, 4, 4, 4), 4
    s, op, U = setup(dims, Ls, mf=0.05, sub=(4, 4, 4, 4))
    s.set_solver(tol=1e-10, maxiter=100, inner_iters=2)
    say("[gpu] zero source")
    x, st = s.solve(np.zeros((Ls, op.vh, 4, 3), dtype=complex))
    assert st.status == 0 and np.all(x == 0)
    b = W.gaussian_source(dims, Ls, 71)
    b[0, 0, 0, 0] = np.nan
    say("[gpu] nan source")
    with pytest.raises(MSPCGError) as e:
        s.solve(b)
    assert e.value.status == MSPCG_ERR_BREAKDOWN
    s.set_solver(tol=1e-10, maxiter=3, inner_iters=2)
    say("[gpu] maxiter 3")
    x, st = s.solve(W.gaussian_source(dims, Ls, 72))
    assert st.status == MSPCG_NOT_CONVERGED and st.outer_iters == 3
    assert abs(oracle_resid(op, W.gaussian_source(dims, Ls, 72), x) - st.true_rel_resid) < 1e-9


def test_warm_start_and_device_buffers():
    import torch
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op, U = setup(dims, Ls, mf=0.05, sub=sub)
    b = W.gaussian_source(dims, Ls, 81)
    s.set_solver(tol=1e-10, maxiter=2000, inner_iters=4)
    say("[gpu] device buffers solve")
    bt = torch.from_numpy(b.view(np.float64).copy()).cuda()
    xt = torch.empty_like(bt)
    st = s.solve_device(bt.data_ptr(), xt.data_ptr())
    x = xt.cpu().numpy().view(np.complex128).reshape(b.shape)
    assert st.status == 0 and oracle_resid(op, b, x) < 2e-10
    # warm start from the solution: converges at once
    x2, st2 = s.solve(b, x0=x)
    assert st2.status == 0 and st2.outer_iters <= 1


def test_profiling_counters():
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op, U = setup(dims, Ls, mf=0.05, sub=sub)
    s.set_solver(tol=1e-8, maxiter=500, inner_iters=3)
    s.set_profiling(True)
    say("[gpu] profiled solve")
    x, st = s.solve(W.gaussian_source(dims, Ls, 91))
    n0, ms0 = s.kernel_time(0)
    n1, ms1 = s.kernel_time(1)
    s.set_profiling(False)
    assert n0 >= 4 * st.outer_iters and ms0 > 0
    assert n1 == 4 * 3 * st.outer_iters and ms1 > 0
    # sampled: one launch in 4 of each subdomain hop stage (3 inner
    # iterations per outer one, each stage once per inner iteration)
    s.set_profiling(True, stride=4)
    say("[gpu] profiled solve, one launch in 4")
    x2, st2 = s.solve(W.gaussian_source(dims, Ls, 91))
    n1s, ms1s = s.kernel_time(1)
    n12, _ = s.kernel_time(12)
    s.set_profiling(False)
    assert np.array_equal(x2, x) and st2.outer_iters == st.outer_iters
    assert n12 == (3 * st.outer_iters + 3) // 4 and n1s == 4 * n12 and ms1s > 0


# ---------------------------------------------------------------- vector-ALU epilogue

@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("Ls,mfma", [(20, True), (12, False)])
def test_vector_alu_epilogue_paths(prec, Ls, mfma):
    """The fifth-dimension epilogue on the vector ALUs: always for Ls > 16,
    and for every Ls with the MFMA engine switched off (mspcg_set_mfma)."""
    import paper_2104_05615_amd as M
    dims, sub = (8, 4, 4, 4), (4, 4, 4, 4)
    U = W.gauge_field(dims, 0.5, 31)
    op = oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, 0.1)
    til = oracle.Tiling(dims, sub)
    psi = rand_field(Ls, op.vh, 33)
    M.mspcg_set_mfma(1 if mfma else 0)
    try:
        s = M.MSPCG(dims)
        s.load_gauge(U)
        s.set_mobius(Ls, 1.5, 0.5, 1.8, 0.1)
        s.set_subdomains(sub)
        say(f"[gpu] VALU epilogue {prec} Ls={Ls} mfma={mfma}")
        check(s.apply("A", prec, psi), op.A(psi), TOL_A[prec], ("A", prec))
        got = s.apply("A_sub", prec, psi)
        ref = til.prolong(oracle.local_operator(op, til, til.restrict(psi)), op.vh)
        check(got, ref, TOL_A[prec], ("A_sub", prec))
        s.close()
    finally:
        M.mspcg_set_mfma(1)


# ---------------------------------------------------------------- full 5D system

@pytest.mark.parametrize("outer,inner", [("fp64", "fp64"), ("fp32", "fp16")])
def test_full_five_dimensional_solve(outer, inner):
    """M psi = phi on both parities through the even-odd Schur complement:
    the oracle applies the unpreconditioned block operator [[M5, M4_eo],
    [M4_oe, M5]] to the library's (psi_e, psi_o); the odd half equals the
    oracle's reconstruction from psi_e."""
    dims, Ls, sub = (8, 4, 4, 4), 4, (4, 4, 4, 4)
    s, op, U = setup(dims, Ls, mf=0.05, sub=sub)
    phi_e, phi_o = rand_field(Ls, op.vh, 51), rand_field(Ls, op.vh, 52)
    s.set_solver(tol=1e-12, maxiter=4000, inner_iters=4, inner_prec=inner, outer_prec=outer)
    say(f"[gpu] full 5D solve outer={outer} inner={inner}")
    psi_e, psi_o, st, res = s.solve_full(phi_e, phi_o)
    me, mo = op.full(psi_e, psi_o)
    r = np.sqrt((np.linalg.norm(phi_e - me) ** 2 + np.linalg.norm(phi_o - mo) ** 2)
                / (np.linalg.norm(phi_e) ** 2 + np.linalg.norm(phi_o) ** 2))
    say(f"      even solve {st.outer_iters} iterations, full residual oracle {r:.2e} library {res:.2e}")
    assert st.status == 0
    assert r < 1e-9 and abs(r - res) < 1e-11
    assert rel(psi_o, op.reconstruct_odd(psi_e, phi_o)) < 1e-12


# ---------------------------------------------------------------- block orders

def test_block_orders_of_full_lattice_hops_keep_results():
    """The chunked time-slice sweeps of the full-lattice hops (mspcg_set_schedule,
    tchunk 1..4) visit the same site blocks as the lexicographic order: A in
    FP32 and FP64 and an MSPCG solve (whose <p, Ap> is fused into the last
    hop, one partial per site block) are bit-identical under every order."""
    from paper_2104_05615_amd import KIND_FP64, KIND_OUTER, MSPCG
    dims, Ls, sub = (8, 8, 8, 8), 8, (4, 4, 4, 4)
    U = W.gauge_field(dims, 0.5, 43)
    op = oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, 0.1)
    s = MSPCG(dims)
    s.load_gauge(U)
    s.set_mobius(Ls, 1.5, 0.5, 1.8, 0.1)
    s.set_subdomains(sub)
    s.set_solver(tol=1e-10, maxiter=400, inner_iters=3, inner_prec="fp16", outer_prec="fp32")
    psi = rand_field(Ls, op.vh, 41)
    b = W.gaussian_source(dims, Ls, 42)
    ref = op.A(psi)
    base, xs = {}, {}
    for tchunk in range(5):
        for kind in (KIND_OUTER, KIND_FP64):
            s.set_schedule(kind, 1, order=0, xcd=1, tchunk=tchunk)
            assert s.tchunk(kind, 1) == tchunk
        say(f"[gpu] block order tchunk={tchunk}: A fp32/fp64, MSPCG solve")
        for prec in ("fp32", "fp64"):
            got = s.apply("A", prec, psi)
            if tchunk == 0:
                base[prec] = got
                assert rel(got, ref) < TOL_A[prec], prec
            else:
                assert np.array_equal(got, base[prec]), (prec, tchunk)
        x, st = s.solve(b)
        assert st.status == 0
        xs[tchunk] = x
        assert np.array_equal(x, xs[0]), tchunk
    s.close()
