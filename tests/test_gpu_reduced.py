"""GPU: the reduced-Ls preconditioner (Sec. 3.3) against the oracle.

z = (T^dag Mhat^-1 T + mu) r, the training loss chi^2 and its gradient, and
the training loop, each against the oracle's definition on the same seeded
inputs; with Lhat = Ls and T = 1 the reduced preconditioner is the full one
bit for bit; MSPCG with the reduced preconditioner reaches the FP64 true
residual, and its batched solve reproduces the single-RHS solves.
Tolerances as the full preconditioner's: FP64 1e-11, FP32 1e-5, FP16 3e-2
(relative L2); loss and gradient in FP64 1e-9.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

DIMS, LS, LH, SUB, K = (8, 4, 4, 4), 6, 3, (4, 4, 4, 4), 3
MOB = (1.5, 0.5, 1.8)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rand(shape, seed):
    g = np.random.default_rng(seed).standard_normal(shape + (2,))
    return g[..., 0] + 1j * g[..., 1]


def setup(mf=0.1, Ls=LS):
    from paper_2104_05615_amd import MSPCG
    U = W.gauge_field(DIMS, 0.5, 31)
    s = MSPCG(DIMS)
    s.load_gauge(U)
    s.set_mobius(Ls, *MOB, mf)
    s.set_subdomains(SUB)
    return s, U


def transform0(Lh, Ls, seed=5, scale=0.3):
    """A decimation (slices 0, 2, 4, .. of the full field) plus a seeded perturbation."""
    T = scale * rand((Lh, 4, Ls, 4), seed)
    for j in range(Lh):
        T[j, :, (j * Ls) // Lh, :] += np.eye(4)
    return T


def dev(arrs):
    import torch
    return torch.from_numpy(np.concatenate([np.ascontiguousarray(a).view(np.float64).ravel() for a in arrs])).cuda()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5), ("fp16", 3e-2)])
def test_reduced_preconditioner_parity(prec, tol):
    s, U = setup()
    T, mu = transform0(LH, LS), 0.1
    s.set_solver(inner_iters=K)
    s.set_reduced(LH, mu=mu, T=T)
    assert s.reduced()[0] == LH and np.array_equal(s.reduced()[1], T)
    op_hat = oracle.MobiusDWF(U, LH, *MOB, 0.1)
    til = oracle.Tiling(DIMS, SUB)
    r = rand((LS, s.vh, 4, 3), 7)
    say(f"[gpu] reduced preconditioner {prec}")
    got = s.apply("precond", prec, r)
    ref = oracle.reduced_precondition(op_hat, til, T, mu, r, K)
    e = rel(got, ref)
    say(f"      rel err {e:.2e}")
    assert e < tol


def test_reduced_identity_is_the_full_preconditioner():
    s, U = setup()
    s.set_solver(inner_iters=K)
    r = rand((LS, s.vh, 4, 3), 8)
    for prec in ("fp64", "fp32", "fp16"):
        say(f"[gpu] Lhat = Ls, T = 1, mu = 0, {prec}")
        s.set_reduced(0)
        z_full = s.apply("precond", prec, r)
        s.set_reduced(LS, mu=0.0, T=np.eye(4 * LS).reshape(LS, 4, LS, 4))
        z_red = s.apply("precond", prec, r)
        assert np.array_equal(z_full, z_red)


def test_loss_and_gradient_parity():
    s, U = setup()
    T, mu = transform0(LH, LS, seed=9), 0.2
    s.set_solver(inner_iters=K, inner_prec="fp64", outer_prec="fp64")
    s.set_reduced(LH, mu=mu, T=T)
    vs = [rand((LS, s.vh, 4, 3), 40 + i) for i in range(2)]
    vt = dev(vs)
    say("[gpu] chi^2 and gradient, FP64")
    c, g = s.reduced_loss(2, vt.data_ptr(), gradient=True)
    op = oracle.MobiusDWF(U, LS, *MOB, 0.1)
    op_hat = oracle.MobiusDWF(U, LH, *MOB, 0.1)
    til = oracle.Tiling(DIMS, SUB)
    c_ref, g_ref = oracle.chi2(op, op_hat, til, T, mu, vs, K, gradient=True)
    say(f"      chi2 {c:.10e} oracle {c_ref:.10e}; grad rel {rel(g, g_ref):.2e}")
    assert abs(c - c_ref) < 1e-9 * c_ref
    assert rel(g, g_ref) < 1e-9


def test_training_parity():
    s, U = setup()
    T0, mu = transform0(LH, LS, seed=11), 0.2
    s.set_solver(inner_iters=K, inner_prec="fp64", outer_prec="fp64")
    s.set_reduced(LH, mu=mu, T=T0)
    vs = [rand((LS, s.vh, 4, 3), 50 + i) for i in range(2)]
    vt = dev(vs)
    say("[gpu] training, 2 steps, FP64")
    hist = s.train_reduced(2, vt.data_ptr(), 2, momentum=0.5)
    T = s.reduced()[1]
    op = oracle.MobiusDWF(U, LS, *MOB, 0.1)
    op_hat = oracle.MobiusDWF(U, LH, *MOB, 0.1)
    til = oracle.Tiling(DIMS, SUB)
    T_ref, h_ref = oracle.train_transform(op, op_hat, til, T0, mu, vs, K, 2, momentum=0.5)
    say(f"      history {hist} oracle {np.array(h_ref)}; T rel {rel(T, T_ref):.2e}")
    assert np.allclose(hist, h_ref, rtol=1e-6)
    assert rel(T, T_ref) < 1e-6
    assert hist[-1] < hist[0]


def test_mspcg_with_reduced_preconditioner_converges_and_batches():
    s, U = setup(mf=0.05)
    op = oracle.MobiusDWF(U, LS, *MOB, 0.05)
    s.set_solver(tol=1e-10, maxiter=4000, inner_iters=4, inner_prec="fp16", outer_prec="fp32")
    s.set_reduced(LH, mu=0.3, T=transform0(LH, LS, scale=0.0))
    bs = [W.gaussian_source(DIMS, LS, 60 + i) for i in range(3)]
    say("[gpu] MSPCG, reduced-Ls preconditioner, single solves")
    singles = []
    for b in bs:
        x, st = s.solve(b)
        res = float(np.linalg.norm(b - op.A(x)) / np.linalg.norm(b))
        say(f"      iters {st.outer_iters} lib {st.true_rel_resid:.2e} oracle {res:.2e}")
        assert st.status == 0 and res < 2e-10
        singles.append((x, st))
    import torch
    bt = dev(bs)
    xt = torch.empty_like(bt)
    say("[gpu] MSPCG, reduced-Ls preconditioner, batched")
    stat, stats = s.solve_batch_device(3, bt.data_ptr(), xt.data_ptr())
    assert stat == 0
    xs = xt.cpu().numpy().view(np.complex128).reshape((3,) + bs[0].shape)
    for i in range(3):
        assert stats[i].outer_iters == singles[i][1].outer_iters
        assert np.array_equal(xs[i], singles[i][0])
