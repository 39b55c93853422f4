"""Pins for the oracle's reduced-Ls preconditioner (Sec. 3.3): the transform
T, the preconditioner (T^dag Mhat^-1 T + mu) r, the training loss chi^2, its
gradient, the quartic line search and the training loop.

* T^dag is the adjoint of T (fails a missing conjugate or swapped indices);
* T acts as the identity in colour and on the sites (fails a colour mix);
* with Lhat = Ls, T = 1 and mu = 0 the reduced preconditioner is the full
  one, and with an exact Mhat^-1 the loss is zero at T = 1 -- the paper's
  own statement of the Lhat = Ls case;
* the gradient matches central finite differences of chi^2 for a linear
  Hermitian Mhat^-1, in every real and imaginary direction sampled (fails a
  dropped term, a missing factor 2 or conjugate);
* the line quartic equals chi^2 along the line for a linear Mhat^-1, and its
  minimiser is exact;
* training with a linear Mhat^-1 never increases chi^2 and lowers it.
"""
import numpy as np
import pytest

import oracle
import workloads as W

RNG = np.random.default_rng(2105)
DIMS, SUB = (8, 2, 2, 2), (4, 2, 2, 2)


def rand(shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def ops(Ls, Lh, mf=0.1):
    U = W.gauge_field(DIMS, 0.4, 7)
    return (oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, mf), oracle.MobiusDWF(U, Lh, 1.5, 0.5, 1.8, mf),
            oracle.Tiling(DIMS, SUB))


def identity_T(Ls):
    T = np.zeros((Ls, 4, Ls, 4), dtype=np.complex128)
    for s in range(Ls):
        T[s, :, s, :] = np.eye(4)
    return T


def dense_local_inverse(op, til):
    """Exact ((+)_s A_s)^-1 on the tiny lattice, from the dense local operator."""
    n = op.Ls * op.vh * 12
    cols = np.stack([oracle.local_op_full(op, til, e.reshape(op.Ls, op.vh, 4, 3)).ravel()
                     for e in np.eye(n, dtype=np.complex128)], axis=1)
    inv = np.linalg.inv(cols)
    return lambda x: (inv @ x.ravel()).reshape(x.shape)


def test_transform_adjoint_and_colour_trivial():
    op, oph, til = ops(6, 3)
    T = rand((3, 4, 6, 4))
    v = rand((6, op.vh, 4, 3))
    w = rand((3, op.vh, 4, 3))
    lhs = np.vdot(w, oracle.transform(T, v))
    rhs = np.vdot(oracle.transform_dag(T, w), v)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # a colour rotation per site commutes with T
    Q, _ = np.linalg.qr(rand((op.vh, 3, 3)))
    rot = lambda f: np.einsum("xab,...xmb->...xma", Q, f)
    assert np.allclose(oracle.transform(T, rot(v)), rot(oracle.transform(T, v)), atol=1e-12)
    # the identity transform
    assert np.array_equal(oracle.transform(identity_T(6), v), v)


def test_full_ls_identity_reduces_to_the_original_preconditioner():
    op, _, til = ops(4, 4)
    r = rand((4, op.vh, 4, 3))
    z1 = oracle.reduced_precondition(op, til, identity_T(4), 0.0, r, 3)
    z0 = oracle.precondition(op, til, r, 3)
    assert np.allclose(z1, z0, rtol=0, atol=1e-13 * np.abs(z0).max())
    # the mu shift adds mu r
    z2 = oracle.reduced_precondition(op, til, identity_T(4), 0.25, r, 3)
    assert np.allclose(z2 - z1, 0.25 * r, atol=1e-13 * np.abs(r).max())


def test_loss_vanishes_at_identity_with_exact_inverse():
    op, _, til = ops(2, 2)
    H = dense_local_inverse(op, til)
    vs = [rand((2, op.vh, 4, 3)) for _ in range(2)]
    c, g = oracle.chi2(op, op, til, identity_T(2), 0.0, vs, 0, inverse=H, gradient=True)
    scale = sum(oracle.norm2(v) for v in vs)
    assert c < 1e-20 * scale
    assert np.abs(g).max() < 1e-9 * np.sqrt(scale)


def test_gradient_matches_finite_differences():
    op, oph, til = ops(4, 2)
    Hmat = rand((2 * oph.vh * 12, 2 * oph.vh * 12))
    Hmat = Hmat @ Hmat.conj().T / Hmat.shape[0] + np.eye(Hmat.shape[0])      # Hermitian positive
    H = lambda x: (Hmat @ x.ravel()).reshape(x.shape)
    T = 0.3 * rand((2, 4, 4, 4))
    vs = [rand((4, op.vh, 4, 3)) for _ in range(2)]
    mu = 0.1
    _, g = oracle.chi2(op, oph, til, T, mu, vs, 0, inverse=H, gradient=True)
    eps = 1e-6
    for _ in range(6):
        idx = tuple(RNG.integers(0, n) for n in T.shape)
        for unit in (1.0, 1j):
            E = np.zeros_like(T)
            E[idx] = unit
            fp = oracle.chi2(op, oph, til, T + eps * E, mu, vs, 0, inverse=H)
            fm = oracle.chi2(op, oph, til, T - eps * E, mu, vs, 0, inverse=H)
            fd = (fp - fm) / (2 * eps)
            an = float(np.real(np.conj(g[idx]) * unit))
            assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (idx, unit, fd, an)


def test_line_quartic_is_chi2_along_the_line_for_a_linear_inverse():
    op, oph, til = ops(4, 2)
    H = dense_local_inverse(oph, til)
    T = 0.3 * rand((2, 4, 4, 4))
    d = rand((2, 4, 4, 4))
    vs = [rand((4, op.vh, 4, 3)) for _ in range(2)]
    c = oracle.line_quartic(op, oph, til, T, d, 0.1, vs, 0, inverse=H)
    for eta in (0.0, 0.37, -1.3, 2.0):
        direct = oracle.chi2(op, oph, til, T + eta * d, 0.1, vs, 0, inverse=H)
        assert abs(np.polyval(c[::-1], eta) - direct) < 1e-10 * direct


def test_quartic_min_is_exact():
    # 3 (e - 1.7)^2 ((e - 1.7)^2 + 0.5) + 2, expanded
    p = np.polynomial.polynomial.Polynomial([-1.7, 1.0])
    q = 3 * p ** 2 * (p ** 2 + 0.5) + 2
    assert abs(oracle.quartic_min(q.coef) - 1.7) < 1e-9
    # the minimum over eta >= 0 of an increasing quartic is at 0
    assert oracle.quartic_min([1.0, 2.0, 1.0, 0.0, 1.0]) == 0.0


def test_training_lowers_the_loss():
    op, oph, til = ops(4, 2)
    H = dense_local_inverse(oph, til)
    vs = [rand((4, op.vh, 4, 3)) for _ in range(2)]
    T0 = np.zeros((2, 4, 4, 4), dtype=np.complex128)
    for s in range(2):
        T0[s, :, 2 * s, :] = np.eye(4)
    T, hist = oracle.train_transform(op, oph, til, T0, 0.1, vs, 0, iters=4, inverse=H)
    assert hist[-1] < 0.5 * hist[0]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    assert hist[-1] < 0.9 * hist[0]
