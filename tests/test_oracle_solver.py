"""Pins for the oracle's local operator A_s, the inner CG and the outer solvers.

* A_s = R_s A R_s^T agrees with the paper's padded-field construction (a zero
  pad of two sites around the subdomain, Sec. 3.1.2), built here as a
  separate small lattice whose links across the outer pad boundary are zero;
* per-hop Dirichlet truncation differs from A_s (Sec. 2.3, eq. diri);
* the k-step inner CG equals the Galerkin projection onto the Krylov space;
* the preconditioner is local: r outside subdomain s does not change z_s;
* CG and MSPCG reach the dense solution; PCG with the exact inverse as its
  preconditioner converges in one step; residual histories are gauge
  invariant.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.fields import gauge_transform_field, parity_coords

RNG = np.random.default_rng(17)


def rand_field(shape):
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


def make(dims, Ls, mf=0.1, eps=0.5, seed=5):
    return oracle.MobiusDWF(W.gauge_field(dims, eps, seed), Ls, 1.5, 0.5, 1.8, mf)


def dense_A(op):
    n = op.Ls * op.vh * 12
    cols = []
    eye = np.eye(n, dtype=np.complex128)
    for j0 in range(0, n, 256):
        e = eye[j0:j0 + 256].reshape(-1, op.Ls, op.vh, 4, 3)
        cols.append(op.A(e).reshape(-1, n))
    return np.concatenate(cols).T


# ---------------------------------------------------------------- tiling / A_s

def test_tiling_validation():
    assert oracle.tiling_ok((8, 8, 8, 8), (4, 4, 4, 4))
    assert oracle.tiling_ok((16, 16, 16, 32), (4, 4, 4, 8))
    assert oracle.tiling_ok((8, 4, 4, 4), (4, 4, 4, 4))
    assert not oracle.tiling_ok((6, 4, 4, 4), (4, 4, 4, 4))    # does not divide
    assert oracle.tiling_ok((12, 4, 4, 4), (6, 4, 4, 4))
    assert oracle.tiling_ok((8, 4, 4, 4), (2, 4, 4, 4))
    assert oracle.tiling_ok((6, 4, 4, 4), (2, 4, 4, 4))
    assert not oracle.tiling_ok((4, 4, 4, 4), (2, 4, 4, 4))    # 4 - 2 < 4
    assert not oracle.tiling_ok((12, 4, 4, 4), (3, 4, 4, 4))   # odd extent


def padded_local_operator(op, tiling, k, v):
    """A_s v through the padded-field construction of Sec. 3.1.2."""
    dims, sub = tiling.dims, tiling.sub
    part = [s < d for d, s in zip(dims, sub)]
    nb = [d // s for d, s in zip(dims, sub)]
    bx = [k % nb[0], (k // nb[0]) % nb[1], (k // (nb[0] * nb[1])) % nb[2], k // (nb[0] * nb[1] * nb[2])]
    origin = [bx[m] * sub[m] for m in range(4)]
    L = [sub[m] + 4 if part[m] else dims[m] for m in range(4)]
    X, Y, Z, T = L
    Upad = np.empty((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    for t in range(T):
        for z in range(Z):
            for y in range(Y):
                for x in range(X):
                    loc = (x, y, z, t)
                    g = [(origin[m] - 2 + loc[m]) % dims[m] if part[m] else loc[m] for m in range(4)]
                    Upad[t, z, y, x] = op.U[g[3], g[2], g[1], g[0]]
                    for m in range(4):
                        if part[m] and loc[m] == L[m] - 1:
                            Upad[t, z, y, x, m] = 0.0
    pop = oracle.MobiusDWF(Upad, op.Ls, op.b, op.c, op.M5, op.mf)
    # global even sites of the subdomain -> padded single-parity index
    cg = parity_coords(dims, 0)[tiling.index[k]]
    loc = np.stack([(cg[:, m] - origin[m] + 2) if part[m] else cg[:, m] for m in range(4)], axis=1)
    lex = loc[:, 0] + X * (loc[:, 1] + Y * (loc[:, 2] + Z * loc[:, 3]))
    assert np.all((loc.sum(axis=1) % 2) == 0)
    idx = lex // 2
    full = np.zeros((op.Ls, pop.vh, 4, 3), dtype=np.complex128)
    full[:, idx] = v
    return pop.A(full)[:, idx]


@pytest.mark.parametrize("dims,sub", [((8, 4, 4, 4), (4, 4, 4, 4)),
                                      ((12, 4, 2, 2), (4, 4, 2, 2)),
                                      ((8, 8, 4, 2), (4, 4, 4, 2)),
                                      ((8, 8, 8, 8), (4, 4, 4, 4))])
def test_local_operator_equals_padded_field(dims, sub):
    """Three constructions of A_s agree: R_s A R_s^T by embedding, the
    oracle's padded-field operator, and the padded field built here site by
    site (an independent copy of the Sec. 3.1.2 construction)."""
    op = make(dims, 3, eps=0.7, seed=3)
    til = oracle.Tiling(dims, sub)
    ks = [0, til.nsub - 1]
    vs = rand_field((len(ks), op.Ls, len(til.index[0]), 4, 3))
    As = oracle.local_operator(op, til, vs, subset=ks)
    Ap = oracle.local_operator(op, til, vs, subset=ks, padded=True)
    for j, k in enumerate(ks):
        ref = padded_local_operator(op, til, k, vs[j])
        assert np.max(np.abs(As[j] - ref)) < 1e-12 * np.max(np.abs(ref))
        assert np.max(np.abs(Ap[j] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_padded_inner_cg_equals_embedded_inner_cg():
    dims, sub = (12, 4, 4, 4), (4, 4, 4, 4)
    op = make(dims, 4, mf=0.05, seed=4)
    til = oracle.Tiling(dims, sub)
    r = rand_field((op.Ls, op.vh, 4, 3))
    z1 = oracle.inner_cg(op, til, r, 3, subset=[1, 2])
    z2 = oracle.inner_cg(op, til, r, 3, subset=[1, 2], padded=True)
    assert np.max(np.abs(z1 - z2)) < 1e-12 * np.max(np.abs(z1))


def test_snake_terms_matter():
    """Per-hop Dirichlet truncation (each hop confined to the subdomain)
    is not the local part of the four-hop operator."""
    dims, sub = (8, 8, 4, 4), (4, 4, 4, 4)
    op = make(dims, 4, eps=0.5, seed=9)
    til = oracle.Tiling(dims, sub)
    k = 0
    inside = {p: None for p in (0, 1)}
    for p in (0, 1):
        c = parity_coords(dims, p)
        inside[p] = np.all(c < np.array(sub)[None, :], axis=1)     # subdomain 0 is the origin block
    assert np.array_equal(np.nonzero(inside[0])[0], til.index[k])

    def trunc(f, p):
        g = f.copy()
        g[:, ~inside[p]] = 0
        return g

    def D_tr(psi):
        t = trunc(op.m4(psi, 1), 1)
        t = oracle.apply5(op.M5inv, t)
        t = trunc(op.m4(t, 0), 0)
        return psi - oracle.apply5(op.M5inv, t)

    def Ddag_tr(chi):
        t = oracle.apply5(op.M5inv_dag, chi)
        t = trunc(op.m4_dag(t, 1), 1)
        t = oracle.apply5(op.M5inv_dag, t)
        t = trunc(op.m4_dag(t, 0), 0)
        return chi - t

    v = rand_field((op.Ls, len(til.index[k]), 4, 3))
    full = np.zeros((op.Ls, op.vh, 4, 3), dtype=np.complex128)
    full[:, til.index[k]] = v
    a_trunc = Ddag_tr(D_tr(full))[:, til.index[k]]
    a_s = oracle.local_operator(op, til, v[None], subset=[k])[0]
    rel = np.linalg.norm(a_s - a_trunc) / np.linalg.norm(a_s)
    assert rel > 1e-3
    # the oracle's per-hop truncated operator (the comparator of the GPU
    # tests) is this construction
    a_or = oracle.truncated_local_operator(op, til, v[None], subset=[k])[0]
    assert np.max(np.abs(a_or - a_trunc)) < 1e-13 * np.max(np.abs(a_trunc))
    # and reduces to A when the subdomain is the whole lattice
    til1 = oracle.Tiling(dims, dims)
    w = rand_field((op.Ls, op.vh, 4, 3))
    a1 = oracle.truncated_local_operator(op, til1, w[:, til1.index[0]][None], subset=[0])[0]
    assert np.max(np.abs(a1 - op.A(w)[:, til1.index[0]])) < 1e-12 * np.max(np.abs(a1))


def test_local_operator_hpd():
    dims, sub = (8, 2, 2, 2), (4, 2, 2, 2)
    op = make(dims, 4)
    til = oracle.Tiling(dims, sub)
    n = op.Ls * len(til.index[0]) * 12
    eye = np.eye(n, dtype=np.complex128).reshape(n, op.Ls, -1, 4, 3)
    cols = [oracle.local_operator(op, til, eye[j0:j0 + 64], subset=[0] * len(eye[j0:j0 + 64]))
            for j0 in range(0, n, 64)]
    As = np.concatenate(cols).reshape(n, n).T
    assert np.max(np.abs(As - As.conj().T)) < 1e-13 * np.max(np.abs(As))
    assert np.min(np.linalg.eigvalsh(As)) > 0
    # principal submatrix of the dense A
    Afull = dense_A(op)
    sel = (np.arange(op.Ls)[:, None, None, None] * op.vh * 12
           + til.index[0][None, :, None, None] * 12
           + np.arange(4)[None, None, :, None] * 3 + np.arange(3)[None, None, None, :]).reshape(-1)
    assert np.max(np.abs(Afull[np.ix_(sel, sel)] - As)) < 1e-13 * np.max(np.abs(As))


# ---------------------------------------------------------------- inner CG

@pytest.mark.parametrize("k", [1, 3, 6])
def test_inner_cg_is_galerkin_projection(k):
    dims, sub = (8, 2, 2, 2), (4, 2, 2, 2)
    op = make(dims, 4, mf=0.05)
    til = oracle.Tiling(dims, sub)
    r = rand_field((op.Ls, op.vh, 4, 3))
    z = oracle.inner_cg(op, til, r, k)
    for s in range(til.nsub):
        rs = r[:, til.index[s]]
        K = [rs]
        for _ in range(k - 1):
            K.append(oracle.local_operator(op, til, K[-1][None], subset=[s])[0])
        V, _ = np.linalg.qr(np.stack([v.reshape(-1) for v in K], axis=1))
        AV = np.stack([oracle.local_operator(op, til, V[:, j].reshape(rs.shape)[None], subset=[s])[0].reshape(-1)
                       for j in range(V.shape[1])], axis=1)
        zg = V @ np.linalg.solve(V.conj().T @ AV, V.conj().T @ rs.reshape(-1))
        assert np.linalg.norm(z[s].reshape(-1) - zg) < 1e-9 * np.linalg.norm(zg)


def test_preconditioner_is_local():
    dims, sub = (8, 4, 4, 4), (4, 4, 4, 4)
    op = make(dims, 4)
    til = oracle.Tiling(dims, sub)
    r = rand_field((op.Ls, op.vh, 4, 3))
    r2 = r.copy()
    r2[:, til.index[1]] = rand_field((op.Ls, len(til.index[1]), 4, 3))
    z1 = oracle.inner_cg(op, til, r, 4)
    z2 = oracle.inner_cg(op, til, r2, 4)
    assert np.array_equal(z1[0], z2[0])
    assert not np.array_equal(z1[1], z2[1])


def test_inner_cg_zero_rhs_subdomain():
    dims, sub = (8, 4, 4, 4), (4, 4, 4, 4)
    op = make(dims, 4)
    til = oracle.Tiling(dims, sub)
    r = rand_field((op.Ls, op.vh, 4, 3))
    r[:, til.index[1]] = 0
    z = oracle.inner_cg(op, til, r, 3)
    assert np.all(z[1] == 0) and np.linalg.norm(z[0]) > 0


# ---------------------------------------------------------------- outer solvers

def test_cg_and_mspcg_reach_dense_solution():
    dims, sub = (8, 2, 2, 2), (4, 2, 2, 2)
    op = make(dims, 4, mf=0.05, eps=0.4)
    til = oracle.Tiling(dims, sub)
    b = W.gaussian_source(dims, op.Ls, 77)
    Ad = dense_A(op)
    xs = np.linalg.solve(Ad, b.reshape(-1)).reshape(b.shape)
    ev = np.linalg.eigvalsh(Ad)
    kappa = ev[-1] / ev[0]
    tol = 1e-10
    for x, info in (oracle.cg(op, b, tol, 2000), oracle.mspcg(op, til, b, 4, tol, 500)):
        assert info.converged and info.true_rel_resid < 2 * tol
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < kappa * tol


def test_pcg_exact_preconditioner_one_step():
    dims = (4, 2, 2, 2)
    op = make(dims, 4, mf=0.05)
    Ad = dense_A(op)
    Ainv = np.linalg.inv(Ad)
    b = W.gaussian_source(dims, op.Ls, 78)
    x, info = oracle.pcg(op, b, 1e-12, 10,
                         precond=lambda r: (Ainv @ r.reshape(-1)).reshape(r.shape), beta_rule="PR")
    assert info.iters == 1 and info.converged


def test_mspcg_fewer_outer_iterations_and_gauge_invariant_history():
    dims, sub = (8, 4, 4, 4), (4, 4, 4, 4)
    U = W.gauge_field(dims, 0.5, 55)
    op = oracle.MobiusDWF(U, 4, 1.5, 0.5, 1.8, 0.05)
    til = oracle.Tiling(dims, sub)
    b = W.gaussian_source(dims, 4, 56)
    _, i_cg = oracle.cg(op, b, 1e-7, 3000)
    _, i_ms = oracle.mspcg(op, til, b, 4, 1e-7, 500)
    print('outer iterations: cg', i_cg.iters, 'mspcg', i_ms.iters)
    assert i_cg.converged and i_ms.converged
    assert i_ms.iters < i_cg.iters
    # gauge-rotated problem: identical residual history up to rounding
    Om = W.random_gauge_transform(dims, 57)
    opg = oracle.MobiusDWF(W.gauge_transform_links(U, Om), 4, 1.5, 0.5, 1.8, 0.05)
    _, i_g = oracle.mspcg(opg, til, gauge_transform_field(b, Om, 0), 4, 1e-7, 30)
    n = min(len(i_ms.history), len(i_g.history), 15)
    h1, h2 = np.array(i_ms.history[:n]), np.array(i_g.history[:n])
    assert np.max(np.abs(h1 - h2) / h1) < 1e-9


def _successive_conjugacy(op, til, b, k, beta_rule, iters=8):
    """max over outer iterations of |Re<p_{j+1}, A p_j>| / (|p_{j+1}|_A |p_j|_A)
    for Alg. 1 with the k-step inner-CG preconditioner.  The search
    directions are read off the iterates: x_j - x_{j-1} = alpha_j p_j, and the
    ratio is invariant under the scale alpha_j."""
    xs = [np.zeros_like(b)]
    oracle.pcg(op, b, 1e-30, iters, precond=lambda r: oracle.precondition(op, til, r, k),
               beta_rule=beta_rule, callback=lambda it, x, r: xs.append(x.copy()))
    dx = [xs[j + 1] - xs[j] for j in range(len(xs) - 1)]
    Adx = [op.A(d) for d in dx]
    worst = 0.0
    for j in range(len(dx) - 1):
        num = abs(np.vdot(dx[j + 1], Adx[j]).real)
        den = np.sqrt(np.vdot(dx[j + 1], Adx[j + 1]).real * np.vdot(dx[j], Adx[j]).real)
        worst = max(worst, num / den)
    return worst


def test_polak_ribiere_beta_keeps_successive_directions_conjugate():
    """Pin of the Polak-Ribiere beta (Sec. 3.2).  With r_{j+1} - r_j =
    -alpha_j A p_j and alpha_j = <r_j, z_j>/<p_j, A p_j>, the PR choice
    beta = <z_{j+1}, r_{j+1} - r_j>/<z_j, r_j> makes <p_{j+1}, A p_j> vanish
    exactly for any preconditioner, also an inexact, nonlinear one such as
    the fixed-k inner CG.  The Fletcher-Reeves beta of Alg. 1 (planted here
    as the mistake) does not: the k-step preconditioner is not a fixed
    linear map, so its directions lose conjugacy by O(1e-2)."""
    dims, sub = (8, 4, 4, 4), (4, 4, 4, 4)
    op = make(dims, 4, mf=0.05, eps=0.5, seed=21)
    til = oracle.Tiling(dims, sub)
    b = W.gaussian_source(dims, op.Ls, 22)
    pr = _successive_conjugacy(op, til, b, 3, "PR")
    fr = _successive_conjugacy(op, til, b, 3, "FR")
    print("successive A-conjugacy: PR", pr, "FR", fr)
    assert pr < 1e-12
    assert fr > 1e-5
