"""Pins for the FP64 oracle's operators (CPU only).

Each check ties the oracle to something other than itself: an algebraic
identity of the gamma matrices, the momentum-space closed form of the free
Wilson hopping term, adjointness, gauge covariance, the closed form of the
inverse of the fifth-dimension matrix, the Pauli-Villars ratio of the free
domain-wall operator against the Mobius overlap formula, and the even-odd
block decomposition of Sec. 2.2.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from workloads.fields import gauge_transform_field, parity_coords

RNG = np.random.default_rng(7)


def rand_field(Ls, vh, nrhs=None):
    shape = (Ls, vh, 4, 3) if nrhs is None else (nrhs, Ls, vh, 4, 3)
    return RNG.standard_normal(shape) + 1j * RNG.standard_normal(shape)


# ---------------------------------------------------------------- gamma basis

def test_gamma_clifford_algebra():
    G = oracle.GAMMA
    for mu in range(4):
        assert np.allclose(G[mu], G[mu].conj().T, atol=0)
        for nu in range(4):
            anti = G[mu] @ G[nu] + G[nu] @ G[mu]
            assert np.allclose(anti, 2.0 * (mu == nu) * np.eye(4), atol=1e-15)
    g5 = oracle.GAMMA5
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)
    for mu in range(4):
        assert np.allclose(g5 @ G[mu] + G[mu] @ g5, 0, atol=1e-15)
    assert np.allclose(oracle.P_PLUS + oracle.P_MINUS, np.eye(4))
    assert np.allclose(oracle.P_PLUS @ oracle.P_MINUS, 0)


# ---------------------------------------------------------------- hopping term

@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0),
                               (0, 0, 0, 1), (1, 2, 3, 4), (3, 5, 7, 9)])
@pytest.mark.parametrize("out_parity", [0, 1])
def test_hop_free_field_plane_wave(n, out_parity):
    """U = 1, psi(x) = e^{i p.x} u: D^w psi = e^{i p.x} [2 sum cos p_mu - 2i sum gamma_mu sin p_mu] u.
    Unequal extents catch a mix-up of directions."""
    dims = (4, 6, 8, 10)
    Ls = 2
    U = W.unit_gauge_field(dims)
    p = np.array([2 * np.pi * n[m] / dims[m] for m in range(4)])
    u = RNG.standard_normal((Ls, 4, 3)) + 1j * RNG.standard_normal((Ls, 4, 3))
    cin = parity_coords(dims, 1 - out_parity)
    cout = parity_coords(dims, out_parity)
    psi = np.exp(1j * cin @ p)[None, :, None, None] * u[:, None]
    out = oracle.wilson_hop(U, psi, out_parity)
    Dp = 2 * np.sum(np.cos(p)) * np.eye(4) - 2j * sum(oracle.GAMMA[m] * np.sin(p[m]) for m in range(4))
    expect = np.exp(1j * cout @ p)[None, :, None, None] * np.einsum("ab,sbc->sac", Dp, u)[:, None]
    assert np.max(np.abs(out - expect)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 2, 2), (6, 4, 2, 8)])
def test_hop_adjoint_and_gamma5_hermiticity(dims):
    Ls = 3
    U = W.gauge_field(dims, 0.7, 11)
    vh = np.prod(dims) // 2
    x_e, y_o = rand_field(Ls, vh), rand_field(Ls, vh)
    lhs = np.vdot(x_e, oracle.wilson_hop(U, y_o, 0))
    rhs = np.vdot(oracle.wilson_hop(U, x_e, 1, dagger=True), y_o)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # D^w^dag = gamma5 D^w gamma5
    g5 = oracle.GAMMA5
    a = oracle.wilson_hop(U, y_o, 0, dagger=True)
    b = np.einsum("ab,sibc->siac", g5, oracle.wilson_hop(U, np.einsum("ab,sibc->siac", g5, y_o), 0))
    assert np.max(np.abs(a - b)) < 1e-13


def test_hop_gauge_covariance():
    dims = (4, 4, 6, 4)
    Ls = 2
    U = W.gauge_field(dims, 0.9, 12)
    Om = W.random_gauge_transform(dims, 13)
    Ug = W.gauge_transform_links(U, Om)
    vh = np.prod(dims) // 2
    psi_o = rand_field(Ls, vh)
    for dag in (False, True):
        lhs = oracle.wilson_hop(Ug, gauge_transform_field(psi_o, Om, 1), 0, dagger=dag)
        rhs = gauge_transform_field(oracle.wilson_hop(U, psi_o, 0, dagger=dag), Om, 0)
        assert np.max(np.abs(lhs - rhs)) < 1e-12


def test_generated_links_are_su3():
    U = W.gauge_field((4, 4, 4, 4), 0.6, 104).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(U @ np.conj(np.swapaxes(U, 1, 2)) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(U) - 1)) < 1e-14


# ---------------------------------------------------------------- fifth dimension

@pytest.mark.parametrize("Ls,b,c,M5,mf", [(8, 1.5, 0.5, 1.8, 0.1), (12, 1.5, 0.5, 1.8, 0.01),
                                           (5, 1.0, 0.0, 1.6, 0.3), (16, 2.0, 1.0, 1.4, 0.005)])
def test_m5_inverse_closed_form(Ls, b, c, M5, mf):
    """(a0 + a1 S)^-1 with S^Ls = -mf: entry kappa^{s-t}/(a0(1 + mf kappa^Ls)) for s >= t and
    -mf kappa^{s-t+Ls}/(a0(1 + mf kappa^Ls)) for s < t, kappa = -a1/a0 (geometric series)."""
    a0 = b * (4 - M5) + 1
    a1 = c * (4 - M5) - 1
    kap = -a1 / a0
    den = a0 * (1 + mf * kap ** Ls)
    s = np.arange(Ls)[:, None]
    t = np.arange(Ls)[None, :]
    closed = np.where(s >= t, kap ** (s - t), -mf * kap ** (s - t + Ls)) / den
    Minv = oracle.inverse5(oracle.m5_matrix(Ls, b, c, M5, mf))
    assert np.max(np.abs(Minv[:, 0, :, 0] - closed)) < 1e-13 * np.max(np.abs(closed))
    assert np.max(np.abs(Minv[:, 1, :, 1] - closed)) < 1e-13 * np.max(np.abs(closed))
    assert np.max(np.abs(Minv[:, 2, :, 2] - closed.T)) < 1e-13 * np.max(np.abs(closed))
    # no chirality or spin mixing
    for al in range(4):
        for be in range(4):
            if al != be:
                assert np.max(np.abs(Minv[:, al, :, be])) == 0.0
    M = oracle.m5_matrix(Ls, b, c, M5, mf).reshape(4 * Ls, 4 * Ls)
    assert np.max(np.abs(Minv.reshape(4 * Ls, 4 * Ls) @ M - np.eye(4 * Ls))) < 1e-13


def test_m5_mphi_commute():
    for Ls, mf in ((8, 0.1), (12, 0.00078)):
        A = oracle.m5_matrix(Ls, 1.5, 0.5, 1.8, mf).reshape(4 * Ls, -1)
        B = oracle.mphi_matrix(Ls, 1.5, 0.5, mf).reshape(4 * Ls, -1)
        assert np.max(np.abs(A @ B - B @ A)) < 1e-15


@pytest.mark.parametrize("Ls,b,c,M5", [(8, 1.5, 0.5, 1.8), (12, 1.5, 0.5, 1.8), (7, 1.0, 0.0, 1.2),
                                       (10, 2.0, 1.0, 1.6)])
@pytest.mark.parametrize("mf", [0.1, 0.01, 0.3])
def test_free_domain_wall_pauli_villars_ratio(Ls, b, c, M5, mf):
    """Free field at p = 0: per chirality, det D5(mf) / det D5(mf=1) equals the Mobius
    overlap operator at finite Ls, (1+mf)/2 + (1-mf)/2 eps, with
    eps = ((1+h)^Ls - (1-h)^Ls)/((1+h)^Ls + (1-h)^Ls) and kernel
    h = (b+c) D_W / (2 + (b-c) D_W), D_W(p=0) = -M5 (Wilson kernel of mass -M5).
    The 5D matrix D5(0) is read off the oracle's full operator on constant fields."""
    dims = (2, 2, 2, 2)
    U = W.unit_gauge_field(dims)
    vh = 8

    def d5_at_p0(mf_):
        op = oracle.MobiusDWF(U, Ls, b, c, M5, mf_)
        D = np.zeros((Ls * 4, Ls * 4), dtype=complex)
        for t in range(Ls):
            for be in range(4):
                u = np.zeros((Ls, vh, 4, 3), dtype=complex)
                u[t, :, be, 0] = 1.0
                pe, _ = op.full(u, u)
                D[:, t * 4 + be] = pe[:, 0, :, 0].reshape(-1)
        return D.reshape(Ls, 4, Ls, 4)

    def det_chiral(D, spins):
        blk = D[:, spins][:, :, :, spins].reshape(Ls * len(spins), Ls * len(spins))
        return np.linalg.det(blk)

    DW = -M5
    h = (b + c) * DW / (2 + (b - c) * DW)
    eps = ((1 + h) ** Ls - (1 - h) ** Ls) / ((1 + h) ** Ls + (1 - h) ** Ls)
    dov = (1 + mf) / 2 + (1 - mf) / 2 * eps
    Dm, D1 = d5_at_p0(mf), d5_at_p0(1.0)
    for spins in ([0], [1], [2], [3]):
        ratio = det_chiral(Dm, spins) / det_chiral(D1, spins)
        assert abs(ratio - dov) < 1e-12 * max(1.0, abs(dov))


def test_even_odd_block_decomposition():
    """Sec. 2.2: with phi = [[M5, M4_eo], [M4_oe, M5]] psi, D psi_e = phi^_e and
    psi_o = M5^-1 (phi_o - M4_oe psi_e)."""
    dims = (4, 4, 2, 6)
    Ls = 6
    U = W.gauge_field(dims, 0.5, 21)
    op = oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, 0.05)
    vh = op.vh
    pe, po = rand_field(Ls, vh), rand_field(Ls, vh)
    fe, fo = op.full(pe, po)
    assert np.max(np.abs(op.D(pe) - op.phi_hat(fe, fo))) < 1e-12 * np.max(np.abs(pe))
    assert np.max(np.abs(op.reconstruct_odd(pe, fo) - po)) < 1e-12 * np.max(np.abs(po))


# ---------------------------------------------------------------- D, D^dag, A

def _op(dims=(4, 4, 4, 4), Ls=4, mf=0.1, eps=0.5, seed=31):
    return oracle.MobiusDWF(W.gauge_field(dims, eps, seed), Ls, 1.5, 0.5, 1.8, mf)


def test_ddag_is_adjoint_and_A_hermitian_positive():
    op = _op()
    x, y = rand_field(op.Ls, op.vh), rand_field(op.Ls, op.vh)
    lhs = np.vdot(x, op.D(y))
    rhs = np.vdot(op.Ddag(x), y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    xa, ya = np.vdot(x, op.A(y)), np.vdot(op.A(x), y)
    assert abs(xa - ya) < 1e-13 * abs(xa)
    q = np.vdot(x, op.A(x))
    assert q.real > 0 and abs(q.imag) < 1e-12 * q.real


def test_A_gauge_covariance():
    dims = (4, 4, 4, 2)
    U = W.gauge_field(dims, 0.8, 41)
    Om = W.random_gauge_transform(dims, 42)
    a = oracle.MobiusDWF(U, 4, 1.5, 0.5, 1.8, 0.1)
    g = oracle.MobiusDWF(W.gauge_transform_links(U, Om), 4, 1.5, 0.5, 1.8, 0.1)
    psi = rand_field(4, a.vh)
    lhs = g.A(gauge_transform_field(psi, Om, 0))
    rhs = gauge_transform_field(a.A(psi), Om, 0)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 0, 2, 1), (2, 3, 1, 5)])
def test_schur_operator_free_field_momentum_space(n):
    """U = 1, psi_e = e^{ip.x} u on even sites: D psi_e = e^{ip.x} D(p) u with the
    (4Ls)x(4Ls) matrix D(p) = 1 - M5^-1 H(p) M_phi M5^-1 H(p) M_phi, H(p) = D^w(p) x 1_s."""
    dims = (4, 6, 4, 8)
    Ls = 5
    op = oracle.MobiusDWF(W.unit_gauge_field(dims), Ls, 1.5, 0.5, 1.8, 0.05)
    p = np.array([2 * np.pi * n[m] / dims[m] for m in range(4)])
    Dw = 2 * np.sum(np.cos(p)) * np.eye(4) - 2j * sum(oracle.GAMMA[m] * np.sin(p[m]) for m in range(4))
    H = np.kron(np.eye(Ls), Dw)
    M5i = op.M5inv.reshape(4 * Ls, -1)
    Mp = op.Mphi.reshape(4 * Ls, -1)
    Dp = np.eye(4 * Ls) - M5i @ H @ Mp @ M5i @ H @ Mp
    u = RNG.standard_normal((Ls, 4, 3)) + 1j * RNG.standard_normal((Ls, 4, 3))
    ce = parity_coords(dims, 0)
    psi = np.exp(1j * ce @ p)[None, :, None, None] * u[:, None]
    got = op.D(psi)
    Du = (Dp @ u.reshape(4 * Ls, 3)).reshape(Ls, 4, 3)
    expect = np.exp(1j * ce @ p)[None, :, None, None] * Du[:, None]
    assert np.max(np.abs(got - expect)) < 1e-12 * np.max(np.abs(expect))


def test_degrees_of_freedom_table():
    """Table 1 and Table 2 quote the number of real degrees of freedom V4 * Ls * 24."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "dof_table.json")))
    for row in g["rows"]:
        X, Y, Z, T = row["dims"]
        dof = X * Y * Z * T * row["Ls"] * 24
        if row.get("consistent", True):
            assert abs(dof / row["dof"] - 1) < 0.05, row
