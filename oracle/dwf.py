"""FP64 CPU oracle for the even-odd preconditioned Mobius domain-wall
operator and the multi-splitting preconditioned CG (MSPCG) built on it.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP library (``paper_2104_05615_amd``) and never imports it.

Every function writes out the plain definition it follows (cited by section
and equation of arxiv 2104.05615) in FP64, without blocking, fusion or
reordering beyond what the definition states.  The Wilson hopping term is a C
loop (``hop.c``); all fifth-dimension operators are dense
``(4 Ls) x (4 Ls)`` complex matrices in spin x s space built from their
definitions, applied with a matrix product.

Readings taken where the paper is silent:

* gamma matrices: chiral basis, gamma_5 = diag(1, 1, -1, -1);
* periodic boundaries in all four directions;
* the fifth-dimension operators follow the Mobius construction the paper
  cites for details: with the chirality-twisted shift
  ``(P~ psi)(s) = P_- psi(s+1) + P_+ psi(s-1)``,
  ``psi(Ls) = -mf psi(0)``, ``psi(-1) = -mf psi(Ls-1)``,
  ``M_5 = (b(4 - M5) + 1) + (c(4 - M5) - 1) P~`` and
  ``M_phi = -(b + c P~)/2``, so that ``M^4 = D^w M_phi`` as written in the paper;
* inner CG: per-subdomain scalars, fixed k iterations, no early exit;
* outer MSPCG: Polak-Ribiere beta, plain CG: Fletcher-Reeves beta, stop on
  the L2 residual relative to ||b||.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_hop.so")

# --------------------------------------------------------------------------
# C hopping term
# --------------------------------------------------------------------------


def build_hop_library(force: bool = False) -> str:
    """Compile ``hop.c`` with gcc (OpenMP) into ``oracle/_hop.so``."""
    src = os.path.join(_HERE, "hop.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fcx-limited-range", "-fopenmp", "-fPIC", "-shared",
                               src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _hop_lib():
    global _lib
    if _lib is None:
        build_hop_library()
        # idle OpenMP workers must not spin: they would starve the BLAS
        # threads that apply the fifth-dimension matrices
        os.environ.setdefault("OMP_WAIT_POLICY", "PASSIVE")
        os.environ.setdefault("GOMP_SPINCOUNT", "0")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_wilson_hop.restype = None
        lib.oracle_wilson_hop.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int] * 7
        _lib = lib
    return _lib


# --------------------------------------------------------------------------
# gamma matrices (Sec. 2.2 uses gamma_mu in D^w; basis not given -> chiral)
# --------------------------------------------------------------------------

_S1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
_S2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
_S3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)


def _chiral_gamma(sig):
    return np.block([[_Z2, -1j * sig], [1j * sig, _Z2]])


GAMMA = np.ascontiguousarray(np.stack([
    _chiral_gamma(_S1),                    # x
    _chiral_gamma(_S2),                    # y
    _chiral_gamma(_S3),                    # z
    np.block([[_Z2, _I2], [_I2, _Z2]]),    # t
]))
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
P_PLUS = 0.5 * (np.eye(4) + GAMMA5)
P_MINUS = 0.5 * (np.eye(4) - GAMMA5)


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------


def parity_coords(dims, parity):
    """(x, y, z, t) of the sites of one parity in single-parity order (lex/2)."""
    X, Y, Z, T = dims
    vh = X * Y * Z * T // 2
    lex0 = 2 * np.arange(vh)
    x0 = lex0 % X
    y = (lex0 // X) % Y
    z = (lex0 // (X * Y)) % Z
    t = lex0 // (X * Y * Z)
    x = x0 + ((y + z + t + parity) & 1)
    return np.stack([x, y, z, t], axis=1)


def wilson_hop(U, psi, out_parity, dagger=False):
    """D^w (or its adjoint) from parity ``1 - out_parity`` to ``out_parity``.

    Sec. 2.2, definition of D^w_{x,y}.  ``psi``: ``[..][Ls][V/2][4][3]``; leading
    batch axes are folded into the fifth dimension, on which D^w is diagonal."""
    T, Z, Y, X = U.shape[:4]
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    shape = psi.shape
    vh = shape[-3]
    assert shape[-2:] == (4, 3) and vh == X * Y * Z * T // 2
    ls_tot = int(np.prod(shape[:-3])) if len(shape) > 3 else 1
    out = np.empty_like(psi)
    U = np.ascontiguousarray(U, dtype=np.complex128)
    _hop_lib().oracle_wilson_hop(U.ctypes.data, GAMMA.ctypes.data, psi.ctypes.data,
                                 out.ctypes.data, X, Y, Z, T, ls_tot,
                                 int(out_parity), 1 if dagger else 0)
    return out


# --------------------------------------------------------------------------
# fifth-dimension operators: dense (Ls,4,Ls,4) complex matrices
# --------------------------------------------------------------------------


def ptilde(Ls, mf):
    """Chirality-twisted shift P~ with the -mf wall coupling:
    (P~ psi)(s) = P_- psi(s+1) + P_+ psi(s-1), psi(Ls) = -mf psi(0),
    psi(-1) = -mf psi(Ls-1).  Indexed [s, alpha, t, beta]."""
    P = np.zeros((Ls, 4, Ls, 4), dtype=np.complex128)
    for s in range(Ls):
        if s + 1 < Ls:
            P[s, :, s + 1, :] += P_MINUS
        else:
            P[s, :, 0, :] += -mf * P_MINUS
        if s - 1 >= 0:
            P[s, :, s - 1, :] += P_PLUS
        else:
            P[s, :, Ls - 1, :] += -mf * P_PLUS
    return P


def _eye5(Ls):
    return np.eye(4 * Ls, dtype=np.complex128).reshape(Ls, 4, Ls, 4)


def m5_matrix(Ls, b, c, M5, mf):
    """M_5 = (b(4 - M5) + 1) 1 + (c(4 - M5) - 1) P~ (Mobius, diagonal in 4D)."""
    a0 = b * (4.0 - M5) + 1.0
    a1 = c * (4.0 - M5) - 1.0
    return a0 * _eye5(Ls) + a1 * ptilde(Ls, mf)


def mphi_matrix(Ls, b, c, mf):
    """M_phi = -(b 1 + c P~)/2, so that M^4 = D^w M_phi (Sec. 2.2)."""
    return -0.5 * (b * _eye5(Ls) + c * ptilde(Ls, mf))


def inverse5(M):
    Ls = M.shape[0]
    return np.linalg.inv(M.reshape(4 * Ls, 4 * Ls)).reshape(Ls, 4, Ls, 4)


def adjoint5(M):
    Ls = M.shape[0]
    return np.conj(M.reshape(4 * Ls, 4 * Ls).T).reshape(Ls, 4, Ls, 4)


def apply5(M, psi):
    """(M psi)(s, x, alpha, a) = sum_{t, beta} M[s, alpha, t, beta] psi(t, x, beta, a)."""
    Ls = M.shape[0]
    lead = psi.shape[:-4]
    vh = psi.shape[-3]
    p = np.moveaxis(psi, -2, -3)                       # [..][Ls][4][V/2][3]
    p = p.reshape(lead + (4 * Ls, vh * 3))
    o = M.reshape(4 * Ls, 4 * Ls) @ p
    o = o.reshape(lead + (Ls, 4, vh, 3))
    return np.ascontiguousarray(np.moveaxis(o, -3, -2))


# --------------------------------------------------------------------------
# the Mobius domain-wall operator
# --------------------------------------------------------------------------


def norm2(a):
    return float(np.vdot(a, a).real)


@dataclass
class MobiusDWF:
    """Even-odd preconditioned Mobius operator on a gauge field.

    Sec. 2.2: with M^4_{eo/oe} = D^w M_phi,
      D    = 1 - M_5^-1 M^4_eo M_5^-1 M^4_oe                  (eq. dirac_equation)
      A    = D^dag D                                           (eq. normal_equation)
    """
    U: np.ndarray
    Ls: int
    b: float
    c: float
    M5: float
    mf: float

    def __post_init__(self):
        T, Z, Y, X = self.U.shape[:4]
        self.dims = (X, Y, Z, T)
        self.vh = X * Y * Z * T // 2
        self.M5op = m5_matrix(self.Ls, self.b, self.c, self.M5, self.mf)
        self.M5inv = inverse5(self.M5op)
        self.Mphi = mphi_matrix(self.Ls, self.b, self.c, self.mf)
        self.M5inv_dag = adjoint5(self.M5inv)
        self.Mphi_dag = adjoint5(self.Mphi)

    # M^4 restricted to one parity block: D^w M_phi
    def m4(self, psi, out_parity):
        return wilson_hop(self.U, apply5(self.Mphi, psi), out_parity)

    def m4_dag(self, psi, out_parity):
        """(M^4_{out,in})^dag = M_phi^dag (D^w)^dag, mapping parity 1-out -> out."""
        return apply5(self.Mphi_dag, wilson_hop(self.U, psi, out_parity, dagger=True))

    def D(self, psi_e):
        """D psi_e = psi_e - M5^-1 M^4_eo M5^-1 M^4_oe psi_e."""
        t = self.m4(psi_e, 1)
        t = apply5(self.M5inv, t)
        t = self.m4(t, 0)
        t = apply5(self.M5inv, t)
        return psi_e - t

    def Ddag(self, chi_e):
        """D^dag = 1 - (M^4_oe)^dag M5^-dag (M^4_eo)^dag M5^-dag."""
        t = apply5(self.M5inv_dag, chi_e)
        t = self.m4_dag(t, 1)          # (M^4_eo)^dag: even -> odd
        t = apply5(self.M5inv_dag, t)
        t = self.m4_dag(t, 0)          # (M^4_oe)^dag: odd -> even
        return chi_e - t

    def A(self, psi_e):
        """A = D^dag D (Sec. 2.3, eq. DdagD)."""
        return self.Ddag(self.D(psi_e))

    # the unpreconditioned 5D operator on both parities (Sec. 2.2 block form)
    def full(self, psi_e, psi_o):
        """[[M_5, M^4_eo], [M^4_oe, M_5]] (psi_e, psi_o)."""
        phi_e = apply5(self.M5op, psi_e) + self.m4(psi_o, 0)
        phi_o = self.m4(psi_e, 1) + apply5(self.M5op, psi_o)
        return phi_e, phi_o

    def phi_hat(self, phi_e, phi_o):
        """phi^_e = M5^-1 phi_e - M5^-1 M^4_eo M5^-1 phi_o (eq. dirac_equation)."""
        t = apply5(self.M5inv, phi_o)
        t = self.m4(t, 0)
        return apply5(self.M5inv, phi_e) - apply5(self.M5inv, t)

    def reconstruct_odd(self, psi_e, phi_o):
        """psi_o = M5^-1 (phi_o - M^4_oe psi_e), the second block row."""
        return apply5(self.M5inv, phi_o - self.m4(psi_e, 1))


# --------------------------------------------------------------------------
# subdomains and the local operator A_s (Sec. 2.3-2.4)
# --------------------------------------------------------------------------


def tiling_ok(dims, sub):
    """Tilings on which A_s = R_s A R_s^T is what a zero pad of two sites
    around the subdomain evaluates: even extents that divide the lattice, and
    in every partitioned direction at least four sites outside the subdomain."""
    for d, s in zip(dims, sub):
        if d % 2 or s % 2 or s <= 0 or d % s:
            return False
        if s < d and d - s < 4:
            return False
    return True


@dataclass
class Tiling:
    """Block decomposition of the even sites into subdomains (Sec. 2.1, 2.4)."""
    dims: tuple
    sub: tuple
    index: list = field(init=False)

    def __post_init__(self):
        self.dims = tuple(int(d) for d in self.dims)
        self.sub = tuple(int(s) for s in self.sub)
        if not tiling_ok(self.dims, self.sub):
            raise ValueError(f"tiling {self.sub} not valid on {self.dims}")
        nb = [d // s for d, s in zip(self.dims, self.sub)]
        c = parity_coords(self.dims, 0)
        bx = [c[:, mu] // self.sub[mu] for mu in range(4)]
        label = ((bx[3] * nb[2] + bx[2]) * nb[1] + bx[1]) * nb[0] + bx[0]
        self.nsub = int(np.prod(nb))
        self.label = label
        self.index = [np.nonzero(label == k)[0] for k in range(self.nsub)]

    def restrict(self, v):
        """R_s v for every s: [nsub][Ls][n_s][4][3]."""
        return np.stack([v[:, idx] for idx in self.index])

    def embed(self, vs, vh):
        """R_s^T v_s for every s, each into its own full even field."""
        nsub, Ls = vs.shape[:2]
        out = np.zeros((nsub, Ls, vh, 4, 3), dtype=np.complex128)
        for k, idx in enumerate(self.index):
            out[k][:, idx] = vs[k]
        return out

    def prolong(self, vs, vh):
        """sum_s R_s^T v_s into one full even field."""
        Ls = vs.shape[1]
        out = np.zeros((Ls, vh, 4, 3), dtype=np.complex128)
        for k, idx in enumerate(self.index):
            out[:, idx] = vs[k]
        return out


def padded_operator(op: MobiusDWF, tiling: Tiling, k):
    """The padded field of Sec. 3.1.2 for subdomain k, as an operator of its
    own: a lattice made of the subdomain and a pad of two sites on both sides
    of every partitioned direction, carrying the original links there, with
    zero links from the last site of the box in each partitioned direction
    (so no hop leaves or re-enters the padded box: zero boundary beyond the
    pad).  Unpartitioned directions keep their periodic links.

    Returns the padded operator and the single-parity indices, in it, of the
    subdomain's even sites (in the order of ``tiling.index[k]``)."""
    dims, sub = tiling.dims, tiling.sub
    part = [s < d for d, s in zip(dims, sub)]
    nb = [d // s for d, s in zip(dims, sub)]
    bx = [k % nb[0], (k // nb[0]) % nb[1], (k // (nb[0] * nb[1])) % nb[2], k // (nb[0] * nb[1] * nb[2])]
    origin = [bx[m] * sub[m] for m in range(4)]
    L = [sub[m] + 4 if part[m] else dims[m] for m in range(4)]
    # global coordinate of every local coordinate, per direction
    g = [(origin[m] - 2 + np.arange(L[m])) % dims[m] if part[m] else np.arange(L[m]) for m in range(4)]
    Upad = op.U[np.ix_(g[3], g[2], g[1], g[0])].copy()          # [T][Z][Y][X][mu][3][3]
    for m in range(4):
        if part[m]:
            sl = [slice(None)] * 4
            sl[3 - m] = L[m] - 1                                 # array axes are (t, z, y, x)
            Upad[tuple(sl) + (m,)] = 0.0
    pop = MobiusDWF(Upad, op.Ls, op.b, op.c, op.M5, op.mf)
    cg = parity_coords(dims, 0)[tiling.index[k]]
    loc = np.stack([(cg[:, m] - origin[m] + 2) if part[m] else cg[:, m] for m in range(4)], axis=1)
    lex = loc[:, 0] + L[0] * (loc[:, 1] + L[1] * (loc[:, 2] + L[2] * loc[:, 3]))
    return pop, lex // 2


def local_operator(op: MobiusDWF, tiling: Tiling, vs, subset=None, batch=8, padded=False):
    """A_s v_s = R_s A R_s^T v_s for each subdomain (Sec. 2.3, eq. diri: the
    Dirichlet condition is imposed on the whole four-hop operator, so paths
    that leave the subdomain and return -- the snake terms -- are kept).

    Each v_s is embedded (zero elsewhere) into its own full even field, the
    full A is applied, and the result is restricted back; ``batch`` fields go
    through A together.  With ``padded`` each A_s is applied on the padded
    field of its subdomain instead (``padded_operator``, Sec. 3.1.2), which
    equals R_s A R_s^T on every tiling ``tiling_ok`` accepts and costs the
    padded box instead of the whole lattice."""
    ids = list(range(tiling.nsub)) if subset is None else list(subset)
    if padded:
        out = np.empty_like(vs)
        for j, k in enumerate(ids):
            pop, idx = padded_operator(op, tiling, k)
            full = np.zeros((op.Ls, pop.vh, 4, 3), dtype=np.complex128)
            full[:, idx] = vs[j]
            out[j] = pop.A(full)[:, idx]
        return out
    out = np.empty_like(vs)
    for j0 in range(0, len(ids), batch):
        chunk = ids[j0:j0 + batch]
        full = np.zeros((len(chunk), op.Ls, op.vh, 4, 3), dtype=np.complex128)
        for j, k in enumerate(chunk):
            full[j][:, tiling.index[k]] = vs[j0 + j]
        Af = op.A(full)
        for j, k in enumerate(chunk):
            out[j0 + j] = Af[j][:, tiling.index[k]]
    return out


def inner_cg(op: MobiusDWF, tiling: Tiling, r, k, subset=None, padded=False):
    """Preconditioner z = (+)_s CG_k(A_s, r_s) (Sec. 2.4-2.5).

    On every subdomain independently: z = 0, res = r_s, p = res,
    rho = <res,res>; repeat k times: q = A_s p, alpha = rho/<p,q>,
    z += alpha p, res -= alpha q, rho' = <res,res>, p = res + (rho'/rho) p.
    No precision-based stop.  A subdomain whose rho or <p,q> is zero keeps
    its current z.  Returns the restricted solutions [nsub][Ls][n_s][4][3].
    ``padded``: A_s through the padded field (see ``local_operator``)."""
    ids = list(range(tiling.nsub)) if subset is None else list(subset)
    rs = np.stack([r[:, tiling.index[j]] for j in ids])
    z = np.zeros_like(rs)
    res = rs.copy()
    p = res.copy()
    rho = np.array([norm2(res[j]) for j in range(len(ids))])
    active = rho > 0.0
    for _ in range(k):
        q = local_operator(op, tiling, p, subset=ids, padded=padded)
        for j in range(len(ids)):
            if not active[j]:
                continue
            pq = np.vdot(p[j], q[j]).real
            if pq == 0.0:
                active[j] = False
                continue
            alpha = rho[j] / pq
            z[j] += alpha * p[j]
            res[j] -= alpha * q[j]
            rho_new = norm2(res[j])
            if rho_new == 0.0:
                active[j] = False
                continue
            beta = rho_new / rho[j]
            p[j] = res[j] + beta * p[j]
            rho[j] = rho_new
    return z


def truncated_local_operator(op: MobiusDWF, tiling: Tiling, vs, subset=None):
    """The operator eq. diri of Sec. 2.3 contrasts with A_s: the Dirichlet
    cut applied to every hop separately, D_s = 1 - M5^-1 |M^4_eo| M5^-1 |M^4_oe|
    and D_s^dag likewise, |.| keeping only sites of the subdomain (even and
    odd) after each hop, and A_trunc = D_s^dag D_s.  It drops the snake terms
    (paths that leave the subdomain and come back) and so differs from A_s;
    it is not part of the method and serves only as the comparator that
    shows an A_s test can see the snake terms."""
    ids = list(range(tiling.nsub)) if subset is None else list(subset)
    oc = parity_coords(tiling.dims, 1)
    nb = [d // s for d, s in zip(tiling.dims, tiling.sub)]
    bxo = [oc[:, m] // tiling.sub[m] for m in range(4)]
    label_odd = ((bxo[3] * nb[2] + bxo[2]) * nb[1] + bxo[1]) * nb[0] + bxo[0]
    out = np.empty_like(vs)
    for j, k in enumerate(ids):
        keep = {0: tiling.label == k, 1: label_odd == k}

        def cut(f, par):
            g = f.copy()
            g[:, ~keep[par]] = 0
            return g

        full = np.zeros((op.Ls, op.vh, 4, 3), dtype=np.complex128)
        full[:, tiling.index[k]] = vs[j]
        t = apply5(op.M5inv, cut(op.m4(full, 1), 1))
        d = full - apply5(op.M5inv, cut(op.m4(t, 0), 0))
        t = apply5(op.M5inv_dag, cut(op.m4_dag(apply5(op.M5inv_dag, d), 1), 1))
        a = d - cut(op.m4_dag(t, 0), 0)
        out[j] = a[:, tiling.index[k]]
    return out


def local_operator_stored(op: MobiusDWF, tiling: Tiling, vs, fmt, subset=None):
    """A_s v_s evaluated as the fused kernels of eq. detail (Sec. 3.1.3) on
    the padded field of each subdomain (Sec. 3.1.2), with every kernel's
    output field stored in ``fmt`` and read back (Sec. 3.2: the
    preconditioner's kernels load fixed-point fields, compute in single
    precision and store their output in the fixed-point format).  The input
    is stored first; then, with p the stored input,

        t0 = M_phi p                                    (kernel M_phi)
        a  = M_phi M5^-1 D^w t0                         (kernel M_phi M5^-1 D^w)
        c  = M5^-dag (p - M5^-1 D^w a)  = M5^-dag D p   (kernel M5^-dag M5^-1 D^w
                                                         with the 1 - ... of D)
        e  = M5^-dag M_phi^dag D^w^dag c                (kernel M5^-dag M_phi^dag D^w^dag)
        q  = M5^dag c - M_phi^dag D^w^dag e = D^dag D p (kernel M_phi^dag D^w^dag
                                                         with the 1 - ... of D^dag)

    each output stored.  How the two 1 - ... terms join the kernels is a
    reading (the paper skips them); with ``fmt = 'fp64'`` the chain is A_s
    exactly.  The fifth-dimension operators are applied one after another,
    each in FP64."""
    ids = list(range(tiling.nsub)) if subset is None else list(subset)
    S = lambda f: stored(f, fmt)   # noqa: E731
    out = np.empty_like(vs)
    for j, k in enumerate(ids):
        pop, idx = padded_operator(op, tiling, k)
        p = np.zeros((op.Ls, pop.vh, 4, 3), dtype=np.complex128)
        p[:, idx] = vs[j]
        p = S(p)
        t0 = S(apply5(pop.Mphi, p))
        a = S(apply5(pop.Mphi, apply5(pop.M5inv, wilson_hop(pop.U, t0, 1))))
        c = S(apply5(pop.M5inv_dag, p - apply5(pop.M5inv, wilson_hop(pop.U, a, 0))))
        e = S(apply5(pop.M5inv_dag, apply5(pop.Mphi_dag, wilson_hop(pop.U, c, 1, dagger=True))))
        q = S(apply5(adjoint5(pop.M5op), c) - apply5(pop.Mphi_dag, wilson_hop(pop.U, e, 0, dagger=True)))
        out[j] = q[:, idx]
    return out


def inner_cg_stored(op: MobiusDWF, tiling: Tiling, r, k, fmt, subset=None):
    """The k-step inner CG of ``inner_cg`` with the preconditioner's fields in
    ``fmt`` (Sec. 3.2: the inner CG's matrix multiplications and BLAS
    operations use the fixed-point formats): r_s is stored on entry, every
    vector an iteration produces (z, the residual, the search direction) is
    stored after its update, and q = A_s p comes from
    ``local_operator_stored``; the scalars are FP64 and computed from the
    stored vectors.  With ``fmt = 'fp64'`` it is ``inner_cg``."""
    ids = list(range(tiling.nsub)) if subset is None else list(subset)
    S = lambda f: stored(f, fmt)   # noqa: E731
    rs = S(np.stack([r[:, tiling.index[j]] for j in ids]))
    z = np.zeros_like(rs)
    res = rs.copy()
    p = res.copy()
    rho = np.array([norm2(res[j]) for j in range(len(ids))])
    active = rho > 0.0
    for _ in range(k):
        q = local_operator_stored(op, tiling, p, fmt, subset=ids)
        for j in range(len(ids)):
            if not active[j]:
                continue
            pq = np.vdot(p[j], q[j]).real
            if pq == 0.0:
                active[j] = False
                continue
            alpha = rho[j] / pq
            z[j] = S(z[j] + alpha * p[j])
            res[j] = S(res[j] - alpha * q[j])
            rho_new = norm2(res[j])
            if rho_new == 0.0:
                active[j] = False
                continue
            beta = rho_new / rho[j]
            p[j] = S(res[j] + beta * p[j])
            rho[j] = rho_new
    return z


def stored_links(U, fmt):
    """Links as the preconditioner's kernels hold them: for the 16- and 8-bit
    field formats every real and imaginary part rounded to the nearest FP16
    value (ties to even; a reading: the paper's low-precision kernels keep
    their links in 16 bits), for ``fp32`` to FP32, for ``fp64`` unchanged."""
    U = np.asarray(U, dtype=np.complex128)
    if fmt == "fp64":
        return U.copy()
    t = np.float32 if fmt == "fp32" else np.float16
    return U.real.astype(t).astype(np.float64) + 1j * U.imag.astype(t).astype(np.float64)


def precondition(op, tiling, r, k):
    """z = M^-1 r with M = (+)_s A_s approximated by k inner CG steps."""
    zs = inner_cg(op, tiling, r, k)
    return tiling.prolong(zs, op.vh)


# --------------------------------------------------------------------------
# outer solvers (Sec. 2.4, Alg. 1; Sec. 3.2 Polak-Ribiere beta)
# --------------------------------------------------------------------------


@dataclass
class SolveInfo:
    iters: int
    converged: bool
    history: list
    true_rel_resid: float


def pcg(op: MobiusDWF, b, tol, maxiter, precond=None, beta_rule="PR", x0=None,
        callback=None, coeffs=None):
    """Preconditioned CG on A x = b (Alg. 1).

    alpha = <r,z>/<p,Ap>, x += alpha p, r -= alpha Ap, z = M^-1 r,
    beta = <z_new, r_new - r_old>/<z_old, r_old> (Polak-Ribiere) or
    <z_new, r_new>/<z_old, r_old> (Fletcher-Reeves, as in Alg. 1), p = z + beta p.
    Stops when ||r|| / ||b|| <= tol.  Without ``precond`` z = r (plain CG).
    ``coeffs`` (a list, optional) receives (alpha, beta) of every iteration
    (beta None on the last one): for plain CG they define the Lanczos
    tridiagonal matrix of A, whose extreme eigenvalues estimate A's."""
    M = (lambda v: v) if precond is None else precond
    bnorm = np.sqrt(norm2(b))
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - op.A(x) if x0 is not None else b.copy()
    z = M(r)
    p = z.copy()
    rho = np.vdot(r, z).real
    hist = [np.sqrt(norm2(r)) / bnorm]
    converged = hist[-1] <= tol
    it = 0
    while not converged and it < maxiter:
        q = op.A(p)
        alpha = rho / np.vdot(p, q).real
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        hist.append(np.sqrt(norm2(r)) / bnorm)
        if callback is not None:
            callback(it, x, r)
        if hist[-1] <= tol:
            converged = True
            if coeffs is not None:
                coeffs.append((alpha, None))
            break
        z = M(r)
        rz = np.vdot(z, r).real
        if beta_rule == "PR":
            beta = (rz - np.vdot(z, r_old).real) / rho
        else:
            beta = rz / rho
        if coeffs is not None:
            coeffs.append((alpha, beta))
        rho = rz
        p = z + beta * p
    true = np.sqrt(norm2(b - op.A(x))) / bnorm
    return x, SolveInfo(it, converged, hist, true)


def mspcg(op, tiling, b, k, tol, maxiter, x0=None):
    """MSPCG: Alg. 1 with the multi-splitting preconditioner and PR beta."""
    return pcg(op, b, tol, maxiter, precond=lambda r: precondition(op, tiling, r, k),
               beta_rule="PR", x0=x0)


def cg(op, b, tol, maxiter, x0=None, coeffs=None):
    """Plain CG (Alg. 1 with M = 1, Fletcher-Reeves beta)."""
    return pcg(op, b, tol, maxiter, precond=None, beta_rule="FR", x0=x0, coeffs=coeffs)


# --------------------------------------------------------------------------
# scaled low-precision storage (Sec. 3.2, fixed-point formats)
# --------------------------------------------------------------------------

STORAGE_FORMATS = ("fp64", "fp32", "fp16", "bf16", "int8")


def stored(psi, fmt):
    """The value a field takes after it is stored in ``fmt`` and read back.

    Sec. 3.2 stores each colour-spinor (3 colours x 4 spins x complex = 24
    reals) as small numbers n with one single-precision scale, the value
    being n / limit x scale.  Readings (the paper fixes no rounding rule,
    and its 16-bit format is an integer one; here the 16-bit formats are
    floating point):

    * every real is first rounded to FP32, and m is the largest magnitude of
      the 24 FP32 reals of the site;
    * ``fp16`` / ``bf16``: n = the FP32 product v x (1/m) rounded to nearest,
      ties to even, in the 16-bit float format; limit 1, scale m;
    * ``int8``: n = v x (127/m), the reciprocal and the product each rounded
      to FP32, rounded to the nearest integer, ties to even, in [-127, 127];
      limit 127, scale m;
    * a site with m = 0 reads back as zeros.

    The read-back value is formed in FP64 from n and m as the definition
    writes it.  ``fp64`` is the identity and ``fp32`` the rounding of every
    real to FP32.  ``psi`` is complex with the 4 x 3 spin-colour components
    in its last two axes.
    """
    if fmt not in STORAGE_FORMATS:
        raise ValueError(fmt)
    psi = np.asarray(psi, dtype=np.complex128)
    if fmt == "fp64":
        return psi.copy()
    lead = psi.shape[:-2]
    v = np.stack([psi.real, psi.imag], axis=-1).reshape(lead + (24,))
    x = v.astype(np.float32)
    if fmt == "fp32":
        out = x.astype(np.float64)
    else:
        m = np.max(np.abs(x), axis=-1, keepdims=True)
        safe = np.where(m > 0, m, np.float32(1))
        if fmt == "int8":
            inv = np.float32(127) / safe                 # FP32, correctly rounded
            n = np.clip(np.rint(x * inv), -127, 127)     # rint: ties to even
            out = n.astype(np.float64) / 127.0 * m.astype(np.float64)
        else:
            t = x * (np.float32(1) / safe)               # FP32 product
            if fmt == "fp16":
                n = t.astype(np.float16).astype(np.float64)
            else:
                import torch
                n = torch.from_numpy(np.ascontiguousarray(t)).to(torch.bfloat16).to(torch.float64).numpy()
            out = n * m.astype(np.float64)
        out = np.where(m > 0, out, 0.0)
    out = out.reshape(lead + (4, 3, 2))
    return out[..., 0] + 1j * out[..., 1]


# --------------------------------------------------------------------------
# reduced-Ls preconditioner (Sec. 3.3)
# --------------------------------------------------------------------------


def transform(Tm, v):
    """[T v](s, x, mu, c) = sum_{t, nu} T[s, mu, t, nu] v(t, x, nu, c).

    Sec. 3.3: T maps a field with Ls slices to one with Lhat slices, mixes
    spin and the fifth dimension and is the identity in colour and on the
    4D sites.  ``Tm`` has shape (Lhat, 4, Ls, 4), ``v`` (..., Ls, V/2, 4, 3)."""
    return np.einsum("smtn,...txnc->...sxmc", Tm, v)


def transform_dag(Tm, w):
    """T^dag w, with [T^dag]_{t nu, s mu} = conj(T_{s mu, t nu})."""
    return np.einsum("smtn,...sxmc->...txnc", Tm.conj(), w)


def local_op_full(op, tiling, v):
    """(+)_s A_s applied to a full even field: every subdomain's part through
    its own local operator, the results put back in place."""
    return tiling.prolong(local_operator(op, tiling, tiling.restrict(v)), op.vh)


def reduced_precondition(op_hat, tiling, Tm, mu, r, k, inverse=None):
    """z = (T^dag Mhat^-1 T + mu 1) r (Sec. 3.3), where Mhat^-1 is the k-step
    inner CG on the reduced-Ls local operator (+)_s Ahat_s, exactly as the
    full-Ls preconditioner applies M^-1.  ``inverse`` replaces Mhat^-1 by a
    given linear map (used by the gradient checks)."""
    rh = transform(Tm, r)
    zh = inverse(rh) if inverse is not None else precondition(op_hat, tiling, rh, k)
    return transform_dag(Tm, zh) + mu * r


def outer_sum(f, g):
    """G[s, mu, t, nu] = sum over 4D sites and colour of f(s, x, mu, c) conj(g(t, x, nu, c))."""
    return np.einsum("...sxmc,...txnc->smtn", f, g.conj())


def chi2(op, op_hat, tiling, Tm, mu, vs, k, inverse=None, gradient=False):
    """Training loss of Sec. 3.3 and its gradient with respect to T.

    chi^2 = sum_i |M (T^dag Mhat^-1 T + mu) v_i - v_i|^2 with M = (+)_s A_s,
    the operator whose k-step inverse the full-Ls preconditioner applies.

    Gradient (derived here; the paper states that it is analytic): with
    H = Mhat^-1 taken as a Hermitian linear map, e_i the residual above,
    m_i = M e_i, b_i = H T v_i and a_i = H T m_i,
        d chi^2 / d Re T + i d chi^2 / d Im T
            = 2 sum_i [ outer_sum(b_i, m_i) + outer_sum(a_i, v_i) ].
    With the k-step CG as H (not linear in its input) this is the gradient
    of the linearised loss, which the training uses as its direction."""
    Hinv = inverse if inverse is not None else (lambda x: precondition(op_hat, tiling, x, k))
    total = 0.0
    g = np.zeros_like(Tm, dtype=np.complex128)
    for v in vs:
        b = Hinv(transform(Tm, v))
        e = local_op_full(op, tiling, transform_dag(Tm, b) + mu * v) - v
        total += norm2(e)
        if gradient:
            m = local_op_full(op, tiling, e)
            a = Hinv(transform(Tm, m))
            g += 2.0 * (outer_sum(b, m) + outer_sum(a, v))
    return (total, g) if gradient else total


def line_quartic(op, op_hat, tiling, Tm, d, mu, vs, k, inverse=None):
    """Coefficients c_0..c_4 of chi^2(T + eta d) = sum_j c_j eta^j with Mhat^-1
    taken as linear (as the gradient takes it): per vector, with
    Ha = Mhat^-1 T v and Hb = Mhat^-1 d v,
        e(eta) = e0 + eta e1 + eta^2 e2,
        e0 = M (T^dag Ha + mu v) - v,  e1 = M (T^dag Hb + d^dag Ha),  e2 = M d^dag Hb,
    and chi^2(eta) = sum |e(eta)|^2 expanded in eta."""
    Hinv = inverse if inverse is not None else (lambda x: precondition(op_hat, tiling, x, k))
    c = np.zeros(5)
    for v in vs:
        ha = Hinv(transform(Tm, v))
        hb = Hinv(transform(d, v))
        e0 = local_op_full(op, tiling, transform_dag(Tm, ha) + mu * v) - v
        e1 = local_op_full(op, tiling, transform_dag(Tm, hb) + transform_dag(d, ha))
        e2 = local_op_full(op, tiling, transform_dag(d, hb))
        re = lambda x, y: float(np.vdot(x, y).real)
        c += [norm2(e0), 2 * re(e0, e1), norm2(e1) + 2 * re(e0, e2), 2 * re(e1, e2), norm2(e2)]
    return c


def quartic_min(c):
    """Minimiser over eta >= 0 of sum_j c_j eta^j (c_4 > 0 or lower degree):
    the best of eta = 0 and the positive real roots of the derivative."""
    roots = np.roots([4 * c[4], 3 * c[3], 2 * c[2], c[1]]) if c[4] != 0 else np.roots([3 * c[3], 2 * c[2], c[1]])
    cand = [0.0] + [r.real for r in roots if abs(r.imag) <= 1e-9 * max(1.0, abs(r)) and r.real > 0]
    val = lambda e: (((c[4] * e + c[3]) * e + c[2]) * e + c[1]) * e + c[0]
    return min(cand, key=val)


def train_transform(op, op_hat, tiling, T0, mu, vs, k, iters, momentum=0.5, inverse=None):
    """Train T by line search along a momentum direction (Sec. 3.3).

    Readings (the paper names the two methods only): search direction
    d_j = -g_j + momentum * d_{j-1} (d_{-1} = 0), g_j the gradient of
    ``chi2``; T_{j+1} = T_j + eta_j d_j with eta_j the minimiser over
    eta >= 0 of the quartic ``line_quartic`` (chi^2 along d_j with Mhat^-1
    taken as linear, exact when it is).  Returns T and the chi^2 history."""
    T = np.array(T0, dtype=np.complex128)
    d_prev = np.zeros_like(T)
    hist = [chi2(op, op_hat, tiling, T, mu, vs, k, inverse)]
    for _ in range(iters):
        _, g = chi2(op, op_hat, tiling, T, mu, vs, k, inverse, gradient=True)
        d = -g + momentum * d_prev
        if not np.any(d):
            break
        eta = quartic_min(line_quartic(op, op_hat, tiling, T, d, mu, vs, k, inverse))
        T = T + eta * d
        d_prev = d
        hist.append(chi2(op, op_hat, tiling, T, mu, vs, k, inverse))
    return T, hist
