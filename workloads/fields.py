"""Seeded gauge fields, sources and gauge transformations (host FP64).

The random-link recipe is ``U = exp(i * eps * H)`` with ``H`` a traceless
Hermitian 3x3 matrix built from a matrix ``G`` of independent complex
Gaussians (real and imaginary parts N(0,1)): ``H = (G + G^dag)/2 - tr/3``.
The exponential is taken through the eigendecomposition of ``H``, so ``U`` is
unitary with unit determinant up to rounding.  Draws use numpy's PCG64
generator; links are drawn one time-slice at a time in the order
``t, z, y, x, mu`` so that the result does not depend on memory limits.
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _su3_from_gaussian(g: np.ndarray, eps: float) -> np.ndarray:
    """``exp(i eps H)`` for ``H`` the traceless Hermitian part of ``g``.

    ``g`` has shape ``(..., 3, 3, 2)`` (real, imaginary draws)."""
    G = g[..., 0] + 1j * g[..., 1]
    H = 0.5 * (G + np.conj(np.swapaxes(G, -1, -2)))
    tr = np.trace(H, axis1=-2, axis2=-1).real / 3.0
    H = H - tr[..., None, None] * np.eye(3)
    w, V = np.linalg.eigh(H)
    phase = np.exp(1j * eps * w)
    return np.einsum("...ik,...k,...jk->...ij", V, phase, np.conj(V))


def gauge_field(dims, eps: float, seed: int) -> np.ndarray:
    """Random SU(3) links ``U[T][Z][Y][X][4][3][3]`` (complex128)."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = _rng(seed)
    U = np.empty((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    for t in range(T):
        g = rng.standard_normal(size=(Z, Y, X, 4, 3, 3, 2))
        U[t] = _su3_from_gaussian(g, eps)
    return U


def unit_gauge_field(dims) -> np.ndarray:
    """Free field: every link is the 3x3 identity."""
    X, Y, Z, T = (int(d) for d in dims)
    U = np.zeros((T, Z, Y, X, 4, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1.0
    return U


def gaussian_source(dims, Ls: int, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Gaussian complex spinor on one parity: ``[Ls][V/2][4][3]``, every real
    and imaginary component N(0,1).  With ``nrhs`` a leading batch axis."""
    X, Y, Z, T = (int(d) for d in dims)
    vh = X * Y * Z * T // 2
    rng = _rng(seed)
    shape = (Ls, vh, 4, 3, 2) if nrhs is None else (nrhs, Ls, vh, 4, 3, 2)
    g = rng.standard_normal(size=shape)
    return g[..., 0] + 1j * g[..., 1]


def parity_coords(dims, parity: int) -> np.ndarray:
    """Coordinates ``(x, y, z, t)`` of the sites of one parity, in the order of
    the single-parity layout (``lex // 2``).  Shape ``(V/2, 4)``."""
    X, Y, Z, T = (int(d) for d in dims)
    vh = X * Y * Z * T // 2
    lex0 = 2 * np.arange(vh)
    x0 = lex0 % X
    y = (lex0 // X) % Y
    z = (lex0 // (X * Y)) % Z
    t = lex0 // (X * Y * Z)
    x = x0 + ((y + z + t + parity) & 1)
    return np.stack([x, y, z, t], axis=1)


def point_smeared_sources(dims, Ls: int, seed: int, nrhs: int = 12,
                          sigma: float = 2.0) -> np.ndarray:
    """``nrhs`` Gaussian-smeared point sources on the even sites.

    A site ``x0`` is drawn at random; source ``k`` is the spin-colour unit
    vector ``e_(k mod 12)`` times ``exp(-|x - x0|^2 / (2 sigma^2))`` (periodic
    distance), the same on every ``s``.  Shape ``[nrhs][Ls][V/2][4][3]``."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = _rng(seed)
    x0 = np.array([rng.integers(0, X), rng.integers(0, Y),
                   rng.integers(0, Z), rng.integers(0, T)])
    c = parity_coords(dims, 0)
    ext = np.array([X, Y, Z, T])
    d = np.abs(c - x0[None, :])
    d = np.minimum(d, ext[None, :] - d)
    prof = np.exp(-np.sum(d.astype(np.float64) ** 2, axis=1) / (2.0 * sigma * sigma))
    vh = c.shape[0]
    out = np.zeros((nrhs, Ls, vh, 4, 3), dtype=np.complex128)
    for k in range(nrhs):
        sp, col = divmod(k % 12, 3)
        out[k, :, :, sp, col] = prof[None, :]
    return out


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """One random SU(3) matrix per 4D site, ``Omega[T][Z][Y][X][3][3]``."""
    X, Y, Z, T = (int(d) for d in dims)
    rng = _rng(seed)
    g = rng.standard_normal(size=(T, Z, Y, X, 3, 3, 2))
    return _su3_from_gaussian(g, 1.0)


def gauge_transform_links(U: np.ndarray, Om: np.ndarray) -> np.ndarray:
    """``U_{x,mu} -> Omega_x U_{x,mu} Omega_{x+mu}^dag`` (periodic)."""
    out = np.empty_like(U)
    # axis of mu in the [T][Z][Y][X] array: x->3, y->2, z->1, t->0
    for mu, ax in enumerate((3, 2, 1, 0)):
        Om_fwd = np.roll(Om, -1, axis=ax)
        out[..., mu, :, :] = Om @ U[..., mu, :, :] @ np.conj(np.swapaxes(Om_fwd, -1, -2))
    return out


def gauge_transform_field(psi: np.ndarray, Om: np.ndarray, parity: int) -> np.ndarray:
    """``psi(x) -> Omega_x psi(x)`` on a single-parity field ``[...][Ls][V/2][4][3]``."""
    T, Z, Y, X = Om.shape[:4]
    c = parity_coords((X, Y, Z, T), parity)
    Om_sites = Om[c[:, 3], c[:, 2], c[:, 1], c[:, 0]]  # (V/2, 3, 3)
    return np.einsum("iab,...sipb->...sipa", Om_sites, psi)
