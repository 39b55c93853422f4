"""Pins for the oracle's scaled low-precision storage (``oracle.stored``).

Sec. 3.2 stores a colour-spinor's 24 reals as small numbers times one scale
per colour-spinor.  The checks tie the definition to properties fixed by
that format, each chosen so that a plausible mistake fails one of them:

* codes that are exactly representable read back exactly (fails truncation
  instead of rounding, a wrong limit, a scale taken per real);
* the error is at most half a step of the site's own scale (fails a global
  scale, rounding away from nearest, a limit other than 127);
* a small real next to a large one in the same site loses its digits, the
  same real in a site of its own keeps them (the scale is per colour-spinor);
* the site's largest real reads back exactly, codes stay in [-127, 127];
* ties go to the even integer (the rounding rule taken as a reading);
* a site of zeros reads back as zeros;
* the 16-bit float formats reproduce every value their format holds and
  round to nearest within half an ulp; the measured error of Gaussian sites
  matches the uniform-rounding model.
"""
import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(2104)


def site(vals):
    """A (1, 4, 3) complex site from 24 reals (re, im interleaved)."""
    v = np.asarray(vals, dtype=np.float64).reshape(4, 3, 2)
    return (v[..., 0] + 1j * v[..., 1])[None]


def reals(psi):
    return np.stack([psi.real, psi.imag], axis=-1).reshape(psi.shape[:-2] + (24,))


def test_exact_codes_read_back_exactly():
    for k in (-6, 0, 3):
        q = RNG.integers(-127, 128, size=(50, 24))
        q[:, 5] = 127 * RNG.choice([-1, 1], size=50)        # the site's largest code
        v = q / 127.0 * 2.0 ** k
        psi = site(v[0])
        for i in range(1, 50):
            psi = np.concatenate([psi, site(v[i])])
        assert np.array_equal(oracle.stored(psi, "int8"), psi)


def test_error_at_most_half_a_step_and_max_exact():
    g = RNG.standard_normal((200, 4, 3, 2)) * np.exp(RNG.uniform(-8, 8, size=(200, 1, 1, 1)))
    psi = g[..., 0] + 1j * g[..., 1]
    out = oracle.stored(psi, "int8")
    x = reals(psi).astype(np.float32).astype(np.float64)
    m = np.max(np.abs(x), axis=-1, keepdims=True)
    err = np.abs(reals(out) - x)
    assert np.all(err <= m / 254.0 * (1 + 1e-6))
    # the largest real of each site is a code of +-127: exact
    i = np.argmax(np.abs(x), axis=-1)
    assert np.array_equal(np.take_along_axis(reals(out), i[:, None], -1), np.take_along_axis(x, i[:, None], -1))
    # every read-back value is an integer multiple of m / 127 in [-m, m]
    n = reals(out) / m * 127.0
    assert np.all(np.abs(n - np.rint(n)) < 1e-9) and np.all(np.abs(n) <= 127 + 1e-9)


def test_scale_is_per_colour_spinor():
    a = np.zeros(24)
    a[0], a[7] = 1.0, 0.003          # 0.003 x 127 = 0.38: below half a step of this site
    b = np.zeros(24)
    b[7] = 0.003
    out = oracle.stored(np.concatenate([site(a), site(b)]), "int8")
    r = reals(out)
    assert r[0, 0] == 1.0 and r[0, 7] == 0.0
    assert abs(r[1, 7] - np.float32(0.003)) < 1e-12


def test_ties_round_to_even_and_zero_site():
    v = np.zeros(24)
    v[0] = 127.0                     # m = 127: the code of each real is the real itself
    v[1], v[2], v[3], v[4] = 2.5, 3.5, -2.5, 0.5
    r = reals(oracle.stored(site(v), "int8"))[0]
    assert list(r[:5]) == [127.0, 2.0, 4.0, -2.0, 0.0]
    z = oracle.stored(site(np.zeros(24)), "int8")
    assert np.array_equal(z, np.zeros_like(z))
    for fmt in oracle.STORAGE_FORMATS:
        assert not np.any(np.isnan(oracle.stored(site(np.zeros(24)), fmt)))


@pytest.mark.parametrize("fmt,mant", [("fp16", 11), ("bf16", 8)])
def test_sixteen_bit_float_formats(fmt, mant):
    # values the format holds, times a power of two, read back exactly
    e = RNG.integers(-6, 1, size=(40, 24))
    f = RNG.integers(1 << (mant - 1), 1 << mant, size=(40, 24)) / float(1 << (mant - 1))   # [1, 2), mant bits
    s = RNG.choice([-1.0, 1.0], size=(40, 24))
    v = s * f * 2.0 ** (e - 1)
    v[:, 0] = 1.0                    # m = 1: the stored numbers are the values themselves
    psi = np.concatenate([site(v[i] * 8.0) for i in range(40)])
    assert np.array_equal(oracle.stored(psi, fmt), psi)
    # general values: within half an ulp (of the format, at the scaled value) of the FP32 real
    g = RNG.standard_normal((100, 4, 3, 2))
    psi = g[..., 0] + 1j * g[..., 1]
    x = reals(psi).astype(np.float32).astype(np.float64)
    m = np.max(np.abs(x), axis=-1, keepdims=True)
    err = np.abs(reals(oracle.stored(psi, fmt)) - x) / m
    t = np.abs(x) / m
    assert np.all(err <= t * 2.0 ** -mant * (1 + 1e-5) + 2.0 ** -24 + 2.0 ** -25)


def test_gaussian_error_matches_uniform_rounding_model():
    """For Gaussian sites the int8 error is uniform in half a step of m / 127:
    relative L2 error sqrt(E[m^2] / (127^2 x 12)) / sigma."""
    g = RNG.standard_normal((20000, 4, 3, 2))
    psi = g[..., 0] + 1j * g[..., 1]
    out = oracle.stored(psi, "int8")
    e = np.linalg.norm(out - psi) / np.linalg.norm(psi)
    m = np.max(np.abs(reals(psi)), axis=-1)
    model = np.sqrt(np.mean(m ** 2) / (127.0 ** 2 * 12))
    assert abs(e / model - 1) < 0.03, (e, model)
    assert np.array_equal(oracle.stored(psi, "fp32"), psi.astype(np.complex64).astype(np.complex128))
    assert np.array_equal(oracle.stored(psi, "fp64"), psi)


# ---------------------------------------------------------------- storage points of the preconditioner

import workloads as W  # noqa: E402


def _case(dims=(8, 4, 4, 4), Ls=4, sub=(4, 4, 4, 4), seed=9):
    U = W.gauge_field(dims, 0.5, 11)
    op = oracle.MobiusDWF(U, Ls, 1.5, 0.5, 1.8, 0.1)
    til = oracle.Tiling(dims, sub)
    g = np.random.default_rng(seed).standard_normal((Ls, op.vh, 4, 3, 2))
    return U, op, til, g[..., 0] + 1j * g[..., 1]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dims,Ls,sub", [((8, 4, 4, 4), 4, (4, 4, 4, 4)), ((8, 8, 4, 2), 6, (4, 4, 4, 2))])
def test_fused_kernel_chain_is_the_local_operator(dims, Ls, sub):
    """The eq.-detail chain of fused kernels on the padded field, stored in
    FP64 (no rounding), equals A_s = R_s A R_s^T built by embedding into the
    whole lattice (pinned independently): a wrong grouping of the fifth-
    dimension operators, a dropped 1 - ... term or a wrong parity fails."""
    U, op, til, r = _case(dims, Ls, sub)
    vs = til.restrict(r)
    assert _rel(oracle.local_operator_stored(op, til, vs, "fp64"), oracle.local_operator(op, til, vs)) < 1e-14


def test_fused_kernel_chain_stores_every_kernel_output(monkeypatch):
    """Six storage points per subdomain: the input and the outputs of the five
    kernels (M_phi, M_phi M5^-1 D^w, M5^-dag M5^-1 D^w, M5^-dag M_phi^dag
    D^w^dag, M_phi^dag D^w^dag); each is a field of the padded box."""
    import oracle.dwf as D
    U, op, til, r = _case()
    vs = til.restrict(r)[:1]
    calls = []
    real = D.stored

    def spy(f, fmt):
        calls.append(f.shape)
        return real(f, fmt)

    monkeypatch.setattr(D, "stored", spy)
    D.local_operator_stored(op, til, vs, "fp16", subset=[0])
    pop, _ = oracle.padded_operator(op, til, 0)
    assert calls == [(op.Ls, pop.vh, 4, 3)] * 6


def test_stored_chain_error_follows_the_formats():
    """Against exact A_s the stored chain errs by a few roundings of its
    format: FP32 ~1e-7, FP16 (2^-11 relative steps) ~3e-4, BF16 (2^-8)
    ~2.5e-3, int8 (steps of m/127) ~1e-2, in that order, each within a
    factor of the one-store error of the input times the six stores."""
    U, op, til, r = _case()
    vs = til.restrict(r)
    ex = oracle.local_operator(op, til, vs)
    errs = {}
    for fmt in ("fp32", "fp16", "bf16", "int8"):
        one = _rel(oracle.stored(vs, fmt), vs)               # one store of the input
        e = _rel(oracle.local_operator_stored(op, til, vs, fmt), ex)
        assert 0.3 * one < e < 6 * one, (fmt, e, one)
        errs[fmt] = e
    assert errs["fp32"] < errs["fp16"] < errs["bf16"] < errs["int8"]


def test_stored_inner_cg():
    """In FP64 the stored inner CG is the inner CG; in the 16- and 8-bit
    formats it departs from it by the order of its format's rounding."""
    U, op, til, r = _case()
    z = oracle.inner_cg(op, til, r, 3)
    assert _rel(oracle.inner_cg_stored(op, til, r, 3, "fp64"), z) < 1e-14
    for fmt, lo, hi in (("fp16", 1e-4, 2e-3), ("bf16", 1e-3, 1e-2), ("int8", 3e-3, 4e-2)):
        e = _rel(oracle.inner_cg_stored(op, til, r, 3, fmt), z)
        assert lo < e < hi, (fmt, e)


def test_stored_links():
    """FP16 links: every real and imaginary part on the FP16 grid, within half
    an FP16 ulp of the FP64 value (values already on the grid unchanged);
    FP64 unchanged."""
    U = W.gauge_field((4, 4, 4, 4), 0.5, 5)
    L = oracle.stored_links(U, "fp16")
    for part in (L.real, L.imag):
        assert np.array_equal(part.astype(np.float16).astype(np.float64), part)
    x = np.concatenate([U.real.ravel(), U.imag.ravel()])
    y = np.concatenate([L.real.ravel(), L.imag.ravel()])
    nz = np.abs(x) > 2.0 ** -14
    assert np.all(np.abs(y - x)[nz] <= 2.0 ** -11 * np.abs(x)[nz] * (1 + 1e-12))
    assert np.array_equal(oracle.stored_links(L, "fp16"), L)
    assert np.array_equal(oracle.stored_links(U, "fp64"), U)
