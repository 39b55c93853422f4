"""The entry point that allocates nothing (mspcg_apply_device_noalloc)
against mspcg_apply_device, through the C ABI: two calls in a row on one
device, the second on a smaller lattice (a second handle), each compared
element by element with the allocating entry point's output on the same
input (same kernels, same inputs: identical results), and a request beyond
the static workspace rejected with INVALID_ARG."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _handle(dims, Ls, sub, seed):
    from paper_2104_05615_amd import MSPCG
    s = MSPCG(dims)
    s.load_gauge(W.gauge_field(dims, 0.5, seed))
    s.set_mobius(Ls, 1.5, 0.5, 1.8, 0.05)
    s.set_subdomains(sub)
    s.set_solver(inner_iters=3)
    return s


CASES = [((8, 8, 8, 8), 8, (4, 4, 4, 4), 41), ((4, 4, 4, 8), 4, (4, 4, 4, 4), 42)]
OPS = [("A", "fp32"), ("A", "fp64"), ("D", "fp16"), ("dslash_eo", "bf16"), ("A_sub", "fp16"), ("precond", "fp16"),
       ("A_sub", "int8")]


def test_noalloc_entry_matches_apply_device_on_two_calls():
    import torch
    handles = [(_handle(d, Ls, sub, seed), d, Ls) for d, Ls, sub, seed in CASES]
    for op, prec in OPS:
        for k, (s, dims, Ls) in enumerate(handles):   # the second call has the smaller input
            n = Ls * int(np.prod(dims)) // 2 * 24
            g = torch.Generator(device="cuda")
            g.manual_seed(100 + k)
            x = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
            ref = torch.empty_like(x)
            got = torch.full_like(x, float("nan"))
            say(f"[gpu] noalloc {op} {prec} dims={dims} Ls={Ls}")
            s.apply_device(op, prec, x.data_ptr(), ref.data_ptr())
            torch.cuda.synchronize()
            s.apply_device_noalloc(op, prec, x.data_ptr(), got.data_ptr())
            torch.cuda.synchronize()
            assert torch.equal(got, ref), (op, prec, dims, float((got - ref).abs().max()))


def test_noalloc_entry_rejects_workspace_beyond_the_static_array():
    import torch
    from paper_2104_05615_amd import MSPCG, MSPCGError
    dims, Ls = (16, 16, 16, 32), 12      # an FP32 A needs ~5 x 75 MB: beyond 128 MiB
    s = MSPCG(dims)
    s.load_gauge(W.gauge_field(dims, 0.5, 43))
    s.set_mobius(Ls, 1.5, 0.5, 1.8, 0.05)
    n = Ls * int(np.prod(dims)) // 2 * 24
    x = torch.zeros(n, device="cuda", dtype=torch.float64)
    y = torch.empty_like(x)
    say(f"[gpu] noalloc A fp32 dims={dims} Ls={Ls}: expect INVALID_ARG")
    with pytest.raises(MSPCGError) as e:
        s.apply_device_noalloc("A", "fp32", x.data_ptr(), y.data_ptr())
    assert e.value.status == -1
    # a later call that fits still works
    s2 = _handle((4, 4, 4, 8), 4, (4, 4, 4, 4), 44)
    m = 4 * 4 * 4 * 4 * 8 // 2 * 24
    a = torch.randn(m, device="cuda", dtype=torch.float64)
    r1, r2 = torch.empty_like(a), torch.empty_like(a)
    s2.apply_device("A", "fp32", a.data_ptr(), r1.data_ptr())
    s2.apply_device_noalloc("A", "fp32", a.data_ptr(), r2.data_ptr())
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
