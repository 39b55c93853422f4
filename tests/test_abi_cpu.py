"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/mspcg.h declares, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "mspcg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mspcg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_2104_05615_amd as M
    lib = ctypes.CDLL(M.LIB_PATH)
    decl = header_functions()
    assert len(decl) >= 12
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(decl) == sorted(M.EXPORTED)


def test_create_validation_and_state_errors():
    import paper_2104_05615_amd as M
    h = ctypes.c_void_p()
    bad = (ctypes.c_int32 * 4)(8, 8, 7, 8)
    assert M.mspcg_create(ctypes.byref(h), bad, 0) == M.MSPCG_ERR_INVALID_ARG
    assert "even" in M.mspcg_last_error().decode()
    ok = (ctypes.c_int32 * 4)(8, 8, 8, 8)
    assert M.mspcg_create(ctypes.byref(h), ok, -1) == M.MSPCG_ERR_INVALID_ARG
    assert M.mspcg_create(ctypes.byref(h), ok, 0) == M.MSPCG_OK
    try:
        # tilings: validated before any device work
        for sub, code in [((3, 4, 4, 4), M.MSPCG_ERR_BAD_TILING),     # odd
                          ((6, 4, 4, 4), M.MSPCG_ERR_BAD_TILING),     # does not divide 8
                          ((6, 8, 8, 8), M.MSPCG_ERR_BAD_TILING)]:
            assert M.mspcg_set_subdomains(h, (ctypes.c_int32 * 4)(*sub)) == code
        assert M.mspcg_set_mobius(h, 1, 1.5, 0.5, 1.8, 0.1) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_mobius(h, 40, 1.5, 0.5, 1.8, 0.1) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_mobius(h, 8, float("nan"), 0.5, 1.8, 0.1) == M.MSPCG_ERR_INVALID_ARG
        # a singular M5: b (4 - M5) + 1 = 0
        assert M.mspcg_set_mobius(h, 8, 1.0, 0.5, 5.0, 0.1) == M.MSPCG_ERR_INVALID_ARG
        p = M.mspcg_solver_params(-1.0, 10, 4, 2, 1, 0.1, 0, 1)
        assert M.mspcg_set_solver(h, ctypes.byref(p)) == M.MSPCG_ERR_INVALID_ARG
        p = M.mspcg_solver_params(1e-10, 10, 4, 2, 2, 0.1, 0, 1)        # FP16 outer
        assert M.mspcg_set_solver(h, ctypes.byref(p)) == M.MSPCG_ERR_INVALID_ARG
        p = M.mspcg_solver_params(1e-10, 10, 4, 2, 1, 0.1, 3, 1)        # beta rule
        assert M.mspcg_set_solver(h, ctypes.byref(p)) == M.MSPCG_ERR_INVALID_ARG
        p = M.mspcg_solver_params(1e-10, 10, 4, 2, 1, 0.1, 0, 1)
        assert M.mspcg_set_solver(h, ctypes.byref(p)) == M.MSPCG_OK
        buf = (ctypes.c_double * 16)()
        st = M.mspcg_stats()
        assert M.mspcg_solve(h, buf, buf, None, ctypes.byref(st)) == M.MSPCG_ERR_NO_GAUGE
        assert M.mspcg_apply(h, 99, 1, buf, buf) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_apply(h, 0, 7, buf, buf) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_apply(h, 0, 1, buf, buf) == M.MSPCG_ERR_NO_GAUGE
        assert M.mspcg_solve(h, None, buf, None, None) == M.MSPCG_ERR_INVALID_ARG
    finally:
        assert M.mspcg_destroy(h) == M.MSPCG_OK
    assert M.mspcg_destroy(None) == M.MSPCG_OK


def test_python_wrapper_raises_on_error():
    import paper_2104_05615_amd as M
    s = M.MSPCG((8, 8, 8, 8), device=0)
    with pytest.raises(M.MSPCGError) as e:
        s.set_subdomains((4, 4, 4, 6))     # 6 does not divide 8
    assert e.value.status == M.MSPCG_ERR_BAD_TILING
    s.close()


def test_tiling_rule_matches_oracle():
    """Library and oracle accept exactly the same tilings (each checks its own copy of the rule)."""
    import paper_2104_05615_amd as M
    import oracle
    dims = (8, 12, 16, 4)
    s = M.MSPCG(dims, device=0)
    try:
        for sx in (2, 4, 6, 8):
            for sy in (2, 4, 6, 12):
                for sz in (4, 8, 16):
                    for st in (2, 4):
                        sub = (sx, sy, sz, st)
                        want = oracle.tiling_ok(dims, sub)
                        try:
                            s.set_subdomains(sub)
                            got = True
                        except M.MSPCGError as e:
                            # a valid tiling on a machine without a GPU fails later, at the device
                            got = e.status != M.MSPCG_ERR_BAD_TILING
                        assert got == want, sub
    finally:
        s.close()


def test_batch_and_tuning_entry_points_validate_before_the_device():
    import paper_2104_05615_amd as M
    h = ctypes.c_void_p()
    assert M.mspcg_create(ctypes.byref(h), (ctypes.c_int32 * 4)(8, 8, 8, 8), 0) == M.MSPCG_OK
    try:
        buf = (ctypes.c_double * 16)()
        stats = (M.mspcg_stats * 2)()
        assert M.mspcg_solve_batch_device(h, 0, buf, buf, None, None, stats) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_solve_batch_device(h, 2000, buf, buf, None, None, stats) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_solve_batch_device(h, 2, None, buf, None, None, stats) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_solve_batch_device(h, 2, buf, buf, None, None, stats) == M.MSPCG_ERR_NO_GAUGE
        assert M.mspcg_autotune(h, 0) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_autotune(h, 2) == M.MSPCG_ERR_NO_GAUGE
        o, x, us = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        assert M.mspcg_get_schedule(h, 5, 1, ctypes.byref(o), ctypes.byref(x), ctypes.byref(us)) == \
            M.MSPCG_ERR_INVALID_ARG
        # untuned default: one RHS keeps the RHS-outer order, XCD ranges on
        assert M.mspcg_get_schedule(h, 0, 1, ctypes.byref(o), ctypes.byref(x), ctypes.byref(us)) == M.MSPCG_OK
        assert (o.value, x.value, us.value) == (0, 1, 0.0)
        assert M.mspcg_get_schedule(h, 2, 4, ctypes.byref(o), ctypes.byref(x), ctypes.byref(us)) == M.MSPCG_OK
        assert o.value == 1
        # block order of the full-lattice hops: chunked t sweep by default,
        # pinned by mspcg_set_schedule; the subdomain kind keeps its order
        t = ctypes.c_int32()
        assert M.mspcg_get_tchunk(h, 0, 1, ctypes.byref(t)) == M.MSPCG_OK and t.value == 3
        assert M.mspcg_get_tchunk(h, 2, 1, ctypes.byref(t)) == M.MSPCG_OK and t.value == 0
        assert M.mspcg_set_schedule(h, 3, 1, 0, 1, 0) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_schedule(h, 0, 0, 0, 1, 0) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_schedule(h, 0, 1, 2, 1, 0) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_schedule(h, 0, 1, 0, 1, 5) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_get_tchunk(h, 0, 1, None) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_schedule(h, 1, 1, 0, 0, 1) == M.MSPCG_OK
        assert M.mspcg_get_tchunk(h, 1, 1, ctypes.byref(t)) == M.MSPCG_OK and t.value == 1
        assert M.mspcg_get_schedule(h, 1, 1, ctypes.byref(o), ctypes.byref(x), ctypes.byref(us)) == M.MSPCG_OK
        assert (o.value, x.value) == (0, 0)
        assert M.mspcg_set_schedule(h, 2, 1, 0, 1, 4) == M.MSPCG_OK
        assert M.mspcg_get_tchunk(h, 2, 1, ctypes.byref(t)) == M.MSPCG_OK and t.value == 0
        assert M.mspcg_set_profiling(h, -1) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_set_profiling(h, 8) == M.MSPCG_OK and M.mspcg_set_profiling(h, 0) == M.MSPCG_OK
        e, a = ctypes.c_int64(), ctypes.c_int64()
        assert M.mspcg_footprint(h, 1, ctypes.byref(e), ctypes.byref(a)) == M.MSPCG_ERR_NO_PARAMS
        assert M.mspcg_share_gauge(h, h) == M.MSPCG_ERR_NO_GAUGE
    finally:
        M.mspcg_destroy(h)


def test_server_lifecycle_and_validation_without_device_work():
    import paper_2104_05615_amd as M
    s = ctypes.c_void_p()
    assert M.mspcg_server_create(ctypes.byref(s), 0, 0, 4) == M.MSPCG_ERR_INVALID_ARG
    assert M.mspcg_server_create(ctypes.byref(s), 0, 1 << 30, 0) == M.MSPCG_ERR_INVALID_ARG
    assert M.mspcg_server_create(ctypes.byref(s), 0, 1 << 30, 3) == M.MSPCG_OK
    try:
        info = M.mspcg_server_stats()
        assert M.mspcg_server_info(s, ctypes.byref(info)) == M.MSPCG_OK
        assert info.budget == 1 << 30 and info.bytes_in_use == 0 and info.inflight == 0
        buf = (ctypes.c_double * 16)()
        r = M.mspcg_request(0, 8, 1.5, 0.5, 1.8, 0.1, (ctypes.c_int32 * 4)(4, 4, 4, 4),
                            M._solver_params(), 1, ctypes.cast(buf, ctypes.c_void_p),
                            ctypes.cast(buf, ctypes.c_void_p))
        t = ctypes.c_int64()
        assert M.mspcg_server_submit(s, ctypes.byref(r), ctypes.byref(t)) == M.MSPCG_ERR_INVALID_ARG  # no field
        assert "field" in M.mspcg_last_error().decode()
        r.nrhs = 0
        assert M.mspcg_server_submit(s, ctypes.byref(r), ctypes.byref(t)) == M.MSPCG_ERR_INVALID_ARG
        d = ctypes.c_int32()
        assert M.mspcg_server_poll(s, 12345, ctypes.byref(d)) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_server_wait(s, 12345, None, None) == M.MSPCG_ERR_INVALID_ARG
    finally:
        assert M.mspcg_server_destroy(s) == M.MSPCG_OK
    assert M.mspcg_server_destroy(None) == M.MSPCG_OK


def test_reduced_ls_entry_points_validate_before_the_device():
    import paper_2104_05615_amd as M
    h = ctypes.c_void_p()
    assert M.mspcg_create(ctypes.byref(h), (ctypes.c_int32 * 4)(8, 8, 8, 8), 0) == M.MSPCG_OK
    try:
        T = (ctypes.c_double * (2 * 4 * 4 * 8 * 4))()
        # no Mobius parameters yet
        assert M.mspcg_set_reduced(h, 4, 1.5, 0.5, 0.1, T) == M.MSPCG_ERR_NO_PARAMS
        assert M.mspcg_set_reduced(h, 0, 0.0, 0.0, 0.0, None) == M.MSPCG_OK     # switching off is always fine
        L = ctypes.c_int32(7)
        assert M.mspcg_get_reduced(h, ctypes.byref(L), None) == M.MSPCG_OK and L.value == 0
        c = ctypes.c_double()
        buf = (ctypes.c_double * 16)()
        assert M.mspcg_reduced_loss(h, 1, buf, ctypes.byref(c), None) == M.MSPCG_ERR_NO_GAUGE
        assert M.mspcg_reduced_loss(h, 0, buf, ctypes.byref(c), None) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_train_reduced(h, 1, buf, -1, 0.5, None) == M.MSPCG_ERR_INVALID_ARG
        assert M.mspcg_train_reduced(h, 1, buf, 2, float("nan"), None) == M.MSPCG_ERR_INVALID_ARG
    finally:
        M.mspcg_destroy(h)


def test_32bit_addressing_limits_are_rejected_before_the_device():
    """Every array of one right-hand side is addressed with 32-bit buffer
    ranges and offsets: sizes that would wrap are refused with INVALID_ARG
    before any device work (the full-size positive cases run on the GPU)."""
    import paper_2104_05615_amd as M
    h = ctypes.c_void_p()
    # 48^3 x 96: the FP64 link records (V * 640 bytes = 6.8 GB) exceed 4 GiB
    assert M.mspcg_create(ctypes.byref(h), (ctypes.c_int32 * 4)(48, 48, 48, 96), 0) == M.MSPCG_ERR_INVALID_ARG
    assert "4 GiB" in M.mspcg_last_error().decode()
    # 1290^4 sites would overflow the 32-bit lexicographic index
    assert M.mspcg_create(ctypes.byref(h), (ctypes.c_int32 * 4)(1290, 1290, 1290, 1290), 0) == M.MSPCG_ERR_INVALID_ARG
    assert "2^31" in M.mspcg_last_error().decode()
    # 32^3 x 64 fits (FP64 links 1.3 GB) ...
    assert M.mspcg_create(ctypes.byref(h), (ctypes.c_int32 * 4)(32, 32, 32, 64), 0) == M.MSPCG_OK
    try:
        # ... but not with Ls = 32: an FP64 5D field is 6.4 GB
        assert M.mspcg_set_mobius(h, 32, 1.5, 0.5, 1.8, 0.1) == M.MSPCG_ERR_INVALID_ARG
        assert "FP64 field" in M.mspcg_last_error().decode()
    finally:
        M.mspcg_destroy(h)
