"""The C-ABI library: it builds, loads, exports every symbol include/cpasvt.h
declares, and its host-only entry points behave (no GPU needed)."""
import ctypes
import os
import math

import numpy as np
import pytest

import paper_1705_07112_amd as cpa
from oracle import chebyshev
from oracle.shrinkage import Shrinkage


def test_library_exports_every_declared_symbol():
    names = cpa.declared_symbols()
    assert "cpa_shrink_dense" in names and "cpa_rpca_iterate" in names
    lib = cpa.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert set(cpa._SIGS) == set(names)


def test_status_strings_and_defaults():
    assert cpa.status_string(0) == "CPA_OK"
    assert cpa.status_string(6) == "CPA_ERR_BOUND"
    o = cpa.CpaOpts()
    cpa.lib().cpa_default_opts(ctypes.byref(o))
    assert o.K == 16 and o.bound == 0 and o.power_iters == 100
    assert o.power_tol == 1e-7 and o.margin == 0.01 and o.growth_tol == 1e-3


def test_struct_layouts_match_header(tmp_path):
    """Every field offset and struct size of the ctypes declarations equals what
    a C compiler makes of include/cpasvt.h."""
    import subprocess
    structs = {"cpa_shrinkage": cpa.CpaShrinkage, "cpa_opts": cpa.CpaOpts, "cpa_info": cpa.CpaInfo,
               "cpa_batched_tuning": cpa.CpaBatchedTuning, "cpa_sparsify": cpa.CpaSparsify}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "cpasvt.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(cpa.HEADER_PATH), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("kind,tau", [(0, 1.3), (1, 0.9), (2, 2.0)])
@pytest.mark.parametrize("K", [1, 2, 5, 16, 30, 64])
def test_host_coefficients_match_oracle(kind, tau, K):
    Lam = 9.0
    got = cpa.chebyshev_coeffs(cpa.CpaShrinkage(kind, 0, tau, 0.0, 0.0, 1.0), Lam, K)
    ref = chebyshev.coefficients_shifted(Shrinkage(kind, tau), Lam, K)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_host_coefficients_weighted_fn_and_edges():
    sh = cpa.weighted_fn(1.5, 0.4, 1e-3)
    ref = chebyshev.coefficients_shifted(Shrinkage(3, 0.0, 1.5, 0.4, 1e-3), 7.0, 20)
    assert np.max(np.abs(cpa.chebyshev_coeffs(sh, 7.0, 20) - ref)) < 1e-13
    assert np.all(cpa.chebyshev_coeffs(cpa.soft(1.0), 0.0, 8) == 0.0)
    # tau^2 >= Lambda: every node lies below the threshold
    assert np.all(cpa.chebyshev_coeffs(cpa.soft(3.0), 9.0, 8) == 0.0)


def test_argument_errors_before_any_device_work():
    lib = cpa.lib()
    c = (ctypes.c_double * 4)()
    with pytest.raises(cpa.CpaError) as e:
        cpa._check(lib.cpa_chebyshev_coeffs(ctypes.byref(cpa.soft(1.0)), 1.0, 0, c))
    assert e.value.status == 1
    with pytest.raises(cpa.CpaError):
        cpa._check(lib.cpa_chebyshev_coeffs(ctypes.byref(cpa.soft(1.0)), float("nan"), 4, c))
    with pytest.raises(cpa.CpaError):
        cpa._check(lib.cpa_chebyshev_coeffs(ctypes.byref(cpa.CpaShrinkage(9, 0, 1.0, 0, 0, 1)), 1.0, 4, c))
    o = cpa.Opts(K=4).to_c()
    sh = cpa.soft(1.0)
    # NULL context is rejected without touching the device
    st = lib.cpa_shrink_dense(None, None, 4, 4, ctypes.c_void_p(16), 4, ctypes.c_void_p(4096), 4,
                              ctypes.byref(sh), ctypes.byref(o), None)
    assert st == 1
    assert b"context" in lib.cpa_last_error()
    assert lib.cpa_rpca_state_floats(3, 5) == 105


def test_inpaint_and_sparsified_argument_errors_before_any_device_work():
    lib = cpa.lib()
    o = cpa.Opts(K=4).to_c()
    assert lib.cpa_inpaint_state_floats(3, 5) == 165
    assert lib.cpa_inpaint_state_floats(0, 5) == 0
    # NULL context
    st = lib.cpa_inpaint_iterate(None, None, 4, 4, ctypes.c_void_p(16), ctypes.c_void_p(4096), None,
                                 ctypes.c_void_p(1 << 20), 1, 1.0, 0.1, ctypes.byref(o), None)
    assert st == 1 and b"context" in lib.cpa_last_error()
    st = lib.cpa_inpaint_init(None, None, 4, 4, ctypes.c_void_p(16), ctypes.c_void_p(4096))
    assert st == 1 and b"context" in lib.cpa_last_error()
    sp = cpa.CpaSparsify(cpa.TRANSFORM_BLOCK_DCT8, 0, 4, 0.0)
    info = cpa.CpaInfo()
    st = lib.cpa_shrink_dense_sparsified(None, None, 8, 8, ctypes.c_void_p(16), 8, ctypes.c_void_p(4096), 8,
                                         ctypes.byref(cpa.soft(1.0)), ctypes.byref(o), ctypes.byref(sp),
                                         ctypes.byref(info), None, None)
    assert st == 1 and b"context" in lib.cpa_last_error()


def test_keep_schedule_matches_oracle():
    """cpa_keep_schedule (integer arithmetic) against the oracle's exact rationals,
    at and around the switch points and for sizes up to the largest int."""
    from oracle.sparsify import keep_schedule
    for d in (1, 7, 8, 44, 45, 96, 141, 1000, 1024, 1920, 46341, 2 ** 31 - 1):
        for E in (math.inf, 10.0, math.nextafter(0.03, 1.0), 0.03, 0.01, math.nextafter(6e-4, 1.0), 6e-4, 0.0, -1.0):
            assert cpa.keep_schedule(E, d) == keep_schedule(E, d), (d, E)
        for E_l, E_m in ((0.5, 0.2), (0.2, 0.2), (1e-3, 0.0)):
            for E in (0.6, 0.5, 0.3, 0.2, 0.1, 0.0):
                assert cpa.keep_schedule(E, d, E_l, E_m) == keep_schedule(E, d, E_l, E_m), (d, E, E_l, E_m)
    lib = cpa.lib()
    k = ctypes.c_int64(0)
    for args, status in (((math.nan, 8, 0.03, 6e-4), 1), ((1.0, 0, 0.03, 6e-4), 2), ((1.0, 8, 1e-4, 1e-2), 1),
                         ((1.0, 8, math.inf, 6e-4), 1), ((1.0, 8, 0.03, -1.0), 1)):
        assert lib.cpa_keep_schedule(*args, ctypes.byref(k)) == status, args
    assert lib.cpa_keep_schedule(1.0, 8, 0.03, 6e-4, None) == 1


def test_scheduled_inpaint_argument_errors_before_any_device_work():
    lib = cpa.lib()
    o = cpa.Opts(K=4).to_c()
    keeps = (ctypes.c_int64 * 2)()

    def call(ctx=None, transform=cpa.TRANSFORM_DCT, E_prev=math.inf, E_l=0.03, E_m=6e-4, Et=ctypes.c_void_p(1 << 24)):
        return lib.cpa_inpaint_iterate_scheduled(ctx, None, 16, 16, ctypes.c_void_p(16), ctypes.c_void_p(4096), None,
                                                 ctypes.c_void_p(1 << 20), 2, 1.0, 0.1, ctypes.byref(o), transform,
                                                 E_prev, E_l, E_m, Et, keeps)
    assert call(transform=9) == 1 and b"transform" in lib.cpa_last_error()
    assert call(E_prev=math.nan) == 1 and b"E_prev" in lib.cpa_last_error()
    assert call(E_l=1e-4, E_m=1e-2) == 1
    assert call(Et=None) == 1 and b"Et" in lib.cpa_last_error()
    assert call() == 1 and b"context" in lib.cpa_last_error()


@pytest.mark.parametrize("K", [1, 2, 7, 30, 256])
def test_damping_factors_match_oracle(K):
    import numpy as np
    from oracle import chebyshev
    for kind in ("none", "jackson", "lanczos"):
        g = np.array(cpa.damping_factors(K, kind))
        assert np.abs(g - chebyshev.damping_factors(K, kind)).max() <= 1e-14
    with pytest.raises(cpa.CpaError):
        cpa._check(cpa.lib().cpa_damping_factors(K, 3, ctypes.c_void_p(16)))
    o = cpa.Opts(K=4).to_c()
    o.damping = 5
    st = cpa.lib().cpa_shrink_dense(ctypes.c_void_p(1), None, 4, 4, ctypes.c_void_p(16), 4, ctypes.c_void_p(4096), 4,
                                    ctypes.byref(cpa.soft(1.0)), ctypes.byref(o), None)
    assert st != 0
