"""C-ABI library checks that need no GPU: it loads, exports every entry point
include/lbm.h declares, and rejects bad arguments before any launch."""
import ctypes as C
import math
import os
import re

import pytest

from paper_2012_14729_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_expected_api():
    names = header_functions()
    for n in ("lbm_init", "lbm_step", "lbm_moments", "lbm_workspace_bytes", "lbm_batch_create", "lbm_batch_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(header_functions()) == set(_lib.exported_names())


def test_params_struct_layout_matches_header():
    # 4 int32 + 14 doubles, doubles 8-aligned
    assert C.sizeof(_lib.LbmParams) == 4 * 4 + 14 * 8
    assert _lib.LbmParams.u_wall_lo.offset == 16


def good(**kw):
    d = dict(nx=64, ny=32, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.1, sigma=0.01, W=4.0, M=0.1, tau_h=0.8)
    d.update(kw)
    return _lib.make_params(**d)


def ws_bytes(p):
    n = C.c_size_t()
    code = _lib.lib().lbm_workspace_bytes(C.byref(p), C.byref(n))
    return code, n.value


def test_workspace_bytes_covers_state():
    code, n = ws_bytes(good())
    assert code == 0
    cells = 64 * 32
    assert n >= cells * (36 * 4 + 8 + 8)   # 2 x (f, h) + J + phi(FP64)


@pytest.mark.parametrize("bad", [dict(nx=4), dict(ny=7), dict(wall_x=3), dict(wall_y=-1), dict(tau_h=0.5),
                                 dict(nu1=0.0), dict(rho2=-1.0), dict(W=0.0), dict(sigma=float("nan")),
                                 dict(eps_n=0.0), dict(wall_x=1, wall_y=1, u_wall_hi=0.01),
                                 dict(wall_y=2, u_wall_lo=-0.01), dict(wall_x=2, wall_y=1, u_wall_hi=0.01),
                                 dict(rho0=float("inf"))])
def test_invalid_params_rejected(bad):
    code, _ = ws_bytes(good(**bad))
    assert code == _lib.LBM_E_INVAL
    assert _lib.lib().lbm_last_error()


def test_grid_size_limit():
    """State arrays are indexed with 64-bit element offsets, so a lattice
    may exceed 2^32 elements per state array; the padded plane (nx rounded
    up to 64, times ny) must stay below 2^31 nodes."""
    code, n = ws_bytes(good(nx=16384, ny=16384))         # 20 * 2^28 elements per state array
    assert code == 0 and n >= 16384 * 16384 * (2 * 20 * 4 + 8)
    ny_max = (2 ** 31 - 1) // 65536
    assert ws_bytes(good(nx=65536, ny=ny_max))[0] == 0
    code, _ = ws_bytes(good(nx=65536, ny=ny_max + 1))
    assert code == _lib.LBM_E_INVAL and b"2^31" in _lib.lib().lbm_last_error()
    code, _ = ws_bytes(good(nx=65536 - 63, ny=ny_max + 1))   # nx is padded to 64 first
    assert code == _lib.LBM_E_INVAL


@pytest.mark.parametrize("ok", [dict(wall_x=2), dict(wall_y=2), dict(wall_x=2, wall_y=2), dict(wall_x=2, wall_y=1),
                                dict(wall_y=1, u_wall_lo=-0.01, u_wall_hi=0.01)])
def test_wall_kinds_accepted(ok):
    code, n = ws_bytes(good(**ok))
    assert code == 0 and n > 0


def test_init_rejects_null_and_misaligned_workspace():
    lib = _lib.lib()
    p = good()
    h = C.c_void_p()
    assert lib.lbm_init(C.byref(h), C.byref(p), None, 1 << 30, C.c_void_p(256), None, None, None) == _lib.LBM_E_INVAL
    assert lib.lbm_init(C.byref(h), C.byref(p), C.c_void_p(4096 + 4), 1 << 30, C.c_void_p(256), None, None,
                        None) == _lib.LBM_E_INVAL
    code, n = ws_bytes(p)
    assert lib.lbm_init(C.byref(h), C.byref(p), C.c_void_p(1 << 20), n - 1, C.c_void_p(256), None, None,
                        None) == _lib.LBM_E_INVAL
    # only one u0 component
    assert lib.lbm_init(C.byref(h), C.byref(p), C.c_void_p(1 << 20), n, C.c_void_p(256), C.c_void_p(512), None,
                        None) == _lib.LBM_E_INVAL


def test_null_handle_rejected():
    lib = _lib.lib()
    assert lib.lbm_step(None, 1, 0, None) == _lib.LBM_E_INVAL
    assert lib.lbm_moments(None, 0, None, None, None, None, None, None) == _lib.LBM_E_INVAL
    assert lib.lbm_destroy(None) == 0


def test_batch_rejects_walls_and_bad_forms():
    lib = _lib.lib()
    arr = (_lib.LbmParams * 2)(good(), good(wall_y=1))
    n = C.c_size_t()
    assert lib.lbm_batch_workspace_bytes(arr, 2, C.byref(n)) == _lib.LBM_E_UNSUPPORTED
    arr = (_lib.LbmParams * 2)(good(), good(nx=4))
    assert lib.lbm_batch_workspace_bytes(arr, 2, C.byref(n)) == _lib.LBM_E_INVAL
    arr = (_lib.LbmParams * 2)(good(), good(nx=96))
    assert lib.lbm_batch_workspace_bytes(arr, 2, C.byref(n)) == 0 and n.value > 0
    assert lib.lbm_batch_workspace_bytes(arr, 0, C.byref(n)) == _lib.LBM_E_INVAL


def test_adjoint_lambda_guard_refuses_what_would_overrun_the_buffer():
    """lbm_adjoint_step reads and writes 20 nx ny doubles through lambda: the
    binding refuses any tensor that does not hold exactly that."""
    import torch
    from paper_2012_14729_amd import check_lambda
    ok = torch.zeros((20, 6, 8), dtype=torch.float64)
    assert check_lambda(ok, 6, 8, "cpu") is ok
    with pytest.raises(TypeError):
        check_lambda(ok.float(), 6, 8, "cpu")          # float32: half the bytes
    with pytest.raises(ValueError):
        check_lambda(torch.zeros((20, 6, 7), dtype=torch.float64), 6, 8, "cpu")
    with pytest.raises(ValueError):
        check_lambda(torch.zeros((20, 8, 6), dtype=torch.float64).transpose(1, 2), 6, 8, "cpu")
    with pytest.raises(ValueError):
        check_lambda(ok, 6, 8, "cuda:0")
    with pytest.raises(TypeError):
        check_lambda(ok.numpy(), 6, 8, "cpu")
