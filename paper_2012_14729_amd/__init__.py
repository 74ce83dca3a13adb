"""MI355X-native phase-field lattice Boltzmann hot path (arXiv:2012.14729).

Python face of the C ABI in include/lbm.h.  PyTorch provides device memory
and streams; every step of the method runs in the HIP kernels of
libpflbm.so.  The classes here only marshal arguments.

    sim = Simulation(params, phi0)          # params: dict or ParamSet-like
    sim.step(1000, "cpf2")
    m = sim.moments("cpf2")                 # dict of float32 cuda tensors
"""
from __future__ import annotations

import ctypes as C
import math

import torch

from ._lib import FORMS, LbmError, check, form_index, lib, make_params

__all__ = ["Simulation", "Batch", "FORMS", "LbmError", "params_struct"]


def params_struct(p):
    """lbm_params from a dict or an object with the same field names."""
    d = p if isinstance(p, dict) else {k: getattr(p, k) for k in (
        "nx", "ny", "wall_x", "wall_y", "u_wall_lo", "u_wall_hi", "rho1", "rho2", "nu1", "nu2", "sigma", "W",
        "M", "tau_h", "gx", "gy", "rho0", "eps_n") if hasattr(p, k)}
    d = dict(d)
    if d.get("rho0") is None:
        d["rho0"] = float("nan")
    return make_params(**d)


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _field(x, ny, nx, device):
    if x is None:
        return None
    t = torch.as_tensor(x, dtype=torch.float32, device=device).contiguous()
    if t.shape != (ny, nx):
        raise ValueError(f"field shape {tuple(t.shape)} != ({ny}, {nx})")
    return t


class Simulation:
    """One lattice (lbm_init / lbm_step / lbm_moments ...)."""

    def __init__(self, params, phi0, ux0=None, uy0=None, device="cuda", stream=None):
        L = lib()
        self.params = params_struct(params)
        self.nx, self.ny = self.params.nx, self.params.ny
        nbytes = C.c_size_t()
        check(L.lbm_workspace_bytes(C.byref(self.params), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        phi0 = _field(phi0, self.ny, self.nx, device)
        ux0 = _field(ux0, self.ny, self.nx, device)
        uy0 = _field(uy0, self.ny, self.nx, device)
        if (ux0 is None) != (uy0 is None):
            ux0 = torch.zeros_like(phi0) if ux0 is None else ux0
            uy0 = torch.zeros_like(phi0) if uy0 is None else uy0
        h = C.c_void_p()
        check(L.lbm_init(C.byref(h), C.byref(self.params), _ptr(self.workspace), nbytes.value, _ptr(phi0), _ptr(ux0),
                         _ptr(uy0), _stream(stream)))
        self._h = h
        self._keep = (phi0, ux0, uy0)   # inputs live until the init kernels have run on the stream

    def step(self, n, form, stream=None):
        check(lib().lbm_step(self._h, int(n), form_index(form), _stream(stream)))

    def moments(self, form, stream=None, out=None):
        out = out or {k: torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.workspace.device)
                      for k in ("phi", "rho", "ux", "uy", "P")}
        check(lib().lbm_moments(self._h, form_index(form), _ptr(out.get("phi")), _ptr(out.get("rho")),
                                _ptr(out.get("ux")), _ptr(out.get("uy")), _ptr(out.get("P")), _stream(stream)))
        return out

    def status(self, stream=None):
        d = C.c_int32()
        code = lib().lbm_status(self._h, C.byref(d), _stream(stream))
        if code not in (0, -3):
            check(code)
        return bool(d.value)

    @property
    def step_count(self):
        v = C.c_int64()
        check(lib().lbm_get_step(self._h, C.byref(v)))
        return v.value

    def state_bytes(self):
        v = C.c_size_t()
        check(lib().lbm_state_bytes(self._h, C.byref(v)))
        return v.value

    def save(self, stream=None):
        blob = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.workspace.device)
        check(lib().lbm_save(self._h, _ptr(blob), _stream(stream)))
        return blob

    def restore(self, blob, stream=None):
        check(lib().lbm_restore(self._h, _ptr(blob), _stream(stream)))

    def set_timing(self, enable=True):
        check(lib().lbm_set_timing(self._h, 1 if enable else 0))

    def kernel_time(self, kernel=0):
        ms, n = C.c_double(), C.c_int64()
        check(lib().lbm_kernel_time(self._h, int(kernel), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent instances advanced together (lbm_batch_*)."""

    def __init__(self, params_list, forms, phi0_list, device="cuda", stream=None):
        L = lib()
        n = len(params_list)
        self.count = n
        arr = (type(params_struct(params_list[0])) * n)(*[params_struct(p) for p in params_list])
        self._params = arr
        self.sizes = [(p.ny, p.nx) for p in arr]
        fa = (C.c_int32 * n)(*[form_index(f) for f in forms])
        nbytes = C.c_size_t()
        check(L.lbm_batch_workspace_bytes(arr, n, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        phis = [_field(x, ny, nx, device) for x, (ny, nx) in zip(phi0_list, self.sizes)]
        ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in phis])
        h = C.c_void_p()
        check(L.lbm_batch_create(C.byref(h), arr, fa, n, _ptr(self.workspace), nbytes.value, ptrs, _stream(stream)))
        self._h = h
        self._keep = phis

    def step(self, n, stream=None):
        check(lib().lbm_batch_step(self._h, int(n), _stream(stream)))

    def moments(self, k, stream=None):
        ny, nx = self.sizes[k]
        out = {key: torch.empty((ny, nx), dtype=torch.float32, device=self.workspace.device)
               for key in ("phi", "rho", "ux", "uy", "P")}
        check(lib().lbm_batch_moments(self._h, int(k), _ptr(out["phi"]), _ptr(out["rho"]), _ptr(out["ux"]),
                                      _ptr(out["uy"]), _ptr(out["P"]), _stream(stream)))
        return out

    def status(self, stream=None):
        flags = (C.c_int32 * self.count)()
        check(lib().lbm_batch_status(self._h, flags, _stream(stream)))
        return [bool(v) for v in flags]

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
