"""Runs the library's step and adjoint, built for the host by the CPU
harness in this folder (hip/hip_runtime.h, hip_cpu_runtime.cpp), against
the oracle.  Host arrays stand in for device memory.  Invoked by
tests/test_cpu_kernels.py in a subprocess that preloads AddressSanitizer,
so an out-of-bounds access in a kernel aborts the run with a report.

    python tests/cpu_hip/driver.py <library.so> forward|adjoint

Prints one JSON object per case, then DONE.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402
from oracle import lbm_ref as R  # noqa: E402
from paper_2012_14729_amd import _lib  # noqa: E402  (ctypes declarations only; the GPU library is not loaded)

torch.set_num_threads(2)
FORMS = R.FORMS


def load(path):
    L = C.CDLL(path)
    for name, (res, args) in _lib._SIGS.items():
        fn = getattr(L, name, None)
        if fn is not None:
            fn.restype = res
            fn.argtypes = args
    return L


class Mem:
    """256-byte aligned host buffer standing in for a device allocation."""

    def __init__(self, nbytes):
        self.raw = np.zeros(nbytes + 256, np.uint8)
        off = (-self.raw.ctypes.data) % 256
        self.buf = self.raw[off:off + nbytes]
        self.ptr = C.c_void_p(self.buf.ctypes.data)


def ok(L, code):
    if code != 0:
        raise RuntimeError(f"lbm error {code}: {L.lbm_last_error().decode()}")


def f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32))


def ptr(a):
    return C.c_void_p(0 if a is None else a.ctypes.data)


def oracle_params(p):
    d = p.as_dict()
    d["rho0"] = None
    return R.Params(**d)


def t64(a):
    return None if a is None else torch.tensor(np.asarray(a, np.float32), dtype=torch.float64)


CASES = {
    "periodic_drop": lambda: (WL.ParamSet(nx=40, ny=20, rho1=5.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=0.01, W=3.0,
                                          M=0.05, tau_h=0.9), WL.droplet(40, 20, 6.0, 3.0, 17.3, 9.2), None, None),
    "shear_walls": lambda: WL.config_shear(nx=36, ny=18, R=5.0, Re=1.0, Ca=0.2),
    "box_gravity": lambda: (WL.ParamSet(nx=34, ny=19, wall_x=1, wall_y=1, rho1=3.0, rho2=1.0, nu1=0.1, nu2=0.1,
                                        sigma=0.01, W=3.0, M=0.05, tau_h=0.9, gx=2e-5, gy=-3e-5),
                            WL.droplet(34, 19, 6.0, 3.0, 15.6, 9.3), None, None),
}


class Sim:
    def __init__(self, L, p, phi0, ux0, uy0):
        self.L, self.p = L, p
        self.params = _lib.make_params(**{k: (float("nan") if v is None else v) for k, v in p.as_dict().items()})
        n = C.c_size_t()
        ok(L, L.lbm_workspace_bytes(C.byref(self.params), C.byref(n)))
        self.ws = Mem(n.value)
        self.phi0, self.ux0, self.uy0 = f32(phi0), None if ux0 is None else f32(ux0), None if uy0 is None else f32(uy0)
        h = C.c_void_p()
        ok(L, L.lbm_init(C.byref(h), C.byref(self.params), self.ws.ptr, n.value, ptr(self.phi0), ptr(self.ux0),
                         ptr(self.uy0), None))
        self.h = h

    def step(self, n, form):
        ok(self.L, self.L.lbm_step(self.h, n, FORMS.index(form), None))

    def moments(self, form):
        ny, nx = self.p.ny, self.p.nx
        out = {k: np.zeros((ny, nx), np.float32) for k in ("phi", "rho", "ux", "uy", "P")}
        ok(self.L, self.L.lbm_moments(self.h, FORMS.index(form), ptr(out["phi"]), ptr(out["rho"]), ptr(out["ux"]),
                                      ptr(out["uy"]), ptr(out["P"]), None))
        return out


def run_forward(L):
    cases = sorted(CASES)
    for j, form in enumerate(FORMS):   # every form, the boundary set-ups in turn
        case = cases[j % len(cases)]
        p, phi0, ux0, uy0 = CASES[case]()
        s = Sim(L, p, phi0, ux0, uy0)
        s.step(6, form)
        got = {k: v.astype(np.float64) for k, v in s.moments(form).items()}
        op = oracle_params(p)
        st = R.run(R.init(op, t64(phi0), t64(ux0), t64(uy0)), form, op, 6)
        ref = {k: v.numpy() for k, v in R.moments(st, form, op).items()}
        umax = float(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max())
        e = {"phi": float(np.abs(got["phi"] - ref["phi"]).max() / np.abs(ref["phi"]).max()),
             "u": float(max(np.abs(got["ux"] - ref["ux"]).max(), np.abs(got["uy"] - ref["uy"]).max()) / umax)}
        print(json.dumps({"kind": "forward", "case": case, "form": form, **e}), flush=True)


def run_adjoint(L):
    for case in sorted(CASES):
        p, phi0, ux0, uy0 = CASES[case]()
        for form in FORMS:
            k = 3
            op = oracle_params(p)
            sig = torch.tensor(op.sigma, dtype=torch.float64, requires_grad=True)
            M = torch.tensor(op.M, dtype=torch.float64, requires_grad=True)
            st = R.run(R.init(op, t64(phi0), t64(ux0), t64(uy0)), form, op, k)
            f = st["f"].clone().requires_grad_(True)
            h = st["h"].clone().requires_grad_(True)
            J = st["J"].clone().requires_grad_(True)
            q = R.Params(**{**op.__dict__, "sigma": sig, "M": M})
            nxt = R.step(dict(f=f, h=h, J=J, rho0=st["rho0"], t=k), form, q)
            out = torch.cat([nxt["f"], nxt["h"], nxt["J"]])
            g = torch.Generator().manual_seed(17)
            lam1 = torch.randn(out.shape, generator=g, dtype=torch.float64)
            gf, gh, gJ, gs, gm = torch.autograd.grad(out, (f, h, J, sig, M), grad_outputs=lam1)
            ref = torch.cat([gf, gh, gJ]).numpy()

            s = Sim(L, p, phi0, ux0, uy0)
            s.step(k, form)
            n = C.c_size_t()
            ok(L, L.lbm_adjoint_workspace_bytes(C.byref(s.params), C.byref(n)))
            aws = Mem(n.value)
            a = C.c_void_p()
            ok(L, L.lbm_adjoint_create(C.byref(a), s.h, aws.ptr, n.value))
            lin = np.ascontiguousarray(lam1.numpy())
            lout = np.zeros_like(lin)
            ok(L, L.lbm_adjoint_step(a, FORMS.index(form), ptr(lin), ptr(lout), None))
            ds, dm = C.c_double(), C.c_double()
            ok(L, L.lbm_adjoint_param_grads(a, C.byref(ds), C.byref(dm), None))
            L.lbm_adjoint_destroy(a)
            err = float(np.abs(lout - ref).max() / np.abs(ref).max())
            print(json.dumps({"kind": "adjoint", "case": case, "form": form, "lambda": err,
                              "dsigma": [ds.value, float(gs)], "dM": [dm.value, float(gm)]}), flush=True)


if __name__ == "__main__":
    L = load(sys.argv[1])
    {"forward": run_forward, "adjoint": run_adjoint}[sys.argv[2]](L)
    print("DONE", flush=True)
