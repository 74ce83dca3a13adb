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
import time

import torch

from ._lib import FORMS, LbmError, check, form_index, lib, make_params

__all__ = ["Simulation", "Batch", "Adjoint", "rollout", "adjoint_gradients", "check_lambda", "FORMS", "LbmError", "params_struct"]


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


def check_lambda(lam, ny, nx, device):
    """The adjoint entry points read and write 20 * nx * ny doubles through
    this pointer: refuse anything but a contiguous float64 [20, ny, nx]
    tensor on the simulation's device."""
    if not torch.is_tensor(lam):
        raise TypeError("lambda must be a torch tensor")
    if lam.dtype != torch.float64:
        raise TypeError(f"lambda must be float64, got {lam.dtype}")
    if tuple(lam.shape) != (20, ny, nx):
        raise ValueError(f"lambda shape {tuple(lam.shape)} != (20, {ny}, {nx})")
    if not lam.is_contiguous():
        raise ValueError("lambda must be contiguous")
    if lam.device != torch.device(device):
        raise ValueError(f"lambda is on {lam.device}, the simulation on {device}")
    return lam


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

    def hydro_pressure(self, form, stream=None, out=None):
        """p_h = P_sf - D_form of the current state (lbm_hydro_pressure)."""
        out = out if out is not None else torch.empty((self.ny, self.nx), dtype=torch.float32,
                                                      device=self.workspace.device)
        if (out.dtype != torch.float32 or tuple(out.shape) != (self.ny, self.nx) or not out.is_contiguous()
                or out.device != self.workspace.device):
            raise ValueError(f"out must be a contiguous float32 [{self.ny}, {self.nx}] tensor on "
                             f"{self.workspace.device}")
        check(lib().lbm_hydro_pressure(self._h, form_index(form), _ptr(out), _stream(stream)))
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

    def step_blobs(self, blob_in, blob_out, form, stream=None):
        """One step from the state in blob_in into blob_out (lbm_step_blobs);
        the simulation itself is not touched."""
        n = self.state_bytes()
        for b in (blob_in, blob_out):
            if not (torch.is_tensor(b) and b.dtype == torch.uint8 and b.numel() == n
                    and b.device == self.workspace.device):
                raise ValueError("blobs must be uint8 tensors from Simulation.save() on the same device")
        check(lib().lbm_step_blobs(self._h, _ptr(blob_in), _ptr(blob_out), form_index(form), _stream(stream)))
        return blob_out

    def set_timing(self, enable=True, period=1):
        """Time the kernels of every `period`-th step (lbm_set_timing); off if not enable."""
        check(lib().lbm_set_timing(self._h, int(period) if enable else 0))

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

    @property
    def config(self):
        """Launch shape chosen at creation: {split, fast, blocks_per_cu, ms_per_step}."""
        sp, fa, bp, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        check(lib().lbm_batch_config(self._h, C.byref(sp), C.byref(fa), C.byref(bp), C.byref(ms)))
        return {"split": sp.value, "fast": fa.value, "blocks_per_cu": bp.value, "ms_per_step": ms.value}

    def tile_shapes(self):
        """Tile shape (tile_x, tile_y) of every instance's step kernels."""
        out = []
        tx, ty = C.c_int32(), C.c_int32()
        for k in range(self.count):
            check(lib().lbm_batch_tile_shape(self._h, k, C.byref(tx), C.byref(ty)))
            out.append((tx.value, ty.value))
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Adjoint:
    """Adjoint of the step of one Simulation (lbm_adjoint_*).  The adjoint
    state is a float64 tensor [20, ny, nx]: dL/df_0..8, dL/dh_0..8, dL/dJ of
    the physical pre-collision state."""

    def __init__(self, sim: Simulation):
        L = lib()
        self.sim = sim
        n = C.c_size_t()
        check(L.lbm_adjoint_workspace_bytes(C.byref(sim.params), C.byref(n)))
        self.workspace = torch.empty(n.value, dtype=torch.uint8, device=sim.workspace.device)
        h = C.c_void_p()
        check(L.lbm_adjoint_create(C.byref(h), sim._h, _ptr(self.workspace), n.value))
        self._h = h

    def new_lambda(self):
        return torch.zeros((20, self.sim.ny, self.sim.nx), dtype=torch.float64, device=self.workspace.device)

    def seed_phi_misfit(self, target, stream=None):
        t = _field(target, self.sim.ny, self.sim.nx, self.workspace.device)
        lam = self.new_lambda()
        loss = C.c_double()
        check(lib().lbm_adjoint_seed_phi_misfit(self._h, _ptr(t), _ptr(lam), C.byref(loss), _stream(stream)))
        return lam, loss.value

    def _out(self, lam, out):
        if out is None:
            out = torch.empty_like(lam)
        check_lambda(out, self.sim.ny, self.sim.nx, self.workspace.device)
        if out.data_ptr() == lam.data_ptr():
            raise ValueError("the adjoint step writes lambda_n to a second array, not in place")
        return out

    def step(self, lam, form, out=None, stream=None):
        """lambda_n from lambda_{n+1} = lam about the simulation's current
        state; written to `out` (a new tensor if None), which is returned."""
        check_lambda(lam, self.sim.ny, self.sim.nx, self.workspace.device)
        out = self._out(lam, out)
        check(lib().lbm_adjoint_step(self._h, form_index(form), _ptr(lam), _ptr(out), _stream(stream)))
        return out

    def step_blob(self, blob, lam, form, out=None, stream=None):
        """Adjoint step about the state in `blob` (a Simulation.save() of this
        adjoint's simulation); lambda_n goes to `out` (new if None)."""
        check_lambda(lam, self.sim.ny, self.sim.nx, self.workspace.device)
        if not (torch.is_tensor(blob) and blob.dtype == torch.uint8 and blob.numel() == self.sim.state_bytes()
                and blob.device == self.workspace.device):
            raise ValueError("blob must be a uint8 tensor from Simulation.save() on the same device")
        out = self._out(lam, out)
        check(lib().lbm_adjoint_step_blob(self._h, _ptr(blob), form_index(form), _ptr(lam), _ptr(out),
                                          _stream(stream)))
        return out

    def step_blob_noalloc(self, blob, lam, form, out, stream=None):
        """step_blob through lbm_adjoint_step_blob_noalloc: its scratch is the
        library's own per-GPU array, so the call allocates nothing (`out` is
        required)."""
        check_lambda(lam, self.sim.ny, self.sim.nx, self.workspace.device)
        if not (torch.is_tensor(blob) and blob.dtype == torch.uint8 and blob.numel() == self.sim.state_bytes()
                and blob.device == self.workspace.device):
            raise ValueError("blob must be a uint8 tensor from Simulation.save() on the same device")
        out = self._out(lam, out)
        check(lib().lbm_adjoint_step_blob_noalloc(self._h, _ptr(blob), form_index(form), _ptr(lam), _ptr(out),
                                                  _stream(stream)))
        return out

    def init(self, lam, phi0, ux0=None, uy0=None, stream=None):
        dev = self.workspace.device
        check_lambda(lam, self.sim.ny, self.sim.nx, dev)
        p = _field(phi0, self.sim.ny, self.sim.nx, dev)
        ux = _field(ux0, self.sim.ny, self.sim.nx, dev)
        uy = _field(uy0, self.sim.ny, self.sim.nx, dev)
        if (ux is None) != (uy is None):
            ux = torch.zeros_like(p) if ux is None else ux
            uy = torch.zeros_like(p) if uy is None else uy
        d = torch.empty((self.sim.ny, self.sim.nx), dtype=torch.float64, device=dev)
        check(lib().lbm_adjoint_init(self._h, _ptr(p), _ptr(ux), _ptr(uy), _ptr(lam), _ptr(d), _stream(stream)))
        return d

    def param_grads(self, stream=None):
        ds, dm = C.c_double(), C.c_double()
        check(lib().lbm_adjoint_param_grads(self._h, C.byref(ds), C.byref(dm), _stream(stream)))
        return ds.value, dm.value

    def reset(self, stream=None):
        check(lib().lbm_adjoint_reset(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib().lbm_adjoint_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Checkpointed:
    """Forward pass of L = 1/2 sum (phi_T - target)^2 with a state checkpoint
    every `every` steps, and the adjoint pass over it.

    forward(): T steps from phi0, keeping (T / every) checkpoints; seeds
    lambda_T and computes L (lbm_adjoint_seed_phi_misfit).
    backward(): per segment in reverse, recompute the segment's per-step
    states from its checkpoint blob to blob (lbm_step_blobs, no copies) into
    a pool of `every - 1` state blobs (allocated once, reused by every
    segment), run the adjoint steps backwards over them; then the adjoint of
    the initialisation.  Memory: (T / every + every) states."""

    def __init__(self, params, form, T, phi0, target, ux0=None, uy0=None, every=None):
        self.form, self.T = form, int(T)
        self.every = max(1, int(math.ceil(math.sqrt(T)))) if every is None else int(every)
        self.phi0, self.ux0, self.uy0, self.target = phi0, ux0, uy0, target
        self.sim = Simulation(params, phi0, ux0, uy0, device=phi0.device)
        self.adj = Adjoint(self.sim)
        self.ckpt = []
        self.lam = None
        self.loss = None

    def forward(self, keep_checkpoints=True):
        sim = self.sim
        if keep_checkpoints:
            for t in range(0, self.T, self.every):
                self.ckpt.append(sim.save())
                sim.step(min(self.every, self.T - t), self.form)
        else:
            sim.step(self.T, self.form)
        self.lam, self.loss = self.adj.seed_phi_misfit(self.target)
        return self.loss

    def backward(self, overlap=True):
        """The adjoint pass.  overlap: recompute the next segment's states on
        a second stream (two pools, alternating) while the adjoint steps of
        the current one run; the kernels and their inputs are the same, so
        the results are bitwise those of the serial order."""
        if self.lam is None or (self.T > 0 and not self.ckpt):
            raise RuntimeError("backward needs a forward pass that kept its checkpoints")
        sim, adj, lam, every = self.sim, self.adj, self.lam, self.every
        spare = torch.empty_like(lam)   # lambda ping-pongs between two arrays
        npool = min(every, self.T) - 1
        nseg = len(self.ckpt)
        overlap = overlap and nseg > 1 and npool > 0
        pools = [[torch.zeros_like(self.ckpt[0]) for _ in range(npool)] if self.ckpt else []
                 for _ in range(2 if overlap else 1)]
        main = torch.cuda.current_stream(lam.device)
        side = torch.cuda.Stream(device=lam.device) if overlap else main   # default priority
        # The loops below issue two library calls per step; arguments are
        # validated here once (blobs from save() of this simulation, lambda
        # arrays by the checks of Adjoint.step_blob), so the calls go straight
        # to the C ABI and the host keeps ahead of the GPU.
        check_lambda(lam, sim.ny, sim.nx, adj.workspace.device)
        check_lambda(spare, sim.ny, sim.nx, adj.workspace.device)
        nbytes = sim.state_bytes()
        for b in [c for c in self.ckpt if c is not None] + [b for pl in pools for b in pl]:
            if not (b.dtype == torch.uint8 and b.numel() == nbytes and b.device == adj.workspace.device):
                raise ValueError("checkpoint blobs must come from Simulation.save() of this simulation")
        L, fi, sh, ah = lib(), form_index(self.form), sim._h, adj._h
        s_main, s_side = _stream(main), _stream(side)
        ready = [None] * nseg    # segment s recomputed (recorded on `side`)
        freed = [None, None]     # pool k no longer read by the adjoint (recorded on `main`)
        if overlap:
            side.wait_stream(main)   # the forward pass and the zeroed pools are complete

        def recompute(s, k):
            t_lo, t_hi = s * every, min(self.T, (s + 1) * every)
            states = [self.ckpt[s]] + pools[k][:t_hi - t_lo - 1]
            if overlap:
                if freed[k] is not None:
                    side.wait_event(freed[k])
                self.ckpt[s].record_stream(side)
            for j in range(1, t_hi - t_lo):
                check(L.lbm_step_blobs(sh, _ptr(states[j - 1]), _ptr(states[j]), fi, s_side))
            if overlap:
                ready[s] = torch.cuda.Event()
                ready[s].record(side)
            return states

        segs = list(reversed(range(nseg)))
        states_next = recompute(segs[0], 0) if (segs and overlap) else None
        for i, s in enumerate(segs):
            k = i % len(pools)
            if overlap:
                states = states_next
                if i + 1 < len(segs):   # the next segment's recompute goes ahead of this segment's adjoint
                    states_next = recompute(segs[i + 1], (i + 1) % len(pools))
            else:
                states = recompute(s, 0)
            if overlap:
                main.wait_event(ready[s])
            t_lo, t_hi = s * every, min(self.T, (s + 1) * every)
            for t in reversed(range(t_lo, t_hi)):
                check(L.lbm_adjoint_step_blob(ah, _ptr(states[t - t_lo]), fi, _ptr(lam), _ptr(spare), s_main))
                lam, spare = spare, lam
            if overlap:
                freed[k] = torch.cuda.Event()
                freed[k].record(main)
            self.ckpt[s] = None   # this checkpoint is no longer needed
        if overlap:
            main.wait_stream(side)
        del pools
        self.ckpt = []
        dphi0 = adj.init(lam, self.phi0, self.ux0, self.uy0)
        dsig, dM = adj.param_grads()
        return dphi0, dsig, dM


def adjoint_gradients(params, form, T, phi0, target, ux0=None, uy0=None, every=None, timings=None, overlap=True):
    """dL/dphi0, dL/dsigma, dL/dM of L = 1/2 sum (phi_T - target)^2.

    Forward T steps keeping a state checkpoint every `every` steps (default
    ceil(sqrt(T))), then the adjoint backwards: each segment is recomputed
    from its checkpoint (one state per step, held for that segment only) and
    the adjoint steps run over it in reverse.  Memory: (T/every + every)
    states (twice `every` with `overlap`, which recomputes the next segment on
    a second stream during the adjoint of the current one).  `timings`, if a
    dict, receives the forward and backward wall times (seconds,
    synchronised).  Returns (loss, dphi0 [float64], dsigma, dM)."""
    sync = timings is not None
    if sync:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
    run = _Checkpointed(params, form, T, phi0, target, ux0, uy0, every)
    loss = run.forward()
    nckpt = len(run.ckpt)
    if sync:
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    dphi0, dsig, dM = run.backward(overlap=overlap)
    if sync:
        torch.cuda.synchronize()
        timings["forward_s"] = t1 - t0
        timings["backward_s"] = time.perf_counter() - t1
        timings["checkpoints"] = nckpt
        timings["every"] = run.every
    return loss, dphi0, dsig, dM


class _Rollout(torch.autograd.Function):
    """forward: the checkpointed forward pass only (L); backward: the adjoint
    pass."""

    @staticmethod
    def forward(ctx, phi0, sigma, M, params, form, T, target, ux0, uy0, every):
        p = dict(params)
        p["sigma"] = float(sigma)
        p["M"] = float(M)
        run = _Checkpointed(p, form, T, phi0.detach().float(), target, ux0, uy0, every)
        loss = run.forward(keep_checkpoints=True)
        ctx.run = run
        return torch.tensor(loss, dtype=torch.float64, device=phi0.device)

    @staticmethod
    def backward(ctx, g):
        run = ctx.run
        if run is None:
            raise RuntimeError("rollout: backward through a forward that kept no checkpoints")
        dphi0, dsig, dM = run.backward()
        ctx.run = None
        g = g.to(torch.float64)
        dsig_t = torch.tensor(dsig, dtype=torch.float64, device=g.device)
        dM_t = torch.tensor(dM, dtype=torch.float64, device=g.device)
        return ((g * dphi0).to(torch.float32), (g * dsig_t).reshape(()), (g * dM_t).reshape(()),
                None, None, None, None, None, None, None)


def rollout(phi0, sigma, M, params, form, T, target, ux0=None, uy0=None, every=None):
    """L = 1/2 sum (phi_T - phi*)^2 after T steps from phi0 with surface
    tension sigma and mobility M (other parameters from `params`), as a
    differentiable scalar: gradients w.r.t. phi0, sigma and M come from the
    hand-written adjoint with checkpoints every ceil(sqrt(T)) steps.  The
    forward call runs the checkpointed forward pass only (none is kept when
    no input needs a gradient, e.g. under torch.no_grad); the adjoint pass
    runs in backward()."""
    if every is None:
        every = max(1, int(math.ceil(math.sqrt(T))))
    sig = sigma if torch.is_tensor(sigma) else torch.tensor(float(sigma), dtype=torch.float64)
    m = M if torch.is_tensor(M) else torch.tensor(float(M), dtype=torch.float64)
    pd = params if isinstance(params, dict) else {k: getattr(params, k) for k in params.__dataclass_fields__}
    if not (torch.is_grad_enabled() and any(torch.is_tensor(t) and t.requires_grad for t in (phi0, sig, m))):
        # nothing to differentiate: one plain forward pass, no checkpoints
        p = dict(pd)
        p["sigma"] = float(sig)
        p["M"] = float(m)
        run = _Checkpointed(p, form, int(T), phi0.detach().float(), target, ux0, uy0, int(every))
        return torch.tensor(run.forward(keep_checkpoints=False), dtype=torch.float64, device=phi0.device)
    return _Rollout.apply(phi0, sig, m, pd, form, int(T), target, ux0, uy0, int(every))
