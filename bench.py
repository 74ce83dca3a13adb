"""Benchmark of the phase-field LBM hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload: the stationary droplet on a 2048x2048 periodic lattice (R = 256,
W = 5, density ratio 1000, dynamic viscosity ratio 100, sigma = 1e-3), one
run per interfacial-force form; a "step" is one time step (fused
collide-stream kernel + order-parameter kernel) of one of the eight
simulations.  The timed K steps (any K >= 1) are consecutive runs, one per
form in the paper's order, of K // 8 steps each plus one more step for each
of the first K % 8 forms; a form with no step is skipped.  All state is
resident in HBM before the timed region.

Prints one JSON line with MLUPS, the roofline of the fused kernel (HIP
events recorded on the launch stream during the timed region), the oracle
timed on the host cores (all of this process's cores and one core),
per-form MLUPS, the spurious-current maximum after 10000 steps per form and
the batched/adjoint figures.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per node of the collide-stream step (FP32): read and write
# the 9 f and 9 h populations (144 B), read and write the (phi u) history
# (16 B), read phi (4 B) = 164 B.
BYTES_FUSED_ALG = 9 * 4 * 2 + 9 * 4 * 2 + 2 * 4 * 2 + 4
# What this design's fused kernel moves per node (FP32 populations, FP64
# phi): read 9 f + 8 h (pulled; d0 is read by the order-parameter kernel) +
# 2 J + phi (8 B); write 9 f + 8 h + d0 + 2 J.  The same 164 B.
BYTES_FUSED = 9 * 4 + 8 * 4 + 2 * 4 + 8 + 9 * 4 + 9 * 4 + 2 * 4
#   order-parameter kernel: read d0 + 8 h (pulled) + phi (8 B); write phi (8 B)
BYTES_PHI = 4 + 8 * 4 + 8 + 8
FORMS = ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2")
TIMING_PERIOD = 8   # kernel durations: HIP events on one step in eight of the timed region
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_droplet2048.json")
# sources of the fused step kernel: the launchers, the tile body and the shared declarations
KERNEL_SRC = [os.path.join(ROOT, "paper_2012_14729_amd", "csrc", f)
              for f in ("lbm_kernels.hip", "lbm_tile.hpp", "lbm_internal.hpp")]


def kernel_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per fused launch from the committed rocprofv3 counter runs,
    or None when missing or taken on a different kernel source."""
    try:
        d = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha") != kernel_sha():
        return None
    return d.get("bytes_per_launch")


def _host_cpu():
    """CPU model and logical-CPU count of the host, read from /proc/cpuinfo."""
    model, n = None, 0
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("processor"):
                n += 1
            elif model is None and line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return model, n


def cpu_baseline(budget_all_s=15.0, budget_one_s=12.0):
    """The oracle (FP64, torch CPU) on the same 2048x2048 droplet, timed
    twice: with every core this process may use (torch intra-op threads =
    its CPU affinity, capped by OMP_NUM_THREADS when set), then on one core.
    Each leg steps (forms round-robin) until about its budget has passed."""
    import numpy as np
    import torch

    import workloads as WL
    from oracle import lbm_ref as R

    p, phi0, _, _ = WL.config_droplet_large(2048)
    op = R.Params(**{k: (None if k == "rho0" else v) for k, v in p.as_dict().items()})
    cells = p.nx * p.ny
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(avail, int(omp)) if omp.isdigit() and int(omp) > 0 else avail
    prev = torch.get_num_threads()

    def leg(nthreads, budget, st):
        torch.set_num_threads(nthreads)
        n, t0 = 0, time.perf_counter()
        while True:
            st = R.step(st, FORMS[n % 8], op)
            n += 1
            el = time.perf_counter() - t0
            if el > budget or n >= 64:
                return st, n, el

    try:
        torch.set_num_threads(threads)
        st = R.init(op, torch.tensor(np.asarray(phi0, np.float32), dtype=torch.float64))
        st = R.step(st, "stf1", op)   # warm-up
        st, n_all, el_all = leg(threads, budget_all_s, st)
        st, n_one, el_one = leg(1, budget_one_s, st)
    finally:
        torch.set_num_threads(prev)
    model, logical = _host_cpu()
    small = oracle_droplet64(threads)
    all_rate = cells * n_all / el_all / 1e6
    one_rate = cells * n_one / el_one / 1e6
    return {"value": round(all_rate, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n_all} time steps of the 2048x2048 droplet (forms round-robin, FP64 torch CPU, "
                      f"{threads} threads) after 1 warm-up step, {el_all:.1f} s",
            "one_core": {"value": round(one_rate, 3), "unit": "MLUPS", "cores": 1,
                         "sample": f"{n_one} further time steps on 1 thread, {el_one:.1f} s"},
            "host": {"cpu_model": model, "logical_cpus_on_host": logical, "cpus_available_to_process": avail},
            "oracle_droplet64": small}


def oracle_droplet64(threads, steps=1000):
    """The 64x64 stationary droplet (R = 16, W = 4, density ratio 10, sigma =
    0.01, tau_f = tau_h = 0.8, CPF-2) run by the oracle alone for 1000 steps,
    timed on `threads` cores, with its Laplace-law check (sigma from R_num
    (p_in - p_out), Sec. V.A) and the drift of sum(phi).  The pressure still
    rings acoustically at 1000 steps (period about 75 steps, +-40 %), so sigma
    is the mean of ten samples 25 steps apart over the last 250 steps."""
    import numpy as np
    import torch

    import workloads as WL
    from oracle import lbm_ref as R

    p, phi0, _, _ = WL.config_droplet64()
    op = R.Params(**{k: (None if k == "rho0" else v) for k, v in p.as_dict().items()})
    prev = torch.get_num_threads()
    try:
        torch.set_num_threads(threads)
        st = R.init(op, torch.tensor(np.asarray(phi0, np.float32), dtype=torch.float64))
        s0 = float(R.moments(st, "cpf2", op)["phi"].sum())
        t0 = time.perf_counter()
        st = R.run(st, "cpf2", op, steps - 250)
        samples = []
        for _ in range(10):
            st = R.run(st, "cpf2", op, 25)
            samples.append(R.laplace_sigma(R.moments(st, "cpf2", op), op))
        el = time.perf_counter() - t0
    finally:
        torch.set_num_threads(prev)
    m = R.moments(st, "cpf2", op)
    sig = sum(v[0] for v in samples) / len(samples)
    rn = samples[-1][1]
    return {"workload": "64x64 droplet, R=16, W=4, density ratio 10, sigma=0.01, tau_f=tau_h=0.8, CPF-2, FP64",
            "steps": steps, "seconds": round(el, 2), "cores": threads,
            "note": "seconds include the ten Laplace samples (moments) of the last 250 steps",
            "MLUPS": round(64 * 64 * steps / el / 1e6, 3),
            "laplace_sigma_num": round(sig, 6), "laplace_rel_error": round(abs(sig - op.sigma) / op.sigma, 4),
            "R_num": round(rn, 3), "phi_sum_drift": float(m["phi"].sum()) - s0}


def bench_batched(steps, loop_steps):
    """512 independent two-droplet instances (sides 32..512, random force form,
    density ratio and sigma; numpy default_rng(14729)), one persistent
    graph-replayed batched step vs looping the single-lattice lbm_step."""
    import numpy as np
    import torch

    import paper_2012_14729_amd as P
    import workloads as WL

    insts = WL.batch_instances(512, seed=14729)
    params = [p.as_dict() for p, _, _ in insts]
    forms = [f for _, f, _ in insts]
    phis = [np.asarray(x, np.float32) for _, _, x in insts]
    cells = sum(p["nx"] * p["ny"] for p in params)
    print(f"[bench] batched: 512 instances, {cells} nodes", file=sys.stderr, flush=True)
    tc = time.perf_counter()
    b = P.Batch(params, forms, phis)   # includes timing the candidate launch shapes
    create_s = time.perf_counter() - tc
    shape = b.config
    classes = {}   # tile shapes chosen per instance-size class
    for p_, ts in zip(params, b.tile_shapes()):
        cls = "small (side <= 128)" if p_["nx"] <= 128 else ("medium (<= 320)" if p_["nx"] <= 320 else "large")
        key = f"{ts[0]}x{ts[1]}"
        classes.setdefault(cls, {}).setdefault(key, 0)
        classes[cls][key] += 1
    b.step(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    flags = list(b.status())
    unstable = [{"instance": k, "side": params[k]["nx"], "form": FORMS[forms[k]],
                 "rho_ratio": params[k]["rho1"] / params[k]["rho2"], "sigma": float(f"{params[k]['sigma']:.4g}")}
                for k, fl in enumerate(flags) if fl]
    del b
    torch.cuda.empty_cache()
    sims = [P.Simulation(pp, x) for pp, x in zip(params, phis)]
    for s, f in zip(sims, forms):
        s.step(2, f)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(loop_steps):
        for s, f in zip(sims, forms):
            s.step(1, f)
    torch.cuda.synchronize()
    el_loop = time.perf_counter() - t1
    del sims
    torch.cuda.empty_cache()
    batched = cells * steps / el / 1e6
    loop = cells * loop_steps / el_loop / 1e6
    return {"MLUPS": round(batched, 1), "instances": 512, "nodes": cells, "steps": steps,
            "looping_plain_lbm_step_MLUPS": round(loop, 1), "loop_steps": loop_steps,
            "speedup_vs_loop": round(batched / loop, 2), "unstable_instances": len(unstable),
            "unstable": unstable,
            "launch_shape": {"one_kernel_per_form": bool(shape["split"]), "addressing": ("general", "interior + general", "wrapped")[shape["fast"]],
                             "workgroups_per_cu": shape["blocks_per_cu"] or "one per tile",
                             "tuned_ms_per_step": round(shape["ms_per_step"], 4),
                             "tile_shapes_per_size_class": classes},
            "create_s_incl_tuning": round(create_s, 2)}


def bench_adjoint(T):
    """Gradient of L = 1/2 sum (phi_T - phi*)^2 w.r.t. phi0, sigma and M for
    the drop in simple shear (512x256, walls at +-U, R = 64, Re = 1,
    Ca = 0.2, STF-2), phi* from the forward run at 1.1 sigma, T steps with
    checkpoints every ceil(sqrt(T)) steps.  Reported against the plain step
    on the same configuration."""
    import numpy as np
    import torch

    import paper_2012_14729_amd as P
    import workloads as WL

    dev = torch.device("cuda:0")
    p, phi0, ux0, uy0 = WL.config_shear()
    pd = p.as_dict()
    cells = p.nx * p.ny
    phi0 = torch.tensor(np.asarray(phi0, np.float32), device=dev)
    ux = torch.tensor(np.asarray(ux0, np.float32), device=dev)
    uy = torch.tensor(np.asarray(uy0, np.float32), device=dev)
    print(f"[bench] adjoint: shear {p.nx}x{p.ny}, T={T}", file=sys.stderr, flush=True)
    tgt_p = dict(pd, sigma=1.1 * pd["sigma"])
    s = P.Simulation(tgt_p, phi0, ux, uy, device=dev)
    s.step(T, "stf2")
    target = s.moments("stf2")["phi"]
    del s
    s = P.Simulation(pd, phi0, ux, uy, device=dev)
    s.step(50, "stf2")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(T, "stf2")
    torch.cuda.synchronize()
    plain = cells * T / (time.perf_counter() - t0) / 1e6
    del s
    P.adjoint_gradients(pd, "stf2", 16, phi0, target, ux, uy)   # warm-up
    tm, tms = {}, {}
    P.adjoint_gradients(pd, "stf2", T, phi0, target, ux, uy, timings=tms, overlap=False)
    loss, dphi0, dsig, dM = P.adjoint_gradients(pd, "stf2", T, phi0, target, ux, uy, timings=tm)
    bwd_serial = cells * T / tms["backward_s"] / 1e6
    fwd = cells * T / tm["forward_s"] / 1e6
    bwd = cells * T / tm["backward_s"] / 1e6
    tot = cells * T / (tm["forward_s"] + tm["backward_s"]) / 1e6
    print(f"[bench] adjoint: forward {tm['forward_s']:.3f} s, backward {tm['backward_s']:.3f} s", file=sys.stderr,
          flush=True)
    return {"workload": f"drop in shear {p.nx}x{p.ny}, walls +-U, R=64, Re=1, Ca=0.2, STF-2, T={T}, "
                        f"checkpoints every {tm['every']} steps",
            "plain_step_MLUPS": round(plain, 1),
            "forward_with_checkpoints_MLUPS": round(fwd, 1),
            "backward_MLUPS": round(bwd, 1), "gradient_MLUPS": round(tot, 1),
            "backward_vs_plain_step": round(bwd / plain, 3), "gradient_vs_plain_step": round(tot / plain, 3),
            "backward_serial_MLUPS": round(bwd_serial, 1),
            "backward_note": "adjoint steps (FP64) plus the recompute of each segment from its checkpoint, "
                             "the next segment's recompute on a second stream during the current adjoint "
                             "(serial: one stream)",
            "loss": loss, "dL_dsigma": dsig, "dL_dM": dM, "max_abs_dL_dphi0": float(dphi0.abs().max())}


def split_steps(steps, nforms=len(FORMS)):
    """Steps per force form: steps // nforms each, one more for each of the
    first steps % nforms forms."""
    base, extra = divmod(steps, nforms)
    return [base + (1 if k < extra else 0) for k in range(nforms)]


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1600)
    ap.add_argument("--warmup", type=int, default=80)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--spurious-steps", type=int, default=10000,
                    help="steps per form of the spurious-current leg (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--check-args", action="store_true", help="validate the arguments and exit (no GPU work)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported: the multi-GPU slab "
              f"decomposition is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be a positive number of time steps", file=sys.stderr)
        sys.exit(2)
    if args.warmup < 0 or args.spurious_steps < 0 or args.batch_steps < 1 or args.adjoint_steps < 1:
        print("bench.py: --warmup and --spurious-steps must be >= 0, --batch-steps and --adjoint-steps >= 1",
              file=sys.stderr)
        sys.exit(2)
    return args


def spurious_leg(sims, nsteps, cells):
    """Config-2 horizon: every form's droplet advanced to nsteps steps in
    total; max|u| (the spurious current) then, and the rate of this leg."""
    import torch

    umax, done = {}, {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ran = 0
    for f, s in sims.items():
        todo = nsteps - s.step_count
        if todo > 0:
            s.step(todo, f)
            ran += todo
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for f, s in sims.items():
        m = s.moments(f)
        umax[f] = float(f"{float(torch.sqrt(m['ux'] ** 2 + m['uy'] ** 2).max()):.4g}")
        done[f] = s.step_count
    return {"steps_per_form": done, "max_abs_u": umax, "diverged": [f for f, s in sims.items() if s.status()],
            "MLUPS": round(cells * ran / el / 1e6, 1) if ran else None}


def main():
    args = parse_args()
    counts = split_steps(args.steps)
    if args.check_args:
        print(json.dumps({"steps_per_form": dict(zip(FORMS, counts))}))
        return

    import numpy as np
    import torch

    import paper_2012_14729_amd as P
    import workloads as WL

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p, phi0, _, _ = WL.config_droplet_large(args.size)
    phi0 = np.asarray(phi0, np.float32)
    print(f"[bench] building {len(FORMS)} simulations {p.nx}x{p.ny}", file=sys.stderr, flush=True)
    sims = {f: P.Simulation(p.as_dict(), phi0, device=dev) for f in FORMS}
    cells = p.nx * p.ny

    wcounts = split_steps(args.warmup)
    for (f, s), w in zip(sims.items(), wcounts):
        s.step(max(1, w), f)
    torch.cuda.synchronize()
    print("[bench] warm-up done", file=sys.stderr, flush=True)

    # The launch durations are sampled on one step in `period` of each run:
    # timing every launch costs the timed region about 5 %.  A run's first
    # step is slower than the rest (the previous run's state, not this one's,
    # sits in the caches), so the sample is stratified: run j starts sampling
    # at its step j mod period, and every step index mod period is sampled
    # equally often over the runs, the first steps at their own frequency.
    timed = [(f, sims[f], n) for f, n in zip(FORMS, counts) if n > 0]
    period = min([TIMING_PERIOD] + [n for _, _, n in timed])
    for _, s, _ in timed:   # create the event rings outside the timed region
        s.set_timing(True, period=period)
        s.set_timing(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, (f, s, n) in enumerate(timed):
        lead = j % period
        for i in range(n):
            if i == lead:
                s.set_timing(True, period=period)   # no events pending: no synchronisation
            s.step(1, f)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    fused_ms = sum(s.kernel_time(0)[0] for _, s, _ in timed)
    fused_n = sum(s.kernel_time(0)[1] for _, s, _ in timed)
    phi_ms = sum(s.kernel_time(1)[0] for _, s, _ in timed)
    phi_n = sum(s.kernel_time(1)[1] for _, s, _ in timed)
    for _, s, _ in timed:
        s.set_timing(False)
    print(f"[bench] timed {args.steps} steps in {el:.4f} s", file=sys.stderr, flush=True)
    if fused_n == 0 or phi_n == 0:
        raise RuntimeError("no kernel launch was timed")
    diverged = [f for f, s, _ in timed if s.status()]

    # per-form rates, each form alone
    per_form = {}
    nper = max(8, args.steps // 16)
    for f, s in sims.items():
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.step(nper, f)
        torch.cuda.synchronize()
        per_form[f] = round(cells * nper / (time.perf_counter() - t1) / 1e6, 1)

    fused_avg_s = fused_ms / fused_n / 1e3
    phi_avg_s = phi_ms / phi_n / 1e3
    achieved = BYTES_FUSED_ALG * cells / fused_avg_s / 1e9
    achieved_design = BYTES_FUSED * cells / fused_avg_s / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_fused (collide-stream, all forms)", "bytes_per_node": BYTES_FUSED_ALG,
                "bytes_basis": "algorithmic: f and h read+write, (phi u) read+write, phi read (FP32)",
                "nodes_per_launch": cells, "avg_launch_us": round(fused_avg_s * 1e6, 2),
                "timed_launches": fused_n,
                "design_basis": {"bytes_per_node": BYTES_FUSED, "achieved": round(achieved_design, 1),
                                 "frac": round(achieved_design / HBM_PEAK_GBS, 4),
                                 "note": "8 pulled h (d0 goes to the order-parameter kernel) and phi in FP64: the same total"},
                "phi_kernel": {"avg_launch_us": round(phi_avg_s * 1e6, 2),
                               "achieved_GBs": round(BYTES_PHI * cells / phi_avg_s / 1e9, 1),
                               "bytes_per_node": BYTES_PHI}}

    value = cells * args.steps / el / 1e6
    out = {
        "metric": "MLUPS & HBM GB/s (% peak) FP32 1 GPU; batched/adjoint vs plain step",
        "value": round(value, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"stationary droplet {p.nx}x{p.ny} periodic, R={p.nx // 8}, W=5, rho1/rho2=1000, "
                               f"mu1/mu2=100, sigma=1e-3, one run per force form in the paper's order",
                   "steps_per_form": dict(zip(FORMS, counts)),
                   "precision": "FP64 arithmetic (collision, stencils, forces) and FP64 phi; "
                                "FP32 storage of f, h and (phi u)",
                   "storage_dtype": "fp32",
                   "step_bytes_per_node": BYTES_FUSED + BYTES_PHI,
                   "step_GBs": round((BYTES_FUSED + BYTES_PHI) * value * 1e6 / 1e9, 1)},
        "roofline": roofline,
        "per_form_MLUPS": per_form,
        "diverged": diverged,
        "spurious_current": None,
        "batched": None,
        "adjoint": None,
    }
    if args.spurious_steps:
        print(f"[bench] spurious-current leg: {args.spurious_steps} steps per form", file=sys.stderr, flush=True)
        out["spurious_current"] = spurious_leg(sims, args.spurious_steps, cells)
    del sims
    torch.cuda.empty_cache()
    if not args.no_batch:
        out["batched"] = bench_batched(args.batch_steps, 20)
        out["batched"]["vs_plain_step"] = round(out["batched"]["MLUPS"] / value, 3)
        if out["spurious_current"]:   # the plain step's long-run rate (10^4 steps per form)
            out["batched"]["vs_plain_step_long_run"] = round(
                out["batched"]["MLUPS"] / out["spurious_current"]["MLUPS"], 3)
    if not args.no_adjoint:
        torch.cuda.empty_cache()
        out["adjoint"] = bench_adjoint(args.adjoint_steps)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
