"""GPU adjoint (lbm_adjoint_*) against the oracle's adjoint (torch autograd
through the FP64 oracle, itself pinned by finite differences and complex
step in test_oracle_adjoint.py)."""
import math

import numpy as np
import pytest
import torch

import workloads as WL
from oracle import lbm_ref as R

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def oracle_params(p):
    d = p.as_dict()
    d["rho0"] = None
    return R.Params(**d)


def t64(a):
    return None if a is None else torch.tensor(np.asarray(a, np.float32), dtype=torch.float64)


CASES = {
    "shear_walls": lambda: WL.config_shear(nx=32, ny=16, R=4.0, Re=1.0, Ca=0.2),
    "periodic_drop": lambda: (WL.ParamSet(nx=24, ny=20, rho1=5.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=0.01, W=3.0,
                                          M=0.05, tau_h=0.9), WL.droplet(24, 20, 5.0, 3.0, 10.3, 9.2), None, None),
    "box_gravity": lambda: (WL.ParamSet(nx=20, ny=24, wall_x=1, wall_y=1, rho1=3.0, rho2=1.0, nu1=0.1, nu2=0.1,
                                        sigma=0.01, W=3.0, M=0.05, tau_h=0.9, gx=2e-5, gy=-3e-5),
                            WL.droplet(20, 24, 5.0, 3.0, 9.6, 12.3), None, None),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("form", ["stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2"])
def test_one_adjoint_step_matches_oracle_vjp(case, form):
    check_one_adjoint_step(*CASES[case](), case, form)


def test_full_size_adjoint_step_matches_oracle_vjp():
    """One adjoint step on the benchmark's sheared drop (512 x 256, walls at
    +-U, STF-2), the size and form the benchmark's adjoint leg runs."""
    check_one_adjoint_step(*WL.config_shear(), "shear_512x256", "stf2")


def check_one_adjoint_step(p, phi0, ux0, uy0, case, form):
    import paper_2012_14729_amd as P
    k = 4
    op = oracle_params(p)
    sig = torch.tensor(op.sigma, requires_grad=True)
    M = torch.tensor(op.M, requires_grad=True)
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

    # dL/dsigma and dL/dM are sums of signed per-node terms that can nearly
    # cancel (PF-2 on the sheared drop).  The GPU evaluates them at its own
    # FP32-stored state, ~1e-7 away from the oracle's (storage rounding), so
    # each summed term may move by ~1e-7 of itself: the bound adds 1e-7 of the
    # size of the summed terms, sum_j |d out_j / d theta| |lambda_j|, with the
    # derivative vector from a central difference of the oracle step.
    def term_scale(name):
        v = float(getattr(op, name))
        d = 1e-6 * v
        outs = []
        with torch.no_grad():
            for s in (1, -1):
                qq = R.Params(**{**op.__dict__, name: v + s * d})
                nn = R.step(dict(f=st["f"], h=st["h"], J=st["J"], rho0=st["rho0"], t=k), form, qq)
                outs.append(torch.cat([nn["f"], nn["h"], nn["J"]]))
        return float(((outs[0] - outs[1]).abs() / (2 * d) * lam1.abs()).sum())

    scale_s, scale_m = term_scale("sigma"), term_scale("M")

    sim = P.Simulation(p.as_dict(), np.asarray(phi0, np.float32), ux0, uy0)
    sim.step(k, form)
    adj = P.Adjoint(sim)
    lam = adj.step(lam1.to("cuda"), form)
    got = lam.cpu().numpy()
    ds, dm = adj.param_grads()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"[adjoint-step] {case} {form}: rel err {err:.2e} dsig {ds:.6e}/{float(gs):.6e} dM {dm:.6e}/{float(gm):.6e} "
          f"term scales {scale_s:.3e} {scale_m:.3e}",
          flush=True)
    assert err < 1e-5
    assert abs(ds - float(gs)) <= 1e-5 * abs(float(gs)) + 1e-7 * scale_s
    assert abs(dm - float(gm)) <= 1e-5 * abs(float(gm)) + 1e-7 * scale_m


@pytest.mark.parametrize("form", ["stf2", "cpf2", "csf1"])
def test_rollout_gradients_match_oracle(form):
    """Shear drop 64x32 (R = 8), 120 steps, target from the forward run at
    1.1 sigma; sqrt(T) checkpoints.  Bound 1e-4: the seed phi_T - phi* is a
    small difference (|r| ~ 1e-3) of fields the GPU stores in FP32, so its
    relative error is ~1e-7 / 1e-3 before the 120 adjoint steps."""
    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = WL.config_shear(nx=64, ny=32, R=8.0, Re=1.0, Ca=0.2)
    T = 120
    op = oracle_params(p)
    phi0_64, ux_64, uy_64 = t64(phi0), t64(ux0), t64(uy0)
    with torch.no_grad():
        q = R.Params(**{**op.__dict__, "sigma": op.sigma * 1.1})
        target = R.run(R.init(q, phi0_64, ux_64, uy_64), form, q, T)["h"].sum(0)
    sig = torch.tensor(op.sigma, requires_grad=True)
    M = torch.tensor(op.M, requires_grad=True)
    ph = phi0_64.clone().requires_grad_(True)
    q = R.Params(**{**op.__dict__, "sigma": sig, "M": M})
    phiT = R.run(R.init(q, ph, ux_64, uy_64), form, q, T)["h"].sum(0)
    Lref = 0.5 * ((phiT - target) ** 2).sum()
    Lref.backward()

    dev = torch.device("cuda")
    phi0_t = torch.tensor(np.asarray(phi0, np.float32), device=dev, requires_grad=True)
    sig_t = torch.tensor(op.sigma, dtype=torch.float64, requires_grad=True)
    M_t = torch.tensor(op.M, dtype=torch.float64, requires_grad=True)
    tgt = target.float().to(dev)
    L = P.rollout(phi0_t, sig_t, M_t, p.as_dict(), form, T, tgt,
                  ux0=torch.tensor(np.asarray(ux0, np.float32), device=dev),
                  uy0=torch.tensor(np.asarray(uy0, np.float32), device=dev))
    L.backward()
    e_s = abs(float(sig_t.grad) - float(sig.grad)) / abs(float(sig.grad))
    e_m = abs(float(M_t.grad) - float(M.grad)) / abs(float(M.grad))
    gp = phi0_t.grad.double().cpu().numpy()
    rp = ph.grad.numpy()
    e_p = np.abs(gp - rp).max() / np.abs(rp).max()
    print(f"[rollout] {form}: L {float(L):.6e}/{float(Lref):.6e} e_sigma {e_s:.2e} e_M {e_m:.2e} e_phi0 {e_p:.2e}",
          flush=True)
    assert abs(float(L) - float(Lref)) <= 1e-4 * float(Lref)
    assert e_s < 1e-4 and e_m < 1e-4 and e_p < 1e-4


def test_gradients_match_fp64_central_differences_shear_64x32():
    """The small version of the shear-drop gradient problem: 64x32, R = 8,
    U = 0.025, sigma = 6.25e-3, STF-2, 400 steps, phi* from the oracle's
    forward run at 1.1 sigma.  GPU adjoint (sqrt(T) checkpoints) against
    FP64 central differences of the oracle loss, h = 1e-6, for sigma, M and
    phi0 at interface nodes."""
    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = WL.config_shear(nx=64, ny=32, R=8.0, Re=1.0, Ca=0.2)
    T, form, h = 400, "stf2", 1e-6
    op = oracle_params(p)
    phi0_64, ux_64, uy_64 = t64(phi0), t64(ux0), t64(uy0)

    def phi_T(sigma=op.sigma, M=op.M, phi_init=phi0_64):
        q = R.Params(**{**op.__dict__, "sigma": sigma, "M": M})
        with torch.no_grad():
            return R.run(R.init(q, phi_init, ux_64, uy_64), form, q, T)["h"].sum(0)

    target = phi_T(sigma=1.1 * op.sigma).float().double()   # the GPU gets the same FP32 target

    def loss(**kw):
        return float(0.5 * ((phi_T(**kw) - target) ** 2).sum())

    L0 = loss()
    fd_sigma = (loss(sigma=op.sigma + h) - loss(sigma=op.sigma - h)) / (2 * h)
    fd_M = (loss(M=op.M + h) - loss(M=op.M - h)) / (2 * h)
    nodes = [(16, 24), (16, 32 + 8), (8, 32)]          # (y, x) on the drop's interface (centre (16, 32), R = 8)
    fd_phi = []
    for (y, x) in nodes:
        e = torch.zeros_like(phi0_64)
        e[y, x] = h
        fd_phi.append((loss(phi_init=phi0_64 + e) - loss(phi_init=phi0_64 - e)) / (2 * h))

    dev = torch.device("cuda")
    L, dphi0, ds, dm = P.adjoint_gradients(
        p.as_dict(), form, T, torch.tensor(np.asarray(phi0, np.float32), device=dev), target.float().to(dev),
        torch.tensor(np.asarray(ux0, np.float32), device=dev), torch.tensor(np.asarray(uy0, np.float32), device=dev))
    gp = [float(dphi0[y, x]) for (y, x) in nodes]
    e_s, e_m = abs(ds - fd_sigma) / abs(fd_sigma), abs(dm - fd_M) / abs(fd_M)
    e_p = max(abs(a - b) for a, b in zip(gp, fd_phi)) / max(abs(b) for b in fd_phi)
    print(f"[fd-check] L {L:.6e}/{L0:.6e}  dsigma {ds:.6e}/{fd_sigma:.6e} ({e_s:.1e})  dM {dm:.6e}/{fd_M:.6e} "
          f"({e_m:.1e})  dphi0 {gp} / {fd_phi} ({e_p:.1e})", flush=True)
    # FD truncation ~(h/sigma)^2 ~ 3e-8 and round-off ~1e-16 L/h are far
    # below these bounds; what remains is the FP32 storage of the forward
    # state the GPU linearises about (L agrees to ~1e-6).
    assert abs(L - L0) <= 1e-4 * L0
    assert e_s < 1e-5 and e_m < 1e-5
    assert e_p < 5e-5


def test_step_blob_equals_restore_then_step():
    """lbm_adjoint_step_blob about a saved state gives the same lambda, bit for
    bit, as restoring that state and calling lbm_adjoint_step."""
    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = WL.config_shear(nx=80, ny=40, R=8.0, Re=1.0, Ca=0.2)
    sim = P.Simulation(p.as_dict(), np.asarray(phi0, np.float32), ux0, uy0)
    sim.step(5, "csf1")
    blob = sim.save()
    sim.step(3, "csf1")          # move the simulation away from the saved state
    adj = P.Adjoint(sim)
    g = torch.Generator().manual_seed(3)
    lam0 = torch.randn((20, p.ny, p.nx), generator=g, dtype=torch.float64).to("cuda")
    a = adj.step_blob(blob, lam0.clone(), "csf1")
    ga = adj.param_grads()
    adj.reset()
    sim.restore(blob)
    b = adj.step(lam0.clone(), "csf1")
    gb = adj.param_grads()
    assert torch.equal(a, b)
    assert ga == gb


def test_adjoint_refuses_free_slip_walls():
    """The adjoint's extension maps cover periodic and no-slip walls only."""
    import paper_2012_14729_amd as P
    from paper_2012_14729_amd._lib import LbmError
    p = WL.ParamSet(nx=32, ny=16, wall_x=2, rho1=1.0, rho2=1.0, sigma=0.01, W=4.0)
    sim = P.Simulation(p.as_dict(), np.zeros((16, 32), np.float32))
    with pytest.raises(LbmError) as e:
        P.Adjoint(sim)
    assert "free-slip" in str(e.value) or "no-slip" in str(e.value)


def test_rollout_forward_is_one_forward_and_backward_runs_the_adjoint():
    """rollout() under torch.no_grad costs about one plain forward run (no
    checkpoints, no adjoint); with gradients, forward keeps only the
    checkpoints and backward() runs the adjoint.  L and the gradients equal
    those of adjoint_gradients() bit for bit."""
    import time

    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = WL.config_shear(nx=128, ny=64, R=16.0, Re=1.0, Ca=0.2)
    T, form = 400, "stf2"
    dev = torch.device("cuda")
    f32 = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)   # noqa: E731
    phi0_t, ux, uy = f32(phi0), f32(ux0), f32(uy0)
    s = P.Simulation(dict(p.as_dict(), sigma=1.1 * p.sigma), phi0_t, ux, uy, device=dev)
    s.step(T, form)
    target = s.moments(form)["phi"]
    del s
    loss_ref, dphi_ref, ds_ref, dm_ref = P.adjoint_gradients(p.as_dict(), form, T, phi0_t, target, ux, uy)

    def plain():
        sim = P.Simulation(p.as_dict(), phi0_t, ux, uy, device=dev)
        sim.step(T, form)
        return sim.moments(form)["phi"]

    def nograd():
        with torch.no_grad():
            return P.rollout(phi0_t, p.sigma, p.M, p.as_dict(), form, T, target, ux, uy)

    plain(), nograd()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    L0 = nograd()
    torch.cuda.synchronize()
    t_nograd = time.perf_counter() - t0
    print(f"[rollout split] plain forward {t_plain * 1e3:.1f} ms, L under no_grad {t_nograd * 1e3:.1f} ms", flush=True)
    assert float(L0) == loss_ref
    assert t_nograd < 2.0 * t_plain + 0.02

    ph = phi0_t.clone().requires_grad_(True)
    sg = torch.tensor(p.sigma, dtype=torch.float64, requires_grad=True)
    mm = torch.tensor(p.M, dtype=torch.float64, requires_grad=True)
    L = P.rollout(ph, sg, mm, p.as_dict(), form, T, target, ux, uy)
    assert float(L) == loss_ref
    assert ph.grad is None
    L.backward()
    assert float(sg.grad) == ds_ref and float(mm.grad) == dm_ref
    assert torch.equal(ph.grad, dphi_ref.to(torch.float32))


@pytest.mark.parametrize("T,every", [(150, None), (37, 8), (9, 4)])
def test_overlapped_backward_equals_serial(T, every):
    """The backward pass that recomputes the next segment on a second stream
    while the adjoint runs over the current one gives the serial order's
    gradients bit for bit (same kernels, same inputs; two state pools)."""
    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = WL.config_shear(nx=96, ny=48, R=12.0, Re=1.0, Ca=0.2)
    form = "cpf2"
    dev = torch.device("cuda")
    f32 = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)   # noqa: E731
    phi0_t, ux, uy = f32(phi0), f32(ux0), f32(uy0)
    s = P.Simulation(dict(p.as_dict(), sigma=1.2 * p.sigma), phi0_t, ux, uy, device=dev)
    s.step(T, form)
    target = s.moments(form)["phi"]
    del s
    out = []
    for overlap in (False, True):
        run = P._Checkpointed(p.as_dict(), form, T, phi0_t, target, ux, uy, every)
        loss = run.forward()
        out.append((loss, *run.backward(overlap=overlap)))
    torch.cuda.synchronize()
    (l0, d0, s0, m0), (l1, d1, s1, m1) = out
    print(f"[overlap] T={T} every={every}: L {l0:.6e}, dL/dsigma {s0:.6e} / {s1:.6e}", flush=True)
    assert l0 == l1 and s0 == s1 and m0 == m1
    assert torch.equal(d0, d1)
