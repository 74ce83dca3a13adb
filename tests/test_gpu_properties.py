"""GPU checks that hold at any size: conservation, rest state, symmetry,
checkpoint/restore, divergence detection, and one-step parity at the full
benchmark sizes (2048x2048 droplet, 1024x4096 channel)."""
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


def sim_of(p, phi0, ux0=None, uy0=None):
    import paper_2012_14729_amd as P
    return P.Simulation(p.as_dict(), np.asarray(phi0, np.float32), ux0, uy0)


@pytest.mark.parametrize("form", ["stf1", "cpf2", "csf2"])
def test_order_parameter_conserved(form):
    p, phi0, ux0, uy0 = WL.config_shear(nx=128, ny=64, R=16.0)
    s = sim_of(p, phi0, ux0, uy0)
    s0 = float(np.asarray(phi0, np.float32).astype(np.float64).sum())
    s.step(500, form)
    phi = s.moments(form)["phi"].double()
    # phi moments are FP32 copies of the FP64 state: allow their rounding only
    assert abs(float(phi.sum()) - s0) < 1e-7 * phi.numel()


def test_rest_state_stays_at_rest():
    p = WL.ParamSet(nx=64, ny=16, rho1=4.0, rho2=1.0, sigma=0.02)
    s = sim_of(p, np.full((16, 64), 0.3))
    for form in ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2"):
        s.step(5, form)
        m = s.moments(form)
        assert float(m["ux"].abs().max()) == 0.0 and float(m["uy"].abs().max()) == 0.0
        assert float(m["P"].abs().max()) == 0.0


def test_transpose_symmetry():
    """x <-> y swap of the input swaps the output (square periodic grid)."""
    p = WL.ParamSet(nx=64, ny=64, rho1=10.0, rho2=1.0, sigma=0.01, W=4.0)
    phi0 = WL.droplet(64, 64, 12.0, 4.0, xc=27.3, yc=35.9).astype(np.float32)
    a = sim_of(p, phi0)
    b = sim_of(p, phi0.T.copy())
    a.step(50, "stf2")
    b.step(50, "stf2")
    ma, mb = a.moments("stf2"), b.moments("stf2")
    umax = float(torch.sqrt(ma["ux"] ** 2 + ma["uy"] ** 2).max())
    assert float((ma["phi"].T - mb["phi"]).abs().max()) < 1e-6
    assert float((ma["ux"].T - mb["uy"]).abs().max()) < 1e-4 * umax


def test_checkpoint_restore_bitwise():
    p, phi0, ux0, uy0 = WL.config_shear(nx=64, ny=32, R=8.0)
    s = sim_of(p, phi0, ux0, uy0)
    s.step(20, "csf1")
    blob = s.save()
    s.step(30, "csf1")
    a = {k: v.clone() for k, v in s.moments("csf1").items()}
    s.restore(blob)
    s.step(30, "csf1")
    b = s.moments("csf1")
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_divergence_is_reported():
    p = WL.ParamSet(nx=64, ny=16, sigma=0.01)
    phi0 = np.zeros((16, 64), np.float32)
    phi0[3, 7] = np.nan          # non-finite input set on the host
    s = sim_of(p, phi0)
    s.step(3, "cpf2")
    assert s.status() is True
    ok = sim_of(p, np.zeros((16, 64), np.float32))
    ok.step(3, "cpf2")
    assert ok.status() is False


def test_zero_steps_and_timing():
    p, phi0, _, _ = WL.config_droplet64()
    s = sim_of(p, phi0)
    m0 = {k: v.clone() for k, v in s.moments("cpf2").items()}
    s.step(0, "cpf2")
    assert torch.equal(m0["ux"], s.moments("cpf2")["ux"])
    s.set_timing(True)
    s.step(7, "cpf2")
    ms, n = s.kernel_time(0)
    assert n == 7 and ms > 0
    ms1, n1 = s.kernel_time(1)
    assert n1 == 7 and ms1 > 0
    assert s.step_count == 7
    # a period counts from the set_timing call, its first step included
    s.set_timing(True, period=4)
    s.step(5, "cpf2")
    assert s.kernel_time(0)[1] == 2 and s.kernel_time(1)[1] == 2
    s.set_timing(True, period=8)
    s.step(3, "cpf2")
    assert s.kernel_time(0)[1] == 1


def test_kernel_times_fit_inside_the_wall_clock():
    """The timed kernels' events take each kernel's own dispatch start and
    stop: over 24 timed steps of a 1024x1024 droplet the two kernels' summed
    times lie inside the wall-clock time of those steps and cover most of it
    (a broken pair of events would read zero or span the whole queue)."""
    import time
    p, phi0, _, _ = WL.config_droplet_large(1024)
    s = sim_of(p, np.asarray(phi0, np.float32))
    s.step(4, "cpf2")
    torch.cuda.synchronize()
    s.set_timing(True, period=1)
    t0 = time.perf_counter()
    s.step(24, "cpf2")
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    (f_ms, f_n), (p_ms, p_n) = s.kernel_time(0), s.kernel_time(1)
    print(f"[timing] wall {wall_ms:.3f} ms, fused {f_ms:.3f} ms / {f_n}, phi {p_ms:.3f} ms / {p_n}", flush=True)
    assert f_n == 24 and p_n == 24
    assert 0.0 < p_ms < f_ms
    assert 0.5 * wall_ms < f_ms + p_ms <= wall_ms


def test_lattice_past_32_bit_element_offsets():
    """A 16384 x 13312 periodic lattice: a state array (20 FP32 planes) holds
    4.36e9 > 2^32 elements, so the upper rows' offsets need 64 bits.  phi0
    tiles a 1024 x 832 droplet field 16 x 16 times; a periodic lattice is
    translation invariant and every addressing path gives the same bits, so
    after 3 steps each 1024 x 832 block equals the small lattice's fields
    exactly.  Checked: the four corner blocks (the top ones lie past element
    2^32 of the state arrays)."""
    import dataclasses
    bx, by, reps, form = 1024, 832, 16, "cpf2"
    p_small = WL.ParamSet(nx=bx, ny=by, rho1=1000.0, rho2=1.0, nu1=1.0 / 30.0, nu2=1.0 / 3.0, sigma=1e-3, W=5.0,
                          M=0.1, tau_h=0.8)
    phi_s = np.asarray(WL.droplet(bx, by, 128.0, 5.0), np.float32)
    small = sim_of(p_small, phi_s)
    small.step(3, form)
    ms = small.moments(form)
    p_big = dataclasses.replace(p_small, nx=bx * reps, ny=by * reps)
    assert 20 * p_big.nx * p_big.ny > 2 ** 32
    print(f"[big] {p_big.nx}x{p_big.ny}: init", flush=True)
    big = sim_of(p_big, np.tile(phi_s, (reps, reps)))
    big.step(3, form)
    keys = ("phi", "ux", "uy")
    out = {k: torch.empty((p_big.ny, p_big.nx), dtype=torch.float32, device=ms["phi"].device) for k in keys}
    mb = big.moments(form, out=out)
    torch.cuda.synchronize()
    assert not big.status()
    for j in (0, reps - 1):
        for i in (0, reps - 1):
            for k in keys:
                blk = mb[k][j * by:(j + 1) * by, i * bx:(i + 1) * bx]
                assert torch.equal(blk, ms[k]), (j, i, k)
    print(f"[big] corner blocks equal the {bx}x{by} lattice", flush=True)


def _one_step_full_size(p, phi0, form):
    op = R.Params(**{k: (None if k == "rho0" and math.isnan(v) else v) for k, v in p.as_dict().items()})
    phi32 = np.asarray(phi0, np.float32)
    print(f"[full-size] {p.nx}x{p.ny} form={form}: oracle one step", flush=True)
    st = R.step(R.init(op, torch.tensor(phi32, dtype=torch.float64)), form, op)
    ref = {k: v.numpy() for k, v in R.moments(st, form, op).items()}
    s = sim_of(p, phi32)
    s.step(1, form)
    got = {k: v.cpu().numpy().astype(np.float64) for k, v in s.moments(form).items()}
    for k in ("phi", "rho"):
        assert np.abs(got[k] - ref[k]).max() / np.abs(ref[k]).max() < 1e-6, k
    umax = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max()
    eu = max(np.abs(got["ux"] - ref["ux"]).max(), np.abs(got["uy"] - ref["uy"]).max()) / umax
    assert eu < 1e-5, eu


def test_full_size_droplet_one_step():
    """2048x2048 droplet (density ratio 1000), the benchmark launch shape."""
    p, phi0, _, _ = WL.config_droplet_large(2048)
    _one_step_full_size(p, phi0, "stf1")


def test_full_size_channel_one_step():
    """1024x4096 bubble between x-walls with gravity."""
    p, phi0, _, _ = WL.config_bubble()
    _one_step_full_size(p, phi0, "stf2")


@pytest.mark.parametrize("case", ["periodic_stf1", "ywalls_csf2", "xwalls_gravity_pf2", "ragged_strips_csf1",
                                  "small_periodic_cpf2"])
def test_interior_fast_path_bitwise_equals_general_path(case, monkeypatch):
    """Tiles away from the edges take the interior addressing path; with
    PFLBM_GENERAL_PATH=1 every tile takes the general one.  Same arithmetic,
    so the saved states must agree bit for bit.  In the 1000x1000 case the
    last tile column is ragged (1000 = 15 x 64 + 40) and the rows end in
    padding lanes, which must save as zeros in both runs; the 40x24 lattice
    is narrower than a tile, so its tile wraps onto itself."""
    import paper_2012_14729_amd as P
    nx, ny = 320, 96
    if case == "small_periodic_cpf2":
        nx, ny = 40, 24
        p = WL.ParamSet(nx=nx, ny=ny, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=3.0, M=0.1, tau_h=0.8)
        phi0, ux0, uy0, form = WL.droplet(nx, ny, 8.0, 3.0, xc=17.0, yc=11.0), None, None, "cpf2"
    elif case == "ragged_strips_csf1":
        nx = ny = 1000
        p = WL.ParamSet(nx=nx, ny=ny, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=4.0, M=0.1, tau_h=0.8)
        phi0, ux0, uy0, form = WL.two_droplets(nx, ny, 120.0, 90.0, 2.0, 4.0), None, None, "csf1"
    elif case == "periodic_stf1":
        p = WL.ParamSet(nx=nx, ny=ny, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=4.0, M=0.1, tau_h=0.8)
        phi0, ux0, uy0, form = WL.two_droplets(nx, ny, 20.0, 14.0, 2.0, 4.0), None, None, "stf1"
    elif case == "ywalls_csf2":
        p, phi0, ux0, uy0 = WL.config_shear(nx=nx, ny=ny, R=20.0, Re=1.0, Ca=0.2)
        form = "csf2"
    else:
        p = WL.ParamSet(nx=nx, ny=ny, wall_x=1, rho1=1.0, rho2=0.1, nu1=0.1, nu2=0.1, sigma=1e-3, W=4.0, M=0.1,
                        tau_h=0.8, gy=-2e-5)
        phi0, ux0, uy0, form = WL.droplet(nx, ny, 18.0, 4.0, xc=150.0, yc=40.0, inside=-1.0), None, None, "pf2"
    phi0 = np.asarray(phi0, np.float32)
    blobs = []
    for mode in (None, "1"):
        if mode:
            monkeypatch.setenv("PFLBM_GENERAL_PATH", mode)
        else:
            monkeypatch.delenv("PFLBM_GENERAL_PATH", raising=False)
        sim = P.Simulation(p.as_dict(), phi0, ux0, uy0)
        sim.step(40, form)
        blobs.append(sim.save().cpu().numpy())
        assert not sim.status()
    monkeypatch.delenv("PFLBM_GENERAL_PATH", raising=False)
    for mode, b in zip(("1",), blobs[1:]):
        nd = int((blobs[0] != b).sum())
        print(f"[fast-vs-general] {case}: PFLBM_GENERAL_PATH={mode}: {nd} differing bytes of {b.size}", flush=True)
        assert nd == 0


@pytest.mark.parametrize("shape", [1, 2, 3])
@pytest.mark.parametrize("case", ["periodic_cpf1", "ragged_csf2"])
def test_every_tile_shape_is_bitwise_equal(shape, case, monkeypatch):
    """The step kernels run in any of the tile shapes 64x8 (0), 32x16 (1),
    32x8 (2), 64x4 (3); PFLBM_TILE selects one for a periodic lattice.  A
    node's velocity is the same arithmetic whether its own tile or a
    neighbouring tile's ring evaluates it, so every shape must give the same
    state bit for bit (ragged case: 200 = 6 x 32 + 8 = 3 x 64 + 8 columns,
    150 rows)."""
    import paper_2012_14729_amd as P
    if case == "periodic_cpf1":
        nx, ny, form = 320, 96, "cpf1"
        p = WL.ParamSet(nx=nx, ny=ny, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=4.0, M=0.1, tau_h=0.8)
        phi0 = WL.two_droplets(nx, ny, 20.0, 14.0, 2.0, 4.0)
    else:
        nx, ny, form = 200, 150, "csf2"
        p = WL.ParamSet(nx=nx, ny=ny, rho1=100.0, rho2=1.0, nu1=0.1, nu2=0.1, sigma=2e-3, W=4.0, M=0.1, tau_h=0.8)
        phi0 = WL.two_droplets(nx, ny, 30.0, 22.0, 2.0, 4.0)
    phi0 = np.asarray(phi0, np.float32)
    blobs = []
    for sh in (0, shape):
        monkeypatch.setenv("PFLBM_TILE", str(sh))
        sim = P.Simulation(p.as_dict(), phi0)
        sim.step(30, form)
        blobs.append(sim.save().cpu())
        assert not sim.status()
    monkeypatch.delenv("PFLBM_TILE", raising=False)
    a, b = blobs[0].numpy(), blobs[1].numpy()
    nd = int((a != b).sum())
    print(f"[tile shape] {case} shape {shape}: {nd} differing bytes of {a.size}", flush=True)
    assert nd == 0


@pytest.mark.parametrize("case", ["shear_walls_stf2", "ragged_periodic_cpf1"])
def test_step_blobs_equals_restore_step_save(case):
    """lbm_step_blobs (one step from a saved state into another blob) gives
    the blob that restore + lbm_step + lbm_save gives, bit for bit, and
    leaves the simulation untouched."""
    import paper_2012_14729_amd as P
    if case == "shear_walls_stf2":
        p, phi0, ux0, uy0 = WL.config_shear(nx=136, ny=44, R=12.0, Re=1.0, Ca=0.2)
        form = "stf2"
    else:
        p = WL.ParamSet(nx=100, ny=72, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=4.0, M=0.1, tau_h=0.8)
        phi0, ux0, uy0, form = WL.two_droplets(100, 72, 12.0, 9.0, 2.0, 4.0), None, None, "cpf1"
    sim = P.Simulation(p.as_dict(), np.asarray(phi0, np.float32), ux0, uy0)
    sim.step(9, form)
    b0 = sim.save()
    here = sim.save()
    b1 = torch.zeros_like(b0)
    b2 = torch.zeros_like(b0)
    sim.step_blobs(b0, b1, form)
    sim.step_blobs(b1, b2, form)
    assert torch.equal(sim.save(), here)   # the simulation is untouched
    sim.restore(b0)
    sim.step(1, form)
    r1 = sim.save()
    sim.step(1, form)
    r2 = sim.save()
    torch.cuda.synchronize()
    assert torch.equal(b1, r1) and torch.equal(b2, r2)


def test_full_size_channel_bubble_rises_50000_steps():
    """The 1024x4096 channel (no-slip x walls, periodic y) with a bubble of
    R = 128 at y = 512, Eo = 10, Mo = 1e-3, STF-2, for 50000 steps: the launch
    shape of the full-size run, checked through properties that hold at any
    size.  At density ratio 1000 the method diverges within 5000 steps here
    (and a stationary gas bubble at that ratio diverges in the oracle too), so
    the run uses the density and viscosity ratios 10 of the paper's own
    rising bubble (Table IV), W = 4 and Pe = 1/Cn (Sec. V), U_g = 0.01,
    tau_h = 4.  The order parameter is conserved, the bubble rises every
    5000 steps and reaches a steady rise velocity, and it stays round to
    within its deformation at this Eotvos number."""
    import paper_2012_14729_amd as P
    from paper_2012_14729_amd.diagnostics import bubble_metrics
    from paper_2012_14729_amd.units import Groups, lattice_params
    L, W = 256.0, 4.0
    g = Groups(Re=(10.0 ** 3 / 1e-3) ** 0.25, We=10.0, Pe=L / W, Cn=W / L, Fr=1.0, rho_ratio=0.1, mu_ratio=0.1)
    d = lattice_params(g, L_c=L, U_c=0.01, tau_h=4.0, nx=1024, ny=4096, wall_x=1)
    phi0 = np.asarray(WL.droplet(1024, 4096, 128.0, W, xc=512.0, yc=512.0, inside=-1.0), np.float32)
    s = P.Simulation(d, phi0)
    mass0 = float(s.moments("stf2")["phi"].double().sum())
    hist = []
    for k in range(10):
        s.step(5000, "stf2")
        m = s.moments("stf2")
        assert not s.status(), f"diverged by step {(k + 1) * 5000}"
        yc, vc, C = bubble_metrics(m["phi"], m["uy"])
        hist.append((yc, vc, C))
        print(f"[channel] step {(k + 1) * 5000}: y_c {yc:.1f} v_c {vc:.3e} C {C:.3f}", flush=True)
    dm = abs(float(m["phi"].double().sum()) - mass0) / (1024 * 4096)
    assert dm < 1e-9, dm
    ys = [h[0] for h in hist]
    assert all(b > a for a, b in zip([512.0] + ys, ys))
    assert ys[-1] < 4096 - 256
    assert abs(hist[-1][1] - hist[-2][1]) < 0.02 * hist[-1][1]   # steady rise velocity
    assert 0.85 < hist[-1][2] <= 1.0
