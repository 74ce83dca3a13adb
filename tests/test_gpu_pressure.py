"""GPU parity of the hydrodynamic pressure p_h = P_sf - D_form
(lbm_hydro_pressure, Sec. II.B) against the FP64 oracle, for every force
form, on a periodic droplet pair and on the sheared drop between moving
walls (ragged tiles: neither side is a multiple of the 64x8 tile)."""
import math

import numpy as np
import pytest
import torch

import workloads as WL
from oracle import lbm_ref as R

pytestmark = pytest.mark.gpu

TOL_P = 1e-4   # same bar as P_sf in the step parity tests


def _case(name):
    if name == "droplets_periodic":
        nx, ny = 100, 72
        p = WL.ParamSet(nx=nx, ny=ny, rho1=10.0, rho2=1.0, nu1=0.1, nu2=0.2, sigma=5e-3, W=4.0, M=0.1, tau_h=0.8)
        return p, WL.two_droplets(nx, ny, 14.0, 10.0, 2.0, 4.0), None, None
    p, phi0, ux0, uy0 = WL.config_shear(nx=136, ny=44, R=10.0, Re=1.0, Ca=0.2)
    return p, phi0, ux0, uy0


def _oracle_params(p):
    d = p.as_dict()
    if d["rho0"] is None or (isinstance(d["rho0"], float) and math.isnan(d["rho0"])):
        d["rho0"] = None
    return R.Params(**d)


@pytest.mark.parametrize("case", ["droplets_periodic", "shear_walls"])
@pytest.mark.parametrize("form", R.FORMS)
def test_hydro_pressure_parity(case, form):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_14729_amd as P
    p, phi0, ux0, uy0 = _case(case)
    phi0 = np.asarray(phi0, np.float32)
    f32 = lambda a: None if a is None else np.asarray(a, np.float32)
    t64 = lambda a: None if a is None else torch.tensor(np.asarray(a, np.float32), dtype=torch.float64)
    steps = 120
    print(f"[p_h] {case} {p.nx}x{p.ny} form={form} steps={steps}", flush=True)
    op = _oracle_params(p)
    st = R.run(R.init(op, t64(phi0), t64(ux0), t64(uy0)), form, op, steps)
    ref_ph = R.hydro_pressure(st, form, op).numpy()
    ref = {k: v.numpy() for k, v in R.moments(st, form, op).items()}
    sim = P.Simulation(p.as_dict(), phi0, f32(ux0), f32(uy0))
    sim.step(steps, form)
    got_ph = sim.hydro_pressure(form).cpu().numpy().astype(np.float64)
    got_p = sim.moments(form)["P"].cpu().numpy().astype(np.float64)
    assert not sim.status()
    umax = float(np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max())
    scale = max(np.abs(ref["P"]).max(), np.abs(ref_ph).max(), np.abs(ref["rho"]).max() * umax / 3.0)
    e = float(np.abs(got_ph - ref_ph).max() / scale)
    print(f"[p_h]   error {e:.3e}", flush=True)
    assert e < TOL_P, e
    # D_form is what separates the two outputs of the same state
    d_ref = ref["P"] - ref_ph
    d_got = got_p - got_ph
    assert float(np.abs(d_got - d_ref).max()) < TOL_P * scale


def test_hydro_pressure_rejects_bad_output():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_14729_amd as P
    p, phi0, _, _ = WL.config_droplet64()
    sim = P.Simulation(p.as_dict(), np.asarray(phi0, np.float32))
    with pytest.raises(ValueError):
        sim.hydro_pressure("cpf1", out=torch.empty((p.ny, p.nx), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        sim.hydro_pressure("cpf1", out=torch.empty((p.ny, p.nx + 1), dtype=torch.float32, device="cuda"))
