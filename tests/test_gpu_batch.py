"""GPU tests of the batched engine (lbm_batch_*): every instance of a batch
of uneven sizes and force forms matches a single-lattice run of the same
instance bit for bit, and the oracle within the parity bar; divergence is
flagged per instance."""
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


def small_batch(count=10, seed=3):
    insts = WL.batch_instances(count=count, seed=seed, sides=(32, 48, 64, 80, 96, 112))
    return [p for p, _, _ in insts], [f for _, f, _ in insts], [np.asarray(x, np.float32) for _, _, x in insts]


def test_batch_matches_single_lattice_bitwise():
    import paper_2012_14729_amd as P
    params, forms, phis = small_batch()
    print(f"[batch] sizes {[p.nx for p in params]} forms {forms}", flush=True)
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    b.step(37)     # graph chunks + eager remainder
    b.step(21)     # odd start parity
    torch.cuda.synchronize()
    assert not any(b.status())
    for k, (p, f, phi) in enumerate(zip(params, forms, phis)):
        s = P.Simulation(p.as_dict(), phi)
        s.step(58, P.FORMS[f])
        ms, mb = s.moments(P.FORMS[f]), b.moments(k)
        for key in ("phi", "rho", "ux", "uy", "P"):
            assert torch.equal(ms[key], mb[key]), (k, key)


def test_batch_matches_oracle():
    import paper_2012_14729_amd as P
    params, forms, phis = small_batch(count=4, seed=11)
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    b.step(60)
    for k, (p, f, phi) in enumerate(zip(params, forms, phis)):
        op = R.Params(**{kk: (None if kk == "rho0" else v) for kk, v in p.as_dict().items()})
        st = R.run(R.init(op, torch.tensor(phi, dtype=torch.float64)), R.FORMS[f], op, 60)
        ref = {kk: v.numpy() for kk, v in R.moments(st, R.FORMS[f], op).items()}
        got = {kk: v.cpu().numpy().astype(np.float64) for kk, v in b.moments(k).items()}
        assert np.abs(got["phi"] - ref["phi"]).max() < 1e-5
        umax = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max()
        eu = max(np.abs(got["ux"] - ref["ux"]).max(), np.abs(got["uy"] - ref["uy"]).max()) / umax
        print(f"[batch] instance {k} side {p.nx} form {R.FORMS[f]}: e_u {eu:.2e}", flush=True)
        assert eu < 1e-5


def test_batch_flags_only_the_diverged_instance():
    import paper_2012_14729_amd as P
    params, forms, phis = small_batch(count=5, seed=5)
    phis[2] = phis[2].copy()
    phis[2][3, 4] = np.nan    # non-finite input set on the host for instance 2
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    b.step(20)
    assert b.status() == [False, False, True, False, False]


def wide_batch():
    """Instances wide enough to hold interior tiles (sides 96..256), all eight forms."""
    sides = (96, 160, 192, 256, 128, 224, 144, 200)
    params, phis = [], []
    for k, s in enumerate(sides):
        params.append(WL.ParamSet(nx=s, ny=s // 2 + 8 * (k % 3), rho1=(1.0, 10.0, 100.0)[k % 3], rho2=1.0, nu1=0.1,
                                  nu2=0.1, sigma=3e-3, W=4.0, M=0.1, tau_h=0.8))
        phis.append(np.asarray(WL.two_droplets(params[-1].nx, params[-1].ny, s / 8, s / 10, 2.0, 4.0), np.float32))
    return params, list(range(8)), phis


@pytest.mark.parametrize("cfg", ["0,0,1", "0,1,1", "0,0,2", "0,1,2", "0,1,0", "1,0,1", "1,1,1", "1,0,2",
                                 "1,1,2", "1,0,0", "1,1,0", "0,0,0", "0,2,0", "0,2,1", "1,2,0", "1,2,2"])
def test_every_launch_shape_matches_single_lattice(cfg, monkeypatch):
    """Whatever launch shape the tuner picks (one kernel or one per form;
    general, interior or wrapped addressing; persistent or one workgroup
    per tile), the instances evolve bit for bit as single lattices."""
    import paper_2012_14729_amd as P
    params, forms, phis = wide_batch()
    monkeypatch.setenv("PFLBM_BATCH_CFG", cfg)
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    assert b.config["split"] == int(cfg[0]) and b.config["fast"] == int(cfg[2])
    b.step(23)
    torch.cuda.synchronize()
    assert not any(b.status())
    for k, (p, f, phi) in enumerate(zip(params, forms, phis)):
        s = P.Simulation(p.as_dict(), phi)
        s.step(23, P.FORMS[f])
        ms, mb = s.moments(P.FORMS[f]), b.moments(k)
        for key in ("phi", "rho", "ux", "uy", "P"):
            assert torch.equal(ms[key], mb[key]), (cfg, k, key)


def test_tuned_batch_starts_from_phi0(monkeypatch):
    """Creation times the candidate launch shapes by stepping the batch and
    then rebuilds the initial state: a tuned batch and an untuned one give
    identical states."""
    import paper_2012_14729_amd as P
    params, forms, phis = wide_batch()
    params = params[:5]
    forms, phis = forms[:5], phis[:5]
    monkeypatch.delenv("PFLBM_BATCH_CFG", raising=False)
    monkeypatch.delenv("PFLBM_BATCH_TUNE", raising=False)
    tuned = P.Batch([p.as_dict() for p in params], forms, phis)
    cfg = tuned.config
    print(f"[batch] tuned shape {cfg}", flush=True)
    assert cfg["ms_per_step"] > 0 and cfg["split"] in (0, 1) and cfg["fast"] in (0, 1, 2) and cfg["blocks_per_cu"] >= 0
    monkeypatch.setenv("PFLBM_BATCH_TUNE", "0")
    plain = P.Batch([p.as_dict() for p in params], forms, phis)
    for b in (tuned, plain):
        b.step(12)
    torch.cuda.synchronize()
    for k in range(len(params)):
        mt, mp = tuned.moments(k), plain.moments(k)
        for key in ("phi", "rho", "ux", "uy", "P"):
            assert torch.equal(mt[key], mp[key]), (k, key)


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("cfg", ["1,1,2", "0,1,0", "1,2,0"])
def test_every_tile_shape_matches_single_lattice(shape, cfg, monkeypatch):
    """Batched step kernels in every tile shape (PFLBM_BATCH_SHAPE 0-3), and
    with a shape per instance (4: 32x8 where 64-wide tiles idle more lanes,
    so 64x8 and 32x8 tiles share the batch), evolve the instances bit for
    bit as single lattices."""
    import paper_2012_14729_amd as P
    params, forms, phis = wide_batch()
    monkeypatch.setenv("PFLBM_BATCH_CFG", cfg)
    monkeypatch.setenv("PFLBM_BATCH_SHAPE", str(shape))
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    monkeypatch.delenv("PFLBM_BATCH_SHAPE", raising=False)
    shapes = [(64, 8), (32, 16), (32, 8), (64, 4)]
    if shape < 4:
        want = [shapes[shape]] * len(params)
    else:   # the 32-wide shape where it leaves fewer idle lanes in the last tile column
        want = [(32, 8) if (-p.nx) % 32 < (-p.nx) % 64 else (64, 8) for p in params]
        assert len(set(want)) == 2
    assert b.tile_shapes() == want
    b.step(19)
    torch.cuda.synchronize()
    assert not any(b.status())
    for k, (p, f, phi) in enumerate(zip(params, forms, phis)):
        s = P.Simulation(p.as_dict(), phi)
        s.step(19, P.FORMS[f])
        ms, mb = s.moments(P.FORMS[f]), b.moments(k)
        for key in ("phi", "rho", "ux", "uy", "P"):
            assert torch.equal(ms[key], mb[key]), (shape, cfg, k, key)


def test_full_size_batch_sampled_instances():
    """The benchmark's batch (512 instances, sides 32-512, seed 14729, 48.7 M
    nodes) in the launch shape the tuner picks, as the benchmark runs it:
    sampled instances (the smallest, the largest, ragged sides, every force
    form) equal single-lattice runs bit for bit after 40 steps, and the
    smallest sampled instance matches the oracle within the parity bar."""
    import paper_2012_14729_amd as P
    insts = WL.batch_instances(512, seed=14729)
    params = [p for p, _, _ in insts]
    forms = [f for _, f, _ in insts]
    phis = [np.asarray(x, np.float32) for _, _, x in insts]
    b = P.Batch([p.as_dict() for p in params], forms, phis)
    print(f"[full batch] launch shape {b.config}", flush=True)
    steps = 40
    b.step(steps)
    torch.cuda.synchronize()
    sides = [p.nx for p in params]
    pick = {sides.index(min(sides)), sides.index(max(sides))}
    for f in range(8):   # one instance of each form, ragged sides first
        ks = [k for k in range(512) if forms[k] == f and sides[k] % 64 and k not in pick]
        pick.add(ks[0] if ks else forms.index(f))
    for k in sorted(pick):
        p, f, phi = params[k], forms[k], phis[k]
        s = P.Simulation(p.as_dict(), phi)
        s.step(steps, P.FORMS[f])
        ms, mb = s.moments(P.FORMS[f]), b.moments(k)
        for key in ("phi", "rho", "ux", "uy", "P"):
            assert torch.equal(ms[key], mb[key]), (k, p.nx, key)
        assert b.status()[k] == s.status()
    k = min(pick, key=lambda i: sides[i])
    p, f, phi = params[k], forms[k], phis[k]
    op = R.Params(**{kk: (None if kk == "rho0" else v) for kk, v in p.as_dict().items()})
    st = R.run(R.init(op, torch.tensor(phi, dtype=torch.float64)), R.FORMS[f], op, steps)
    ref = {kk: v.numpy() for kk, v in R.moments(st, R.FORMS[f], op).items()}
    got = {kk: v.cpu().numpy().astype(np.float64) for kk, v in b.moments(k).items()}
    umax = np.sqrt(ref["ux"] ** 2 + ref["uy"] ** 2).max()
    eu = max(np.abs(got["ux"] - ref["ux"]).max(), np.abs(got["uy"] - ref["uy"]).max()) / umax
    ephi = np.abs(got["phi"] - ref["phi"]).max()
    print(f"[full batch] {len(pick)} sampled instances bitwise; instance {k} ({p.nx}^2, {R.FORMS[f]}) vs oracle: "
          f"e_phi {ephi:.2e} e_u {eu:.2e}", flush=True)
    assert ephi < 1e-5 and eu < 1e-5
