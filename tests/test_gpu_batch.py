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
