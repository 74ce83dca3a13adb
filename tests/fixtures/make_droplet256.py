"""Writes the oracle fixtures of the 256x256 stationary droplet at density
ratio 1000 (the oracle-sized case of the 2048x2048 benchmark droplet):
phi, u_x, u_y after 1000 and 10000 steps for each of the eight force forms.

    python tests/fixtures/make_droplet256.py [form ...]      (default: all eight)

Calls only the oracle (FP64, torch CPU) and the seeded input generators;
nothing here comes from the HIP library.  One process per form, one thread
each; about 20 minutes per form on one core.  Output:
tests/fixtures/droplet256_<form>.npz with float32 fields [256, 256]
(row-major [y][x]) under keys phi_<n>, ux_<n>, uy_<n> for n in (1000, 10000),
plus the step at which the run went non-finite (-1: stable) and the SHA-256
of this script and of the oracle source.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as WL  # noqa: E402
from oracle import lbm_ref as R  # noqa: E402

SNAPSHOTS = (1000, 10000)
FORMS = R.FORMS


def sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


def params():
    p, phi0, _, _ = WL.config_droplet_large(256, R=32.0, W=5.0)
    return p, np.asarray(phi0, np.float32)


def make(form):
    torch.set_num_threads(1)
    p, phi0 = params()
    op = R.Params(**{k: (None if k == "rho0" else v) for k, v in p.as_dict().items()})
    st = R.init(op, torch.tensor(phi0, dtype=torch.float64))
    out, blew_up, t0 = {}, -1, time.time()
    for n in range(1, SNAPSHOTS[-1] + 1):
        st = R.step(st, form, op)
        if n in SNAPSHOTS or n % 500 == 0:
            m = R.moments(st, form, op)
            if not all(bool(torch.isfinite(m[k]).all()) for k in ("phi", "ux", "uy")):
                blew_up = n
                break
            if n in SNAPSHOTS:
                for k in ("phi", "ux", "uy"):
                    out[f"{k}_{n}"] = m[k].numpy().astype(np.float32)
            print(f"{form}: step {n}, {time.time() - t0:.0f} s", flush=True)
    out["nonfinite_at_step"] = np.int64(blew_up)
    out["script_sha256"] = np.array(sha(os.path.abspath(__file__)))
    out["oracle_sha256"] = np.array(sha(os.path.join(ROOT, "oracle", "lbm_ref.py")))
    np.savez_compressed(os.path.join(HERE, f"droplet256_{form}.npz"), **out)


if __name__ == "__main__":
    for f in (sys.argv[1:] or FORMS):
        make(f)
