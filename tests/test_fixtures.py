"""The stored oracle fixtures are current: each was written by the committed
generator from the committed oracle (both hashed into the file), and holds
finite fields of the expected shape.  A change to either source needs the
fixtures written again (python tests/fixtures/make_droplet256.py)."""
import hashlib
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FIX = os.path.join(ROOT, "tests", "fixtures")
FORMS = ("stf1", "stf2", "cpf1", "cpf2", "pf1", "pf2", "csf1", "csf2")


def _sha(path):
    return hashlib.sha256(open(path, "rb").read()).hexdigest()


@pytest.mark.parametrize("form", FORMS)
def test_droplet256_fixture_is_current(form):
    d = np.load(os.path.join(FIX, f"droplet256_{form}.npz"))
    assert str(d["script_sha256"]) == _sha(os.path.join(FIX, "make_droplet256.py"))
    assert str(d["oracle_sha256"]) == _sha(os.path.join(ROOT, "oracle", "lbm_ref.py"))
    assert int(d["nonfinite_at_step"]) == -1
    for n in (1000, 10000):
        for k in ("phi", "ux", "uy"):
            a = d[f"{k}_{n}"]
            assert a.shape == (256, 256) and a.dtype == np.float32 and np.isfinite(a).all()
        assert np.abs(d[f"phi_{n}"]).max() < 1.05
