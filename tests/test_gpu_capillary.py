"""End-to-end physics of the GPU path: a capillary wave (Sec. V.C) released
from rest, density ratio 1, H = 80 (box 80 x 240, periodic x, no-slip top
and bottom, Re = 50, We = 1, h0 = 0.01 H).  Its amplitude follows the
analytic solution (Eqs. 44-46) with the time-averaged error E2 (Eq. 47)
that the paper prints in Table III for each force form."""
import json
import os

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", ["stf2", "cpf2", "pf1", "csf2"])
def test_capillary_wave_error_matches_table3(form):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2012_14729_amd.benchmarks import capillary_wave
    tab = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table3_capillary.json")))
    printed = tab["E2"]["ratio1_H80"][tab["forms"].index(form)]
    print(f"[capillary] {form} H=80", flush=True)
    r = capillary_wave(form, H=80)
    print(f"[capillary]   E2={r['E2']:.4f} (Table III {printed})", flush=True)
    assert not r["diverged"]
    assert abs(r["E2"] - printed) < 0.25 * printed + 0.005
    # the first quarter period: the wave crosses zero within 8 % of the analytic
    # time (the diffuse interface, W = 4 on a wavelength of 80, slows it by ~5 %)
    t, h, th = r["t"], r["h"], r["theory"]
    def first(a):
        i = int(((a[1:] < 0) & (a[:-1] >= 0)).nonzero()[0][0])
        return t[i] + (t[i + 1] - t[i]) * a[i] / (a[i] - a[i + 1])
    assert abs(first(h) - first(th)) / first(th) < 0.08
