"""GPU parity at the full workload sizes, against oracle values stored by
tests/golden/make_full_size_golden.py (which runs only the FP64 oracle):
E_rec and the potentials and forces of 64 sampled particles, in the launch
configuration that bench.py times (kpme_evaluate on device-resident inputs).

Tolerances: FP64 path 1e-10 relative; FP32, FP16X3 and BF16X3 paths
relE <= 1e-5 and relative RMS <= 1e-4 over the sampled potentials and forces
(the targets of the mixed-precision path).
"""
import json
import os

import numpy as np
import pytest

from paper_2601_18838_amd import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def relrms(a, b):
    return np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum())


@pytest.mark.parametrize("wl", [systems.WATER_1M, systems.WATER_200K_NONCUBIC],
                         ids=lambda w: w.name)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x3", "bf16x3"])
def test_full_size_against_stored_oracle(wl, prec):
    path = os.path.join(GOLDEN, wl.name + ".json")
    ref = json.load(open(path))
    print(f"[fullsize] {wl.name} {prec}", flush=True)
    from paper_2601_18838_amd import kpme
    pos, q = wl.particles()
    dt = torch.float64 if prec == "fp64" else torch.float32
    pl = kpme.Plan(wl.box, wl.grid, wl.order, wl.beta, tol=wl.tol, precision=prec,
                   max_particles=len(q))
    assert pl.info["rank"] == ref["rank"] and pl.info["r0"] == ref["r0"]
    e4, pot, frc = pl.evaluate(torch.tensor(pos, dtype=dt, device="cuda"),
                               torch.tensor(q, dtype=dt, device="cuda"))
    idx = np.asarray(ref["sample_index"])
    e = float(e4[0])
    phi = pot.double().cpu().numpy()[idx]
    F = frc.double().cpu().numpy()[idx]
    rel_e = abs(e - ref["E_rec"]) / abs(ref["E_rec"])
    print(f"  relE={rel_e:.3e} rmsPhi={relrms(phi, np.asarray(ref['phi'])):.3e} "
          f"rmsF={relrms(F, np.asarray(ref['F'])):.3e}", flush=True)
    if prec == "fp64":
        assert rel_e < 1e-10
        assert relrms(phi, np.asarray(ref["phi"])) < 1e-10
        assert relrms(F, np.asarray(ref["F"])) < 1e-10
    else:
        assert rel_e < 1e-5
        assert relrms(phi, np.asarray(ref["phi"])) < 1e-4
        assert relrms(F, np.asarray(ref["F"])) < 1e-4
