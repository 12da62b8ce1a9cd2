"""GPU check of the allocation-free energy entry point (kpme_energy_noalloc)
against kpme_energy, through the C ABI: bitwise equal on the same inputs
(the same kernels and reduction order, only the scratch array differs), on
two calls in a row, the second with a smaller input."""
import numpy as np
import pytest

from paper_2601_18838_amd import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec", ["fp64", "fp16x3"])
def test_energy_noalloc_matches_energy(prec):
    from paper_2601_18838_amd import kpme
    print(f"[noalloc] energy {prec}", flush=True)
    box, grid, p, beta = (20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35
    pos, q = systems.uniform_pm1(3000, box, 41)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pl = kpme.Plan(box, grid, p, beta, rank=8, precision=prec, max_particles=len(q))
    P = torch.tensor(pos, dtype=dt, device="cuda")
    Qc = torch.tensor(q, dtype=dt, device="cuda")
    _, pot, _ = pl.evaluate(P, Qc)
    for n in (3000, 1001):            # the second call is smaller
        ref = pl.energy(Qc[:n], pot[:n])
        out = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
        pl.energy_noalloc(Qc[:n], pot[:n], out)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        np.testing.assert_array_equal(a, b)
        e_rec = 0.5 * float((Qc[:n].double() * pot[:n].double()).sum())
        assert abs(a[0] - e_rec) < 1e-12 * max(abs(e_rec), 1.0)
