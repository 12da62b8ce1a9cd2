"""GPU parity of the sinc-quadrature SKP (Sec. 2.1.2) against the oracle's
quadrature plan at the same rule (N, h), through the C ABI.

The library builds its own terms from the closed form; the operator, the
whole evaluation and the energies are compared with the FP64 oracle at equal
(N, h).  Tolerances as for the nested-SVD factors: FP64 1e-11; FP32 grids
and potentials 1e-5, forces 2e-5; FP16X3 / BF16X3 grids 1e-5 / 1e-4 of the
largest value (16 significand bits in the BF16 split, see
test_gpu_parity.py) and the mixed-precision targets (relE <= 1e-5, relative
RMS potential and force <= 1e-4) for the whole path.
"""
import numpy as np
import pytest

from oracle import quadrature as qd
from paper_2601_18838_amd import systems

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


PREC = {"fp64": torch.float64, "fp32": torch.float32, "bf16x3": torch.float32,
        "fp16x3": torch.float32}
TOL = {"fp64": dict(grid=1e-11, pot=1e-11, force=1e-11, energy=1e-11),
       "fp32": dict(grid=1e-5, pot=1e-5, force=2e-5, energy=1e-5),
       "bf16x3": dict(grid=1e-4, pot=1e-4, force=1e-4, energy=1e-5),
       "fp16x3": dict(grid=1e-5, pot=1e-5, force=2e-5, energy=1e-5)}

CASES = {
    # name: (box, grid, p, beta, N, n, kind, seed)
    "small_pm1": ((20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35, 6, 1000, "pm1", 31),
    "ragged_noncubic": ((21.0, 26.0, 31.0), (20, 25, 30), 6, 0.6, 9, 1500, "water", 32),
    "k3p_160": ((24.0, 40.0, 160.0), (24, 40, 160), 4, 0.34, 5, 1200, "pm1", 33),
}


def dev(x, prec):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=PREC[prec], device="cuda")


def host(x):
    return x.detach().cpu().double().numpy()


def relmax(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def relrms(a, b):
    return np.sqrt(((a - b) ** 2).sum() / max((b ** 2).sum(), 1e-300))


_ORACLE = {}


def oracle(case):
    if case not in _ORACLE:
        box, grid, p, beta, N, n, kind, seed = CASES[case]
        if kind == "pm1":
            pos, q = systems.uniform_pm1(n, box, seed)
        else:
            pos, q = systems.water(n // 3, box, seed)
        h, _ = qd.best_h(box, grid, p, beta, N)
        pl = qd.Plan(box, grid, p, beta, N=N, h=h)
        _ORACLE[case] = (pl, pos, q, pl.evaluate(pos, q))
    return _ORACLE[case]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp16x3"])
@pytest.mark.parametrize("case", list(CASES))
def test_sinc_quadrature_matches_oracle(case, prec):
    print(f"[sinc] {case} {prec}", flush=True)
    from paper_2601_18838_amd import kpme
    orc, pos, q, ref = oracle(case)
    box, grid, p, beta = CASES[case][:4]
    pl = kpme.Plan(box, grid, p, beta, rank=orc.rank, precision=prec, max_particles=len(q),
                   method="sinc", quad_h=orc.h)
    info = pl.info
    assert info["rank"] == info["r0"] == orc.rank and info["quad_N"] == orc.N
    assert info["skp_method"] == 1 and info["quad_h"] == orc.h
    assert abs(info["zero_mode"] - orc.c0) < 1e-12 * abs(orc.c0)
    tol = TOL[prec]
    Phi = pl.skp_apply(dev(ref["Q"], prec))
    assert relmax(host(Phi), ref["Phi"]) < tol["grid"]
    e4, pot, frc = pl.evaluate(dev(pos, prec), dev(q, prec))
    e4, pot, frc = host(e4), host(pot), host(frc)
    rel_e = abs(e4[0] - ref["E_rec"]) / abs(ref["E_rec"])
    print(f"  relE={rel_e:.2e} rmsPhi={relrms(pot, ref['phi']):.2e} "
          f"rmsF={relrms(frc, ref['F']):.2e}", flush=True)
    assert rel_e < tol["energy"]
    assert relrms(pot, ref["phi"]) < tol["pot"]
    assert relrms(frc, ref["F"]) < tol["force"]


def test_sinc_quadrature_water_100k_tolerance_rule():
    """The 1e5-atom water box with the library's own rule for a 1e-6 symbol
    tolerance: the oracle's symbol error at that rule is within it, and the
    FP16X3 and FP64 evaluations match the oracle at the same rule."""
    wl = systems.WATER_100K
    print(f"[sinc] {wl.name}", flush=True)
    from paper_2601_18838_amd import kpme
    pos, q = wl.particles()
    res = {}
    for prec in ("fp64", "fp16x3"):
        pl = kpme.Plan(wl.box, wl.grid, wl.order, wl.beta, rank=0, tol=1e-6, precision=prec,
                       max_particles=len(q), method="sinc")
        e4, pot, frc = pl.evaluate(dev(pos, prec), dev(q, prec))
        res[prec] = (host(e4), host(pot), host(frc), pl.info)
    info = res["fp64"][3]
    N, h = info["quad_N"], info["quad_h"]
    assert res["fp16x3"][3]["quad_N"] == N and res["fp16x3"][3]["quad_h"] == h
    assert qd.symbol_error(wl.box, wl.grid, wl.order, wl.beta, N, h) <= 1e-6
    orc = qd.Plan(wl.box, wl.grid, wl.order, wl.beta, N=N, h=h)
    ref = orc.evaluate(pos, q)
    for prec, (te, tf) in (("fp64", (1e-10, 1e-10)), ("fp16x3", (1e-5, 1e-4))):
        e, pot, frc, _ = res[prec]
        rel_e = abs(e[0] - ref["E_rec"]) / abs(ref["E_rec"])
        print(f"  {prec} R={2 * N + 1}: relE={rel_e:.2e} rmsF={relrms(frc, ref['F']):.2e}",
              flush=True)
        assert rel_e < te
        assert relrms(pot, ref["phi"]) < tf
        assert relrms(frc, ref["F"]) < tf
