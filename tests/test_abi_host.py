"""Host-side checks of the C ABI: exported symbols, argument validation, and
the FP64 factor construction against the oracle (no device needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import skp
from paper_2601_18838_amd import kpme

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpme.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(kpme_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = kpme.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_status_strings():
    L = kpme.lib()
    for s in range(6):
        assert L.kpme_status_string(s)
    assert L.kpme_status_string(99) == b"unknown status"


def _create(box=(20, 20, 20), grid=(16, 16, 16), p=4, beta=0.35, rank=8, tol=0.0, prec=1,
            nmax=100):
    h = ctypes.c_void_p()
    st = kpme.lib().kpme_plan_create(ctypes.byref(h), kpme._dbl3(box), kpme._int3(grid), p,
                                     beta, rank, tol, prec, nmax, 0)
    return st, h


@pytest.mark.parametrize("kw,code", [
    (dict(box=(0, 20, 20)), 1), (dict(box=(20, float("nan"), 20)), 1),
    (dict(p=5), 2), (dict(p=3), 2), (dict(p=14), 1), (dict(grid=(3, 16, 16)), 1),
    (dict(grid=(16, 16, 300)), 1), (dict(grid=(6, 16, 16), p=8), 1), (dict(beta=-1.0), 1),
    (dict(rank=0, tol=0.0), 1), (dict(rank=0, tol=2.0), 1), (dict(prec=7), 1),
    (dict(nmax=0), 1), (dict(grid=(160, 16, 16)), 2),
    # the split-precision stage-2 kernels hold at most 128 columns
    (dict(grid=(32, 160, 32), prec=2), 2), (dict(grid=(32, 160, 32), prec=3), 2),
])
def test_plan_create_validates_before_touching_a_device(kw, code):
    st, h = _create(**kw)
    assert st == code, (st, kpme.lib().kpme_last_error())
    assert h.value is None


def test_plan_create_without_a_device_reports_device_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    assert kpme.device_count() == 0
    st, h = _create()
    assert st == 4 and h.value is None
    assert b"device" in kpme.lib().kpme_last_error().lower()


def test_calls_on_invalid_handles_fail_cleanly():
    L = kpme.lib()
    null = ctypes.c_void_p()
    assert L.kpme_plan_destroy(null) == 1
    assert L.kpme_spread(null, 0, None, None, None, None) == 1
    assert L.kpme_skp_apply(null, None, None, None) == 1
    assert L.kpme_gather(null, 0, None, None, None, None, None, None) == 1
    assert L.kpme_energy(null, 0, None, None, None, None) == 1
    assert L.kpme_evaluate(null, 0, None, None, None, None, None, None) == 1
    info = kpme.PlanInfo()
    assert L.kpme_plan_info(null, ctypes.byref(info)) == 1


def _rank1(vec, r):
    return (vec[0][r][:, None, None] * vec[1][r][None, :, None] * vec[2][r][None, None, :])


@pytest.mark.parametrize("box,grid,p,beta,rank", [
    ((20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35, None),
    ((9.0, 11.0, 13.0), (8, 10, 12), 4, 0.7, None),
    ((9.0, 11.0, 13.0), (9, 10, 11), 6, 0.7, None),
    ((30.0, 37.5, 45.0), (20, 25, 30), 4, 0.34, 24),
])
def test_factors_match_the_oracle(box, grid, p, beta, rank):
    orc = skp.Plan(box, grid, p, beta, rank=rank)
    lib = kpme.factors_compute(box, grid, p, beta, rank=rank or 10 ** 6)
    th = orc.theta
    scale = np.abs(th).max()
    # the kept operator and its truncation are unique (ties aside): compare
    # the weights, the reconstructed symbol and the scalars
    R = min(len(orc.terms), len(lib["omega"]))
    w_o = np.array([t[0] for t in orc.terms[:R]])
    big = w_o > 1e-10 * w_o[0]
    np.testing.assert_allclose(lib["omega"][:R][big], w_o[big], rtol=1e-9)
    rec_lib = sum(lib["omega"][r] * _rank1(lib["vec"], r) for r in range(len(lib["omega"])))
    rec_orc = skp.reconstruct(orc.terms, th.shape)
    assert np.abs(rec_lib - rec_orc).max() < 1e-11 * scale
    assert abs(lib["theta_norm"] - np.linalg.norm(th)) < 1e-12 * np.linalg.norm(th)
    assert abs(lib["trunc_err"] - orc.trunc_err) < 1e-10 * np.linalg.norm(th) + 1e-6 * orc.trunc_err
    assert abs(lib["zero_mode"] - orc.c0) < 1e-11 * scale
    # each term is a unit-norm rank-1 tensor of even mode vectors
    for j in range(3):
        v = lib["vec"][j]
        np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-12)
        K = v.shape[1]
        np.testing.assert_allclose(v, v[:, np.mod(-np.arange(K), K)], atol=1e-12)


def test_tolerance_rank_matches_the_oracle():
    box, grid = (20.0, 20.0, 20.0), (16, 16, 16)
    orc = skp.Plan(box, grid, 4, 0.35, tol=1e-6)
    lib = kpme.factors_compute(box, grid, 4, 0.35, rank=0, tol=1e-6)
    assert len(lib["omega"]) == orc.rank == 22


def test_factors_compute_rejects_a_small_output_buffer():
    with pytest.raises(kpme.KpmeError) as e:
        kpme.factors_compute((20, 20, 20), (16, 16, 16), 4, 0.35, rank=30, max_terms=8)
    assert e.value.status == 1


@pytest.mark.parametrize("box,grid,p,beta,N", [
    ((20.0, 20.0, 20.0), (16, 16, 16), 4, 0.35, 9),
    ((9.0, 11.0, 13.0), (8, 10, 12), 4, 0.7, 5),
    ((30.0, 37.5, 45.0), (20, 25, 30), 6, 0.34, 14),
])
def test_sinc_quadrature_factors_match_the_oracle(box, grid, p, beta, N):
    """Library sinc-quadrature terms (host FP64) against the oracle's at the
    same rule (N, h): weights, unit mode vectors, the correction constant,
    the Frobenius distance to theta_hat and the symbol error."""
    from oracle import quadrature as qd
    h, err = qd.best_h(box, grid, p, beta, N)
    lib = kpme.factors_compute(box, grid, p, beta, rank=2 * N + 1, method="sinc", quad_h=h)
    orc = qd.Plan(box, grid, p, beta, N=N, h=h)
    assert len(lib["omega"]) == orc.rank == 2 * N + 1
    assert lib["quad_N"] == N and lib["quad_h"] == h
    np.testing.assert_array_equal(lib["group"], np.arange(2 * N + 1))
    w_o = np.array([t[0] for t in orc.terms])
    np.testing.assert_allclose(lib["omega"], w_o, rtol=1e-12)
    for j in range(3):
        v_o = np.array([t[1 + j] for t in orc.terms])
        np.testing.assert_allclose(lib["vec"][j], v_o, atol=1e-13)
    scale = orc.theta.max()
    assert abs(lib["zero_mode"] - orc.c0) < 1e-12 * abs(orc.c0)
    assert abs(lib["zero_mode"] - qd.correction_constant(box, N, h)) < 1e-12 * abs(orc.c0)
    assert abs(lib["trunc_err"] - orc.trunc_err) < 1e-10 * orc.trunc_err + 1e-14 * scale
    assert abs(lib["sym_err"] - err) <= 1e-10 * err + 1e-15


@pytest.mark.parametrize("tol", [1e-4, 1e-7])
def test_sinc_quadrature_selection_meets_the_tolerance(tol):
    """The library's own choice of (N, h) for a tolerance: the oracle's
    symbol error at that rule is within it, and one node pair fewer with the
    oracle's best h is not."""
    from oracle import quadrature as qd
    box, grid, p, beta = (30.0, 37.5, 45.0), (20, 25, 30), 4, 0.34
    lib = kpme.factors_compute(box, grid, p, beta, rank=0, tol=tol, method="sinc")
    N, h = lib["quad_N"], lib["quad_h"]
    assert len(lib["omega"]) == 2 * N + 1
    e = qd.symbol_error(box, grid, p, beta, N, h)
    assert e <= tol and abs(e - lib["sym_err"]) <= 1e-10 * e + 1e-15
    if N > 0:
        assert qd.best_h(box, grid, p, beta, N - 1)[1] > tol


def test_sinc_quadrature_rejects_an_even_rank():
    with pytest.raises(kpme.KpmeError) as e:
        kpme.factors_compute((20, 20, 20), (16, 16, 16), 4, 0.35, rank=8, method="sinc")
    assert e.value.status == 1


@pytest.mark.parametrize("box,Kc,L,M,beta,rank", [
    ((10.0, 11.0, 12.0), (4, 4, 4), 6, 5, 0.6, None),
    ((20.0, 20.0, 20.0), (5, 5, 5), 8, 12, 0.35, 40),
    ((18.0, 21.0, 24.0), (6, 7, 8), 4, 8, 0.5, 30),
])
def test_lagrange_factors_match_the_oracle(box, Kc, L, M, beta, rank):
    """Library factors of the mode-truncated kernel on the Lagrange grid
    (K_j = K_c,j (L - 1) points, |m_j| <= M) against the oracle's nested SVD
    of the same symbol: the kept operator, the truncation and the correction
    constant."""
    from oracle import lagrange as lg
    orc = lg.Plan(box, Kc, L, M, beta, rank=rank)
    grid = orc.K
    lib = kpme.factors_compute(box, grid, L, beta, rank=rank or 10 ** 6,
                               interpolation="lagrange", mode_cutoff=M)
    th = orc.theta
    scale = np.abs(th).max()
    rec_lib = sum(lib["omega"][r] * _rank1(lib["vec"], r) for r in range(len(lib["omega"])))
    rec_orc = skp.reconstruct(orc.terms, th.shape)
    assert len(lib["omega"]) == orc.rank
    assert np.abs(rec_lib - rec_orc).max() < 1e-11 * scale
    assert abs(lib["theta_norm"] - np.linalg.norm(th)) < 1e-12 * np.linalg.norm(th)
    assert abs(lib["trunc_err"] - orc.trunc_err) < 1e-10 * np.linalg.norm(th) + 1e-6 * orc.trunc_err
    assert abs(lib["zero_mode"] - orc.c0) < 1e-11 * scale


def test_lagrange_sinc_quadrature_terms_vanish_beyond_the_cutoff():
    box, grid, L, M, beta = (10.0, 11.0, 12.0), (20, 20, 20), 6, 5, 0.6
    lib = kpme.factors_compute(box, grid, L, beta, rank=0, tol=1e-6, method="sinc",
                               interpolation="lagrange", mode_cutoff=M)
    from oracle import spme
    for j in range(3):
        far = np.abs(spme.signed_modes(grid[j])) > M
        assert np.all(lib["vec"][j][:, far] == 0.0)
    from oracle import lagrange as lg
    th = lg.alpha_hat(box, grid, M, beta)
    rec = sum(lib["omega"][r] * _rank1(lib["vec"], r) for r in range(len(lib["omega"])))
    rec[0, 0, 0] = 0.0
    assert np.abs(rec - th).max() <= 1e-6 * th.max() * (1 + 1e-9)


@pytest.mark.parametrize("grid,M,code", [((20, 21, 20), 5, 1), ((20, 20, 20), 10, 1),
                                         ((20, 20, 20), 0, 1)])
def test_lagrange_plan_options_are_validated(grid, M, code):
    h = ctypes.c_void_p()
    opts = kpme._options("nested_svd", 0.0, "lagrange", M)
    st = kpme.lib().kpme_plan_create_ex(ctypes.byref(h), kpme._dbl3((10, 11, 12)),
                                        kpme._int3(grid), 6, 0.6, 8, 0.0, 1, 100, 0,
                                        ctypes.byref(opts))
    assert st == code and h.value is None
    opts = kpme._options("nested_svd", 0.0, "bspline", 3)
    st = kpme.lib().kpme_plan_create_ex(ctypes.byref(h), kpme._dbl3((10, 11, 12)),
                                        kpme._int3((20, 20, 20)), 6, 0.6, 8, 0.0, 1, 100, 0,
                                        ctypes.byref(opts))
    assert st == 1


def test_rect_form_is_refused_for_split_precisions_before_any_device_work():
    h = ctypes.c_void_p()
    opts = kpme._options("nested_svd", 0.0, "bspline", 0, "rect")
    st = kpme.lib().kpme_plan_create_ex(ctypes.byref(h), kpme._dbl3((20, 20, 20)),
                                        kpme._int3((16, 16, 16)), 4, 0.35, 8, 0.0, 3, 100, 0,
                                        ctypes.byref(opts))
    assert st == 2 and h.value is None
