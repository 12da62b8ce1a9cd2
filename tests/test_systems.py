"""The seeded input generators: determinism, geometry, neutrality."""
import math

import numpy as np

from paper_2601_18838_amd import systems


def test_water_geometry_and_charges():
    box = (30.0, 40.0, 50.0)
    pos, q = systems.water(200, box, seed=9)
    assert pos.shape == (600, 3) and q.shape == (600,)
    assert np.all(pos >= 0) and np.all(pos <= np.asarray(box))
    # charges: O, H, H per molecule, exactly neutral in float32 arithmetic
    np.testing.assert_array_equal(q[0::3], np.float32(-0.834))
    np.testing.assert_array_equal(q[1::3], np.float32(0.417))
    assert q.astype(np.float32).reshape(-1, 3).sum(axis=1).max() == 0.0
    # bond lengths and angle (minimum image, positions were wrapped)
    b = np.asarray(box)
    d1 = pos[1::3] - pos[0::3]
    d2 = pos[2::3] - pos[0::3]
    d1 -= np.round(d1 / b) * b
    d2 -= np.round(d2 / b) * b
    np.testing.assert_allclose(np.linalg.norm(d1, axis=1), 0.9572, atol=2e-5)
    np.testing.assert_allclose(np.linalg.norm(d2, axis=1), 0.9572, atol=2e-5)
    cosang = (d1 * d2).sum(1) / np.linalg.norm(d1, axis=1) / np.linalg.norm(d2, axis=1)
    np.testing.assert_allclose(np.degrees(np.arccos(cosang)), 104.52, atol=5e-3)


def test_float32_representable_and_deterministic():
    pos, q = systems.uniform_pm1(1000, (20.0, 20.0, 20.0), seed=1)
    np.testing.assert_array_equal(pos.astype(np.float32).astype(np.float64), pos)
    pos2, q2 = systems.uniform_pm1(1000, (20.0, 20.0, 20.0), seed=1)
    np.testing.assert_array_equal(pos, pos2)
    assert q.sum() == 0.0


def test_rotations_are_orthonormal():
    R = systems.random_rotations(np.random.default_rng(0), 50)
    np.testing.assert_allclose(np.einsum('nij,nkj->nik', R, R),
                               np.broadcast_to(np.eye(3), (50, 3, 3)), atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)


def test_batch_systems_ranges():
    bs = systems.batch_systems(count=8)
    for wl, pos, q in bs:
        assert 5000 <= wl.n <= 300000 and wl.n % 2 == 0
        assert q.sum() == 0.0 and len(q) == wl.n
        assert wl.grid in systems.BATCH_GRIDS and wl.order in (4, 6)
        assert 6 <= wl.rank <= 24
        assert math.isclose(wl.box[0], wl.grid[0])
