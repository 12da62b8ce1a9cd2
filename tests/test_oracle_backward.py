"""Pin of the oracle's reverse-mode gradient against central finite differences."""
import numpy as np

from oracle import ewald, skp

BOX = np.array([9.0, 11.0, 13.0])


def loss(plan, pos, q, g_e, g_pot):
    r = plan.evaluate(pos, q)
    e_self, e_neu = ewald.self_and_neutral(q, plan.box, plan.beta)
    return g_e * (r["E_rec"] + e_self + e_neu) + float(g_pot @ r["phi"])


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    n = 12
    pos = rng.uniform(0, 1, (n, 3)) * BOX
    q = rng.uniform(-1, 1, n)                    # non-neutral on purpose
    plan = skp.Plan(BOX, (8, 10, 12), 4, 0.7, rank=9)
    g_e, g_pot = 0.7, rng.standard_normal(n)
    gp, gq = skp.backward(plan, pos, q, g_e, g_pot)
    h = 1e-6
    for i in (0, 5, 11):
        for d in range(3):
            a, b = pos.copy(), pos.copy()
            a[i, d] += h
            b[i, d] -= h
            fd = (loss(plan, a, q, g_e, g_pot) - loss(plan, b, q, g_e, g_pot)) / (2 * h)
            assert abs(fd - gp[i, d]) < 1e-6 * max(1.0, abs(gp[i, d]))
        a, b = q.copy(), q.copy()
        a[i] += h
        b[i] -= h
        fd = (loss(plan, pos, a, g_e, g_pot) - loss(plan, pos, b, g_e, g_pot)) / (2 * h)
        assert abs(fd - gq[i]) < 1e-6 * max(1.0, abs(gq[i]))


def test_energy_gradient_is_minus_force():
    rng = np.random.default_rng(4)
    pos = rng.uniform(0, 1, (20, 3)) * BOX
    q = rng.uniform(-1, 1, 20)
    plan = skp.Plan(BOX, (8, 10, 12), 6, 0.7, rank=12)
    gp, _ = skp.backward(plan, pos, q, 1.0, None)
    np.testing.assert_allclose(gp, -plan.evaluate(pos, q)["F"], rtol=1e-12, atol=1e-14)
