"""Arithmetic the single-precision collision relies on, checked in IEEE float32
with numpy (no GPU). The first-order equilibrium term is one rounded product
per direction pair: a1 (c.j) on the axes and a2 (c.j) on the diagonals, with
a1 = fl(omega fl(1/3)) and a2 = (omega - 2 a1)/4. Momentum is conserved to
rounding only if 2 a1 + 4 a2 equals omega exactly (Eqs. bgkCollision and
equilibrium: the first moment of the equilibrium is j)."""
import numpy as np

F32 = np.float32
THIRD_HI = F32(float.fromhex("0x1.555556p-2"))  # the float nearest 1/3


def coefficients(omega):
    a1 = omega * THIRD_HI
    a2 = (omega - F32(2) * a1) * F32(0.25)
    return a1, a2


def omegas():
    rng = np.random.default_rng(7)
    tau = np.concatenate([0.5 + rng.uniform(1e-6, 1e-3, 100000), 0.5 + rng.uniform(1e-3, 1.5, 100000),
                          0.5 + np.geomspace(1e-6, 50.0, 1000)])
    om = (1.0 / tau).astype(F32)
    # the ends of the range BGK allows, and powers of two
    edge = np.array([np.nextafter(F32(2), F32(0)), F32(1), F32(0.5), F32(0.25), np.nextafter(F32(1), F32(2))], F32)
    return np.concatenate([om, edge])


def test_remainder_is_exact_and_momentum_sum_is_omega():
    om = omegas()
    a1, a2 = coefficients(om)
    # the subtraction is exact (Sterbenz: omega / 2 <= 2 a1 <= 2 omega) ...
    r = om - F32(2) * a1
    assert np.all(r.astype(np.float64) == om.astype(np.float64) - 2.0 * a1.astype(np.float64))
    # ... so the two axis terms and the four diagonal terms sum to omega exactly
    assert np.all(2.0 * a1.astype(np.float64) + 4.0 * a2.astype(np.float64) == om.astype(np.float64))
    # and a2 stays within a few ulp of omega / 12
    rel = np.abs(a2.astype(np.float64) * 12.0 / om.astype(np.float64) - 1.0)
    assert rel.max() < 4 * 2.0 ** -24


def test_rounded_third_on_both_terms_does_not_conserve_momentum():
    # the form the remainder replaces: a2 = a1 / 4 with a1 = fl(omega fl(1/3))
    om = omegas()
    a1 = om * THIRD_HI
    a2 = a1 * F32(0.25)
    miss = 2.0 * a1.astype(np.float64) + 4.0 * a2.astype(np.float64) != om.astype(np.float64)
    assert miss.mean() > 0.5
