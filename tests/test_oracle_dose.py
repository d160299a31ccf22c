"""Pins of the oracle's absorbed-dose step (fluence times fluence-to-dose
factors summed over groups)."""
import numpy as np

import oracle
from synthetic.workloads import dose_factors, random_small_problem


def test_uniform_field_single_material_is_a_dot_product():
    p = random_small_problem(5, n=(3, 4, 2), G=4, n_mat=1)
    c = np.array([2.0, 0.5, 1.5, 3.0])
    k = np.array([[1.0, 10.0, 100.0, 1000.0]])
    phi = np.repeat(c[:, None], p.V, axis=1)
    # 2*1 + 0.5*10 + 1.5*100 + 3*1000
    assert np.allclose(oracle.dose(p, phi, k), 3157.0, rtol=0, atol=1e-12)


def test_two_materials_voxel_by_voxel():
    p = random_small_problem(6, n=(4, 3, 2), G=1, n_mat=2)
    rng = np.random.default_rng(1)
    phi = rng.uniform(0.1, 1.0, (1, p.V))
    k = np.array([[3.0], [7.0]])
    got = oracle.dose(p, phi, k)
    for v in range(p.V):
        assert got[v] == phi[0, v] * (3.0 if p.material[v] == 0 else 7.0)


def test_linear_in_the_fluence_and_batched():
    p = random_small_problem(7, n=(5, 4, 3), G=3, n_mat=3)
    rng = np.random.default_rng(2)
    a, b = rng.uniform(0, 1, (2, 3, p.V))
    k = rng.uniform(0.1, 2.0, (3, 3))
    lhs = oracle.dose(p, 2.0 * a - 0.5 * b, k)
    rhs = 2.0 * oracle.dose(p, a, k) - 0.5 * oracle.dose(p, b, k)
    assert np.allclose(lhs, rhs, rtol=1e-14, atol=1e-14)
    both = oracle.dose(p, np.stack([a, b]), k)
    assert np.array_equal(both[0], oracle.dose(p, a, k)) and np.array_equal(both[1], oracle.dose(p, b, k))


def test_dose_factor_generator_orders_materials_and_energies():
    k = dose_factors(19, ["air", "tissue", "bone", "metal"])
    assert k.shape == (4, 19) and (k > 0).all()
    assert (np.diff(k, axis=0) > 0).all()  # heavier materials absorb more at every energy
    # the photoelectric term dominates in tissue at low energy: the factor
    # falls from the lowest group (g = G-1) towards the middle of the range
    assert k[1, -1] > k[1, 9]
