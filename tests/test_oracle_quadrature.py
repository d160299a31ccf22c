"""Pins of the oracle's quadrature and harmonics (no GPU)."""
import os

import numpy as np
import pytest
import scipy.special as sps
from numpy.polynomial import legendre as npleg

import oracle
from oracle.quadrature import class_weights, lqn, lqn_mu1, SUPPORTED_ORDERS
from synthetic.workloads import random_small_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_direction_counts_match_paper():
    # section II.E: S2, S4, S6, S8 give 8, 24, 48, 80 directions
    rows = np.loadtxt(os.path.join(GOLD, "direction_counts.txt"), dtype=int)
    for N, cnt in rows:
        om, w = lqn(N)
        assert len(w) == cnt == N * (N + 2)


@pytest.mark.parametrize("N", SUPPORTED_ORDERS)
def test_weights_sum_to_full_sphere_and_unit_directions(N):
    om, w = lqn(N)
    assert abs(w.sum() - 4 * np.pi) < 1e-14
    assert np.all(w > 0)
    assert np.abs((om ** 2).sum(1) - 1).max() < 1e-15


@pytest.mark.parametrize("N", SUPPORTED_ORDERS)
def test_even_moments_exact_odd_moments_vanish(N):
    om, w = lqn(N)
    # integral over the sphere of mu^(2k) = 4 pi / (2k+1), exact up to k = N/2
    for a in range(3):
        for k in range(0, N // 2 + 1):
            assert abs((w * om[:, a] ** (2 * k)).sum() - 4 * np.pi / (2 * k + 1)) < 2e-14
        for k in range(0, N + 1):
            assert abs((w * om[:, a] ** (2 * k + 1)).sum()) < 1e-14
    # mixed monomials of total degree <= 4 (odd in any axis vanish)
    assert abs((w * om[:, 0] ** 2 * om[:, 1] ** 2).sum() - 4 * np.pi / 15) < 1e-14 or N == 2


def test_closed_forms_s2_s4_s8():
    om, w = lqn(2)
    assert np.allclose(np.abs(om), 1 / np.sqrt(3), atol=2e-16, rtol=0)
    # S4: mu_1^2 = (2 - sqrt(1.6)) / 6 solves the k = 2 moment condition
    assert abs(float(lqn_mu1(4)) - np.sqrt((2 - np.sqrt(1.6)) / 6)) < 1e-16
    # S8: mu_1 = sqrt(1/21); class weights 49/405, 49/540, 5/54
    assert abs(float(lqn_mu1(8)) - np.sqrt(1 / 21)) < 1e-16
    cw = class_weights(8)
    assert abs(cw[(1, 1, 4)] - 49 / 405) < 1e-15
    assert abs(cw[(1, 2, 3)] - 49 / 540) < 1e-15
    assert abs(cw[(2, 2, 2)] - 5 / 54) < 1e-15


def test_s16_point_on_lqn_line_near_standard_table():
    cw = class_weights(16)
    # the 7-digit standard values; the chosen point must be within rounding
    tab = {(1, 1, 8): 0.0489872, (1, 2, 7): 0.0413296, (1, 3, 6): 0.0212326, (1, 4, 5): 0.0256206,
           (2, 2, 6): 0.0360485, (2, 3, 5): 0.0144590, (2, 4, 4): 0.0344958, (3, 3, 4): 0.0085181}
    for k, v in tab.items():
        assert abs(cw[k] - v) < 1e-7
    # octant ordering: reflections of octant 0 in the documented sign pattern
    om, w = lqn(16)
    D = len(w) // 8
    for o in range(8):
        s = np.array([-1 if o & 1 else 1, -1 if o & 2 else 1, -1 if o & 4 else 1])
        assert np.array_equal(om[o * D:(o + 1) * D], om[:D] * s)
        assert np.array_equal(w[o * D:(o + 1) * D], w[:D])


def _real_sph_from_scipy(L, om):
    """Schmidt semi-normalised real harmonics without Condon-Shortley phase,
    built from scipy's complex orthonormal harmonics."""
    theta = np.arccos(np.clip(om[:, 2], -1, 1))
    phi = np.arctan2(om[:, 1], om[:, 0])
    out = np.zeros((len(om), (L + 1) ** 2))
    for l in range(L + 1):
        f = np.sqrt(4 * np.pi / (2 * l + 1))
        for m in range(0, l + 1):
            Y = sps.sph_harm_y(l, m, theta, phi)
            if m == 0:
                out[:, l * l + l] = f * Y.real
            else:
                out[:, l * l + l + m] = f * np.sqrt(2) * (-1) ** m * Y.real
                out[:, l * l + l - m] = f * np.sqrt(2) * (-1) ** m * Y.imag
    return out


def test_harmonics_match_scipy():
    rng = np.random.default_rng(3)
    om = rng.standard_normal((50, 3))
    om /= np.linalg.norm(om, axis=1, keepdims=True)
    L = 7
    R = oracle.harmonics(L, om)
    assert np.abs(R - _real_sph_from_scipy(L, om)).max() < 1e-13


def test_addition_theorem():
    rng = np.random.default_rng(4)
    a = rng.standard_normal((20, 3)); a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = rng.standard_normal((20, 3)); b /= np.linalg.norm(b, axis=1, keepdims=True)
    L = 6
    Ra, Rb = oracle.harmonics(L, a), oracle.harmonics(L, b)
    for l in range(L + 1):
        c = np.zeros(l + 1); c[l] = 1
        lhs = (Ra[:, l * l:(l + 1) ** 2] * Rb[:, l * l:(l + 1) ** 2]).sum(1)
        assert np.abs(lhs - npleg.legval((a * b).sum(1), c)).max() < 1e-14


@pytest.mark.parametrize("N,L", [(2, 0), (4, 1), (6, 2), (8, 3), (12, 4), (16, 5)])
def test_D_times_M_is_identity(N, L):
    p = random_small_problem(0, n=(2, 2, 2), sn=N, L=L)
    M, D = oracle.moment_matrices(p)
    assert np.abs(D @ M - np.eye((L + 1) ** 2)).max() < 1e-13


def test_S16_cannot_resolve_P6():
    # degree-12 products are beyond what S16 integrates: D.M != I at L = 6
    p = random_small_problem(0, n=(2, 2, 2), sn=16, L=6)
    M, D = oracle.moment_matrices(p)
    assert np.abs(D @ M - np.eye(49)).max() > 1e-6


@pytest.mark.parametrize("N,L", [(4, 1), (8, 3)])
def test_moment_form_equals_direct_legendre_sum_of_eq2(N, L):
    """Q_n = sum_n' w_n' sum_l (2l+1)/(4pi) s_l P_l(W_n.W_n') psi_n'  ==  M diag(s) D psi."""
    p = random_small_problem(1, n=(2, 2, 2), sn=N, L=L)
    om, w = lqn(N)
    M, D = oracle.moment_matrices(p)
    rng = np.random.default_rng(5)
    psi = rng.uniform(0, 1, len(w))
    s = rng.uniform(0.1, 1.0, L + 1)
    cos = om @ om.T
    direct = np.zeros(len(w))
    for l in range(L + 1):
        c = np.zeros(l + 1); c[l] = 1
        direct += (2 * l + 1) / (4 * np.pi) * s[l] * npleg.legval(cos, c) @ (w * psi)
    sl = np.concatenate([[s[l]] * (2 * l + 1) for l in range(L + 1)])
    assert np.abs(M @ (sl * (D @ psi)) - direct).max() < 1e-14 * np.abs(direct).max() * 10
