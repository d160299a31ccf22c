"""Pins of the oracle's adjoint and density gradient (no GPU)."""
import numpy as np
import pytest

import oracle
from synthetic.workloads import SourceSpec, random_small_problem


def _sweep_matrix(p, om, sig):
    V = p.V
    A = np.zeros((V, V))
    for v in range(V):
        e = np.zeros(V)
        e[v] = 1.0
        A[:, v] = oracle.sweep(p, om, sig, e)[0]
    return A


def test_dd_sweep_transpose_is_reverse_sweep():
    p = random_small_problem(80, n=(3, 4, 2))
    rng = np.random.default_rng(2)
    sig = rng.uniform(0.1, 2.0, p.V)
    for om in ([0.3, -0.5, 0.81], [-0.6, 0.64, -0.48]):
        om = np.array(om) / np.linalg.norm(om)
        A = _sweep_matrix(p, om, sig)
        B = _sweep_matrix(p, -om, sig)
        assert np.abs(A.T - B).max() < 1e-15 * np.abs(A).max() * 10


def _problem():
    p = random_small_problem(81, n=(3, 4, 3), sn=4, L=1, G=2, n_mat=2, density=True)
    src = SourceSpec(position=(-2.0, 1.5, 1.7), axis=(1.0, 0.1, 0.0), half_angle=np.deg2rad(35),
                     spectrum=np.array([1.0, 0.4]))
    W = np.random.default_rng(3).uniform(0, 1, (p.G, p.V))
    return p, src, W


def test_reciprocity():
    p, src, W = _problem()
    r = oracle.adjoint(p, src, W, tol=1e-15)
    assert abs(r["J"] - r["recip"]) < 1e-12 * abs(r["J"])


def test_gradient_matches_central_differences():
    p, src, W = _problem()
    r = oracle.adjoint(p, src, W, tol=1e-15)
    g = r["grad"]
    h = 1e-3
    fd = np.zeros(p.V)
    for v in range(p.V):
        d = p.density.copy()
        d[v] += h
        jp = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        d[v] -= 2 * h
        jm = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        fd[v] = (jp - jm) / (2 * h)
    assert np.abs(g - fd).max() < 1e-5 * np.abs(fd).max()
    # both the ray back-projection and the scattering terms matter here
    assert np.abs(fd).max() > 0


def test_gradient_source_inside_mesh():
    p = random_small_problem(82, n=(4, 3, 3), sn=2, L=0, G=2, n_mat=2, density=True)
    src = SourceSpec(position=(2.1, 1.3, 1.45), spectrum=np.array([1.0, 0.2]))
    W = np.random.default_rng(4).uniform(0, 1, (p.G, p.V))
    g = oracle.adjoint(p, src, W, tol=1e-15)["grad"]
    h = 1e-3
    for v in (0, 7, 20, 35):
        d = p.density.copy(); d[v] += h
        jp = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        d[v] -= 2 * h
        jm = (W * oracle.solve(p.with_density(d), src, tol=1e-15)["phi_total"]).sum()
        assert abs(g[v] - (jp - jm) / (2 * h)) < 1e-5 * np.abs(g).max()
