"""Pins of the sub-sweep plane math (eqs. 8-22, Table 1) and the ray trace
of the uncollided fluence (eq. 4), no GPU."""
import itertools
import os

import numpy as np
import pytest

import oracle
from synthetic.workloads import ProblemSpec, SourceSpec, random_small_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _brute_plane(S, nx, ny, nz):
    return sum(1 for i in range(nx) for j in range(ny) for k in range(nz) if i + j + k == S)


@pytest.mark.parametrize("n", [(1, 1, 1), (5, 5, 5), (4, 7, 3), (16, 2, 9), (3, 3, 12), (8, 8, 1)])
def test_eq9_plane_size_matches_brute_force(n):
    nx, ny, nz = n
    tot = 0
    for S in range(0, nx + ny + nz - 2):
        P = oracle.plane_count(S, nx, ny, nz)
        assert P == _brute_plane(S, nx, ny, nz)
        assert P == len(oracle.plane_enumerate(S, nx, ny, nz))
        tot += P
    assert tot == nx * ny * nz
    # eq. 8: the last sub-sweep holds a single voxel
    assert oracle.plane_count(nx + ny + nz - 3, nx, ny, nz) == 1
    assert oracle.plane_count(nx + ny + nz - 2, nx, ny, nz) == 0


def test_table1_enumeration():
    rows = np.loadtxt(os.path.join(GOLD, "table1_subsweep_S4.txt"), dtype=int)
    got = oracle.plane_enumerate(4, 5, 5, 5)
    assert np.array_equal(got, rows[:, 1:4])
    assert (rows[:, 1:4].sum(1) == 4).all()


@pytest.mark.parametrize("fixup", [0, 1])
def test_subsweep_order_gives_identical_sweep(fixup):
    p = random_small_problem(11, n=(5, 4, 6), fixup=fixup)
    rng = np.random.default_rng(0)
    sig = rng.uniform(0.1, 2.0, p.V)
    Q = rng.uniform(-0.2, 1.0, p.V)
    for om in ([0.3, -0.5, 0.81], [-0.6, 0.64, -0.48], [0.1, 0.2, -0.97]):
        om = np.array(om) / np.linalg.norm(om)
        a, oa, _ = oracle.sweep(p, om, sig, Q, order=0)
        b, ob, _ = oracle.sweep(p, om, sig, Q, order=1)
        assert np.array_equal(a, b) and np.array_equal(oa, ob)


def _homog(n=(6, 5, 4), d=(0.7, 0.9, 1.1), sigma=0.8):
    nx, ny, nz = n
    return ProblemSpec(nx, ny, nz, *d, np.zeros(nx * ny * nz, np.uint8), None,
                       np.array([[sigma, 0.5 * sigma]]), np.zeros((1, 1, 2, 2)), 4, 0)


def test_uncollided_homogeneous_is_exp_over_r2():
    p = _homog()
    src = SourceSpec(position=(-2.0, 1.3, 7.0), spectrum=np.array([1.0, 2.0]))
    phiu, oms = oracle.raytrace(p, src)
    v = np.arange(p.V)
    i, j, k = v % p.nx, (v // p.nx) % p.ny, v // (p.nx * p.ny)
    c = np.stack([(i + .5) * p.dx, (j + .5) * p.dy, (k + .5) * p.dz], 1)
    d = c - np.array(src.position)
    r = np.linalg.norm(d, axis=1)
    # the part of the path inside the box [0, n_a d_a]: entry parameter is the
    # largest of the per-axis slab entry parameters
    ext = np.array([p.nx * p.dx, p.ny * p.dy, p.nz * p.dz])
    xs = np.array(src.position)
    t_in = np.zeros(p.V)
    for a in range(3):
        if xs[a] < 0:
            t_in = np.maximum(t_in, (0.0 - xs[a]) / d[:, a])
        elif xs[a] > ext[a]:
            t_in = np.maximum(t_in, (ext[a] - xs[a]) / d[:, a])
    lin = r * (1 - t_in)
    for g, (sg, s) in enumerate(zip([0.8, 0.4], [1.0, 2.0])):
        ref = s * np.exp(-sg * lin) / (4 * np.pi * r ** 2)
        assert np.abs(phiu[g] / ref - 1).max() < 1e-13
    assert np.abs(oms - d / r[:, None]).max() < 1e-15


def test_uncollided_source_inside_homogeneous():
    p = _homog(n=(6, 6, 6), d=(1.0, 1.0, 1.0))
    src = SourceSpec(position=(3.0, 3.0, 3.0), spectrum=np.array([1.0, 0.0]))
    phiu, _ = oracle.raytrace(p, src)
    v = np.arange(p.V)
    c = np.stack([(v % 6 + .5), (v // 6 % 6 + .5), (v // 36 + .5)], 1)
    r = np.linalg.norm(c - 3.0, axis=1)
    assert np.abs(phiu[0] / (np.exp(-0.8 * r) / (4 * np.pi * r ** 2)) - 1).max() < 1e-14


def test_two_slab_closed_form():
    # materials change at x = 3 (cm); ray from outside along a slanted path
    nx, ny, nz = 6, 4, 4
    mat = np.zeros((nz, ny, nx), np.uint8)
    mat[:, :, 3:] = 1
    p = ProblemSpec(nx, ny, nz, 1.0, 1.0, 1.0, mat.ravel(), None, np.array([[0.3], [1.1]]),
                    np.zeros((2, 1, 1, 1)), 2, 0)
    xs = np.array([-1.0, 0.2, -0.7])
    for v in [5, 20, 63, 95]:
        i, j, k = v % nx, (v // nx) % ny, v // (nx * ny)
        xe = np.array([i + .5, j + .5, k + .5])
        lam = oracle.ray_material_path(p, xs, xe)
        d = xe - xs
        r = np.linalg.norm(d)
        # exact: the ray is inside the mesh for all t >= max of the entry parameters
        t0 = max((0 - xs[a]) / d[a] if d[a] > 0 else -np.inf for a in range(3))
        t0 = max(t0, (0 - xs[2]) / d[2])
        t3 = (3 - xs[0]) / d[0]
        l0 = r * (min(t3, 1) - t0) if t3 > t0 else 0.0
        l1 = r * (1 - max(t3, t0)) if t3 < 1 else 0.0
        assert abs(lam[0] - max(l0, 0)) < 1e-13 and abs(lam[1] - max(l1, 0)) < 1e-13


def test_path_lengths_match_fine_sampling():
    p = random_small_problem(5, n=(7, 5, 6), n_mat=3, density=True)
    rng = np.random.default_rng(9)
    for _ in range(6):
        xs = rng.uniform(-3, 9, 3)
        v = rng.integers(p.V)
        i, j, k = v % p.nx, (v // p.nx) % p.ny, v // (p.nx * p.ny)
        xe = np.array([(i + .5) * p.dx, (j + .5) * p.dy, (k + .5) * p.dz])
        lam = oracle.ray_material_path(p, xs, xe)
        n = 1_000_000
        t = (np.arange(n) + 0.5) / n
        pts = xs[None, :] + t[:, None] * (xe - xs)[None, :]
        ii = np.floor(pts / np.array([p.dx, p.dy, p.dz])).astype(int)
        ok = ((ii >= 0) & (ii < np.array([p.nx, p.ny, p.nz]))).all(1)
        vv = ii[ok, 0] + p.nx * (ii[ok, 1] + p.ny * ii[ok, 2])
        seg = np.linalg.norm(xe - xs) / n
        ref = np.bincount(p.material[vv], weights=p.density[vv] * seg, minlength=p.n_mat)
        assert np.abs(lam - ref).max() < 1e-5


def test_cone_restricts_uncollided():
    p = _homog(n=(8, 8, 8), d=(1, 1, 1), sigma=0.1)
    src = SourceSpec(position=(20.0, 4.0, 4.0), axis=(-1.0, 0.0, 0.0), half_angle=np.deg2rad(5.0),
                     spectrum=np.array([1.0, 1.0]))
    phiu, oms = oracle.raytrace(p, src)
    ang = np.arccos(np.clip(-oms[:, 0], -1, 1))
    inside = ang <= np.deg2rad(5.0)
    assert inside.any() and (~inside).any()
    assert (phiu[:, ~inside] == 0).all() and (phiu[:, inside] > 0).all()


def _fan_members(p, src):
    """Fan membership by arc-cosines: elevation = 90 deg minus the angle to
    the plane normal; in-plane angle between the axis and the direction's
    projection onto the plane."""
    v = np.arange(p.V)
    c = np.stack([(v % p.nx + .5) * p.dx, (v // p.nx % p.ny + .5) * p.dy, (v // (p.nx * p.ny) + .5) * p.dz], 1)
    d = c - np.array(src.position)
    r = np.linalg.norm(d, axis=1)
    a = np.array(src.axis, dtype=float)
    a /= np.linalg.norm(a)
    n = np.array(src.fan_normal, dtype=float)
    n -= (n @ a) * a
    n /= np.linalg.norm(n)
    elev = np.pi / 2 - np.arccos(np.clip((d @ n) / r, -1, 1))
    proj = d - np.outer(d @ n, n)
    inplane = np.arccos(np.clip((proj @ a) / np.linalg.norm(proj, axis=1), -1, 1))
    return (np.abs(elev) <= src.fan_half_thickness) & (inplane <= src.half_angle), r, d


def test_fan_beam_pure_absorber():
    """A fan beam in a homogeneous pure absorber: e^{-sigma r}/(4 pi r^2)
    inside the fan (membership by an independent angle computation), zero
    outside, and the same with the fan normal reversed."""
    p = _homog(n=(9, 8, 7), d=(1.0, 1.0, 1.0))
    src = SourceSpec(position=(4.37, 3.91, 3.53), axis=(1.0, 0.3, -0.2), half_angle=np.deg2rad(50.0),
                     spectrum=np.array([1.0, 0.0]), fan_normal=(0.1, 0.2, 1.0),
                     fan_half_thickness=np.deg2rad(17.0))
    phiu, _ = oracle.raytrace(p, src)
    inside, r, _ = _fan_members(p, src)
    assert 10 < inside.sum() < p.V // 2
    ref = np.where(inside, np.exp(-0.8 * r) / (4 * np.pi * r ** 2), 0.0)
    assert np.array_equal(phiu[0] > 0, inside)
    assert np.abs(phiu[0] - ref).max() < 1e-14 * ref.max()
    flipped = SourceSpec(**{**src.__dict__, "fan_normal": (-0.1, -0.2, -1.0)})
    assert np.array_equal(oracle.raytrace(p, flipped)[0], phiu)
