"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This module generates problem descriptions only (meshes,
materials, cross-section tables, sources); it holds none of the transport
method's arithmetic.

The paper's own inputs (NJOY/AMPX 90-group libraries, DICOM phantoms, the
X-ray spectrum of its Fig. 10) are not available, so every workload is a
synthetic stand-in with the shapes, sizes and value ranges of the paper's
problems (section II.E): water-like photon cross sections anchored on the
mean free paths the paper quotes (13.9 mm at 20 keV, 60.6 mm at 100 keV),
downscatter-only group matrices, cylinder and ellipsoid phantoms in air, and
a point or cone-beam source outside the phantom.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# material classes: (sigma_t multiplier, scattering-ratio multiplier)
MATERIALS = {
    "air": (0.0012, 1.0),
    "tissue": (1.0, 1.0),
    "bone": (1.8, 0.7),
    "metal": (6.0, 0.3),
}


@dataclass
class ProblemSpec:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    material: np.ndarray            # uint8 [V], v = i + nx*(j + ny*k)
    density: Optional[np.ndarray]   # float64 [V] or None
    sigma_t: np.ndarray             # float64 [n_mat][G]
    sigma_s: np.ndarray             # float64 [n_mat][L+1][G (to)][G (from)]
    sn_order: int
    legendre_order: int
    fixup: int = 0
    name: str = ""

    @property
    def V(self):
        return self.nx * self.ny * self.nz

    @property
    def G(self):
        return self.sigma_t.shape[1]

    @property
    def n_mat(self):
        return self.sigma_t.shape[0]

    def with_density(self, density):
        d = dict(self.__dict__)
        d["density"] = None if density is None else np.ascontiguousarray(density, dtype=np.float64)
        return ProblemSpec(**d)


@dataclass
class SourceSpec:
    position: tuple
    axis: tuple = (1.0, 0.0, 0.0)
    half_angle: float = np.pi        # >= pi: isotropic point source
    spectrum: np.ndarray = field(default_factory=lambda: np.ones(1))
    q_vol: Optional[np.ndarray] = None   # [G][V] volumetric isotropic source (test hook)
    fan_normal: tuple = (0.0, 0.0, 1.0)  # fan beams: normal of the fan plane through the axis
    fan_half_thickness: float = 0.0      # > 0: a fan beam (half_angle in the plane), 0: a cone


# --------------------------------------------------------------------------
# energy grid, spectrum, cross sections
# --------------------------------------------------------------------------
def energy_edges(G, e_min=10.0, e_max=120.0):
    """Group edges in keV, group 0 = highest energy."""
    return np.linspace(e_max, e_min, G + 1)


def energy_mid(G, e_min=10.0, e_max=120.0):
    e = energy_edges(G, e_min, e_max)
    return 0.5 * (e[:-1] + e[1:])


def kramers_spectrum(G, e_min=10.0, e_max=120.0):
    """Bremsstrahlung-like (Kramers) group spectrum, normalised to sum 1."""
    e = energy_edges(G, e_min, e_max)
    hi, lo = e[:-1], e[1:]
    s = e_max * np.log(hi / lo) - (hi - lo)
    return s / s.sum()


def dose_factors(G, material_names, e_min=10.0, e_max=120.0):
    """Synthetic fluence-to-dose factors k[m][g] = E_g (mu_en/rho)_m(E_g) in
    Gy cm^2 per photon, with mu_en/rho = a_m (E/10 keV)^-3 + 0.025 cm^2/g (a
    photoelectric term over a Compton floor; a_m = 0.9, 4.9, 19.6, 98 for
    air, tissue, bone, metal).  A stand-in for tabulated coefficients."""
    a = {"air": 0.9, "tissue": 4.9, "bone": 19.6, "metal": 98.0}
    e = energy_mid(G, e_min, e_max)
    kev_to_j, g_per_kg = 1.602176634e-16, 1e3
    return np.array([[ei * (a[name] * (ei / 10.0) ** -3 + 0.025) * kev_to_j * g_per_kg for ei in e]
                     for name in material_names])


def xs_tables(seed, G, material_names, L, e_min=10.0, e_max=120.0):
    """Water-like multigroup tables scaled per material; downscatter only.

    sigma_t(E) = 0.7194 (E/20 keV)^-0.91486 cm^-1 (through 1/1.39 cm at 20 keV
    and 1/6.06 cm at 100 keV), times U(0.95, 1.05), sorted to rise with g.
    Scattering ratio c_g = 0.25 + 0.65 (E - 10)/110 + U(-0.02, 0.02); a
    fraction f_g ~ U(0.5, 0.8) stays in the group, the rest goes to lower
    groups with weights 0.5^(g''-g-1); Legendre moments sigma_l = sigma_0 gbar^l
    with gbar ~ U(0.05, 0.3) per (material, g -> g'').
    """
    rng = np.random.default_rng(seed)
    em = energy_mid(G, e_min, e_max)
    base = 0.7194 * (em / 20.0) ** (-0.91486) * rng.uniform(0.95, 1.05, G)
    base = np.sort(base)
    c = 0.25 + 0.65 * (em - 10.0) / 110.0 + rng.uniform(-0.02, 0.02, G)
    f = rng.uniform(0.5, 0.8, G)
    M = len(material_names)
    sigma_t = np.zeros((M, G))
    sigma_s = np.zeros((M, L + 1, G, G))
    for m, name in enumerate(material_names):
        mt, mc = MATERIALS[name]
        sigma_t[m] = mt * base
        gbar = rng.uniform(0.05, 0.3, (G, G))
        for g in range(G):
            ss = c[g] * mc * sigma_t[m, g]
            row = np.zeros(G)
            row[g] = f[g] * ss
            if g < G - 1:
                wts = 0.5 ** np.arange(G - g - 1)
                row[g + 1:] = (1.0 - f[g]) * ss * wts / wts.sum()
            for gpp in range(g, G):
                for l in range(L + 1):
                    sigma_s[m, l, gpp, g] = row[gpp] * gbar[g, gpp] ** l
    return sigma_t, sigma_s


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
def _centres(nx, ny, nz, dx, dy, dz):
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    z = (np.arange(nz) + 0.5) * dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def ellipsoid_phantom(seed, n, d, n_ellipsoids, material_ids):
    """Air background, a tissue body, then n_ellipsoids - 1 random rotated
    ellipsoids drawn from material_ids (painter's order)."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    ext = np.array([nx * d, ny * d, nz * d])
    ctr = 0.5 * ext
    X, Y, Z = _centres(nx, ny, nz, d, d, d)
    P = np.stack([X, Y, Z], 1) - ctr
    mat = np.zeros(nx * ny * nz, np.uint8)
    semi = np.array([0.42, 0.38, 0.45]) * ext
    mat[((P / semi) ** 2).sum(1) <= 1.0] = 1
    for _ in range(n_ellipsoids - 1):
        c = rng.uniform(-0.25, 0.25, 3) * ext
        a = rng.uniform(0.03, 0.15, 3) * ext
        Rq, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        m = int(rng.choice(material_ids))
        loc = (P - c) @ Rq
        mat[((loc / a) ** 2).sum(1) <= 1.0] = m
    return mat


def water_cylinder(n, d, radius, height):
    nx, ny, nz = n
    X, Y, Z = _centres(nx, ny, nz, d, d, d)
    cx, cy, cz = nx * d / 2, ny * d / 2, nz * d / 2
    inside = ((X - cx) ** 2 + (Y - cy) ** 2 <= radius ** 2) & (np.abs(Z - cz) <= height / 2)
    return inside.astype(np.uint8)


def cone_source(centre, distance, theta, apex_deg, spectrum, z=None):
    """Cone-beam point source at `distance` from `centre` in direction theta
    (radians, in the x-y plane), aimed at the centre, full apex angle apex_deg."""
    cx, cy, cz = centre
    pos = (cx + distance * np.cos(theta), cy + distance * np.sin(theta), cz if z is None else z)
    axis = (-np.cos(theta), -np.sin(theta), 0.0)
    return SourceSpec(position=pos, axis=axis, half_angle=np.deg2rad(apex_deg) / 2, spectrum=spectrum)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def config1():
    """16^3 x 1 cm, one material, G=2, S4 P1, isotropic unit point source at
    the mesh centre, group 0 only, fixup off, tol 1e-8."""
    rng = np.random.default_rng(1001)
    st = rng.uniform(0.15, 0.25, 2)
    G, L = 2, 1
    sigma_t = st[None, :].copy()
    sigma_s = np.zeros((1, L + 1, G, G))
    sigma_s[0, 0, 0, 0] = 0.6 * st[0]
    sigma_s[0, 0, 1, 1] = 0.6 * st[1]
    sigma_s[0, 0, 1, 0] = 0.2 * st[0]
    sigma_s[0, 1] = 0.2 * sigma_s[0, 0]
    n = 16
    prob = ProblemSpec(n, n, n, 1.0, 1.0, 1.0, np.zeros(n ** 3, np.uint8), None, sigma_t, sigma_s,
                       4, L, fixup=0, name="cfg1-16^3-S4P1-G2")
    src = SourceSpec(position=(8.0, 8.0, 8.0), spectrum=np.array([1.0, 0.0]))
    return prob, src


def config2(G=19):
    """64^3 x 0.5 cm, water cylinder (r 14, h 30 cm) in air, G=19 (10-120 keV),
    S8 P3, cone source 50 cm from the centre along +x, 20 deg apex, fixup on."""
    n, d = 64, 0.5
    mat = water_cylinder((n, n, n), d, 14.0, 30.0)
    sigma_t, sigma_s = xs_tables(1002, G, ["air", "tissue"], 3)
    prob = ProblemSpec(n, n, n, d, d, d, mat, None, sigma_t, sigma_s, 8, 3, fixup=1,
                       name="cfg2-64^3-S8P3-G19")
    src = cone_source((16.0, 16.0, 16.0), 50.0, 0.0, 20.0, kramers_spectrum(G))
    return prob, src


def config3(G=19):
    """128^3 x 0.25 cm, 12 random ellipsoids over air/tissue/bone/metal, G=19,
    S16 P5, cone source as config 2, fixup on."""
    n, d = 128, 0.25
    mat = ellipsoid_phantom(1003, (n, n, n), d, 12, [0, 1, 2, 3])
    sigma_t, sigma_s = xs_tables(1003, G, ["air", "tissue", "bone", "metal"], 5)
    prob = ProblemSpec(n, n, n, d, d, d, mat, None, sigma_t, sigma_s, 16, 5, fixup=1,
                       name="cfg3-128^3-S16P5-G19")
    src = cone_source((16.0, 16.0, 16.0), 50.0, 0.0, 20.0, kramers_spectrum(G))
    return prob, src


def config4(G=10):
    """64^3 x 0.5 cm, 6 ellipsoids over air/tissue/bone, density ~ U(0.8, 1.2),
    G=10, S8 P3, fixup off, detector loss on the exit layer i = 0."""
    n, d = 64, 0.5
    mat = ellipsoid_phantom(1004, (n, n, n), d, 6, [0, 1, 2])
    sigma_t, sigma_s = xs_tables(1004, G, ["air", "tissue", "bone"], 3)
    rng = np.random.default_rng(2004)
    dens = rng.uniform(0.8, 1.2, n ** 3)
    prob = ProblemSpec(n, n, n, d, d, d, mat, dens, sigma_t, sigma_s, 8, 3, fixup=0,
                       name="cfg4-64^3-S8P3-G10-adjoint")
    src = cone_source((16.0, 16.0, 16.0), 50.0, 0.0, 20.0, kramers_spectrum(G))
    return prob, src


def detector_weights(prob, seed=3004):
    """Exit-face detector: W^g(i=0, j, k) = (E_mid^g / 120 keV) U(0.5, 1.5)."""
    rng = np.random.default_rng(seed)
    G, nx, ny, nz = prob.G, prob.nx, prob.ny, prob.nz
    W = np.zeros((G, nz, ny, nx))
    em = energy_mid(G)
    W[:, :, :, 0] = (em / 120.0)[:, None, None] * rng.uniform(0.5, 1.5, (G, nz, ny))
    return W.reshape(G, -1)


def config5_phantoms(G=19):
    out = []
    for n, seed in ((48, 1005), (80, 1006), (96, 1007)):
        d = 0.5
        mat = ellipsoid_phantom(seed, (n, n, n), d, 12, [0, 1, 2, 3])
        sigma_t, sigma_s = xs_tables(1005, G, ["air", "tissue", "bone", "metal"], 3)
        out.append(ProblemSpec(n, n, n, d, d, d, mat, None, sigma_t, sigma_s, 8, 3, fixup=1,
                               name="cfg5-%d^3-S8P3-G19" % n))
    return out


def config5_sources(prob, n_src=90, G=19):
    c = (prob.nx * prob.dx / 2, prob.ny * prob.dy / 2, prob.nz * prob.dz / 2)
    spec = kramers_spectrum(G)
    return [cone_source(c, 50.0, 2 * np.pi * s / n_src, 20.0, spec) for s in range(n_src)]


def table2_water(fine=False, G=90):
    """The run-time benchmark shapes of the paper (section II.E, Table 2): a
    water cylinder of 35 cm diameter centred in a 50 x 50 x 12.5 cm box (axis
    along z, filling the box height), 64x64x16 voxels of 7.81 mm or
    256x256x64 of 1.95 mm, S6 P0, 90 groups of 1 keV over 10-100 keV (a
    Kramers spectrum up to 100 keV), fixup on.  The isotropic point source
    sits "on top of the phantom": 5 cm above the cylinder surface on the +y
    side, at mid height (the paper gives no distance)."""
    n = (256, 256, 64) if fine else (64, 64, 16)
    d = 50.0 / n[0]
    mat = water_cylinder(n, d, 17.5, 12.5)
    sigma_t, sigma_s = xs_tables(1008, G, ["air", "tissue"], 0, e_min=10.0, e_max=100.0)
    prob = ProblemSpec(n[0], n[1], n[2], d, d, d, mat, None, sigma_t, sigma_s, 6, 0, fixup=1,
                       name="table2-%s-%dx%dx%d-S6P0-G%d" % ("fine" if fine else "coarse", n[0], n[1], n[2], G))
    src = SourceSpec(position=(25.0, 25.0 + 17.5 + 5.0, 6.25), spectrum=kramers_spectrum(G, 10.0, 100.0))
    return prob, src


def table2_ct_ring(prob, n_src=16, distance=40.0):
    """The CT mode of the paper's Table 2 (section II.D): 16 cone beams of 30
    degrees (full apex) spaced evenly on a ring in the mid-height plane
    around the phantom, aimed at its centre, solved together in one solve.
    The ring radius is not given; 40 cm from the centre (outside the box)."""
    c = (prob.nx * prob.dx / 2, prob.ny * prob.dy / 2, prob.nz * prob.dz / 2)
    spec = kramers_spectrum(prob.G, 10.0, 100.0)
    return [cone_source(c, distance, 2 * np.pi * s / n_src, 30.0, spec) for s in range(n_src)]


def random_small_problem(seed, n=(5, 6, 7), d=(1.0, 0.8, 1.2), G=2, L=1, sn=4, n_mat=2,
                         fixup=0, density=True):
    """Small random heterogeneous problem for parity and pin tests."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    V = nx * ny * nz
    mat = rng.integers(0, n_mat, V).astype(np.uint8)
    dens = rng.uniform(0.8, 1.2, V) if density else None
    sigma_t = rng.uniform(0.2, 1.0, (n_mat, G))
    sigma_s = np.zeros((n_mat, L + 1, G, G))
    for m in range(n_mat):
        for g in range(G):
            for gpp in range(g, G):
                s0 = rng.uniform(0.1, 0.4) * sigma_t[m, g] * (1.0 if gpp == g else 0.5)
                gbar = rng.uniform(0.05, 0.3)
                for l in range(L + 1):
                    sigma_s[m, l, gpp, g] = s0 * gbar ** l
    return ProblemSpec(nx, ny, nz, d[0], d[1], d[2], mat, dens, sigma_t, sigma_s, sn, L, fixup=fixup,
                       name="random-%d" % seed)
