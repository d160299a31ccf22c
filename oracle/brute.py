"""Brute-force dense/sparse solve of the fully assembled discrete system
(TEST INFRASTRUCTURE ONLY, tiny meshes).

This is an independent check of the oracle's sweep + source iteration: no
sweeping and no iteration.  For every group g, direction n and voxel v the
unknowns are the cell fluence psi and the three downwind face fluences; the
equations are written in their primitive form:

  balance   sum_a |Omega_a|/Delta_a (psi_out,a - psi_in,a) + sigma psi = Q
  closure   psi_out,a = 2 psi - psi_in,a            (diamond difference)
  vacuum    psi_in,a = 0 on the domain boundary

and the scattering source is the direct double sum of eq. 2 with the
Legendre kernel (no moments, no addition theorem):

  Q_n = sum_{g'<=g} sum_{n'} w_{n'} sum_l (2l+1)/(4 pi) rho sigma_{s,l}^{g'->g}
        P_l(Omega_n . Omega_{n'}) psi_{n'}^{g'} + q_n^g

with q_n^g an isotropic volumetric source q^g/(4 pi) and/or the
first-collision source of eq. 5 written directly from the uncollided
fluence phi_u (a delta in the direction source -> voxel):
  sum_{g'<=g} sum_l (2l+1)/(4 pi) rho sigma_{s,l}^{g'->g} P_l(Omega_n . Omega_s) phi_u^{g'}.

The whole system (all groups at once) is solved with scipy's sparse LU.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre as npleg


def _legendre(l, x):
    c = np.zeros(l + 1)
    c[l] = 1.0
    return npleg.legval(x, c)


def solve(prob, omega, w, q_vol=None, phi_u=None, omega_s=None):
    """Returns psi [G][Nd][V] (cell fluences) and phi [G][V] = sum_n w_n psi_n."""
    nx, ny, nz = prob.nx, prob.ny, prob.nz
    V, G, L = prob.V, prob.G, prob.legendre_order
    Nd = len(w)
    rho = np.ones(V) if prob.density is None else np.asarray(prob.density)
    mat = np.asarray(prob.material)
    st, ss = prob.sigma_t, prob.sigma_s
    h = (prob.dx, prob.dy, prob.dz)

    def uid(g, n, v, k):  # k = 0 cell, 1..3 outflow x, y, z
        return ((g * Nd + n) * V + v) * 4 + k

    N = G * Nd * V * 4
    rows, cols, vals = [], [], []
    rhs = np.zeros(N)

    def add(r, c, x):
        rows.append(r); cols.append(c); vals.append(x)

    cosang = omega @ omega.T  # [n][n']
    pl = [_legendre(l, cosang) for l in range(L + 1)]
    for g in range(G):
        for n in range(Nd):
            om = omega[n]
            s = [1 if om[a] > 0 else -1 for a in range(3)]
            for v in range(V):
                i, j, k = v % nx, (v // nx) % ny, v // (nx * ny)
                idx = (i, j, k)
                eq_bal = uid(g, n, v, 0)
                sig = rho[v] * st[mat[v], g]
                add(eq_bal, uid(g, n, v, 0), sig)
                for a in range(3):
                    cc = abs(om[a]) / h[a]
                    add(eq_bal, uid(g, n, v, 1 + a), cc)
                    up = list(idx)
                    up[a] -= s[a]
                    inside = 0 <= up[0] < nx and 0 <= up[1] < ny and 0 <= up[2] < nz
                    if inside:
                        vu = up[0] + nx * (up[1] + ny * up[2])
                        add(eq_bal, uid(g, n, vu, 1 + a), -cc)
                    # closure: psi_out - 2 psi + psi_in = 0
                    eq = uid(g, n, v, 1 + a)
                    add(eq, uid(g, n, v, 1 + a), 1.0)
                    add(eq, uid(g, n, v, 0), -2.0)
                    if inside:
                        add(eq, uid(g, n, vu, 1 + a), 1.0)
                # scattering (moved to the left-hand side)
                m = mat[v]
                for gp in range(g + 1):
                    for n2 in range(Nd):
                        kern = 0.0
                        for l in range(L + 1):
                            kern += (2 * l + 1) / (4 * np.pi) * ss[m, l, g, gp] * pl[l][n, n2]
                        if kern != 0.0:
                            add(eq_bal, uid(gp, n2, v, 0), -w[n2] * rho[v] * kern)
                q = 0.0
                if q_vol is not None:
                    q += q_vol[g, v] / (4 * np.pi)
                if phi_u is not None:
                    ca = float(om @ omega_s[v])
                    for gp in range(g + 1):
                        for l in range(L + 1):
                            q += (2 * l + 1) / (4 * np.pi) * rho[v] * ss[m, l, g, gp] * _legendre(l, ca) * phi_u[gp, v]
                rhs[eq_bal] = q
    A = sps.csc_matrix((vals, (rows, cols)), shape=(N, N))
    x = spla.spsolve(A, rhs)
    psi = x.reshape(G, Nd, V, 4)[..., 0]
    phi = np.einsum("n,gnv->gv", w, psi)
    return psi, phi
