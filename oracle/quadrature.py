"""Level-symmetric S_N quadrature for the oracle (test infrastructure only).

The paper (section II.E) offers the S2, S4, S6 and S8 sets with N(N+2)
directions (8, 24, 48, 80) and uses the weights in the scalar-fluence sum of
eq. 3, but it does not print the sets.  The reading taken here is the
level-symmetric LQn family, built from its defining moment conditions and
solved in 40-digit arithmetic (mpmath), so the FP64 values are correctly
rounded:

* N/2 direction cosines per axis with mu_i^2 = mu_1^2 + (i-1) * 2(1 - 3 mu_1^2)/(N-2);
* octant points (mu_a, mu_b, mu_c) with a + b + c = N/2 + 2 (1-based);
* one weight per permutation class, chosen so that sum_p w_p mu_p^(2k) = 1/(2k+1)
  per octant for k = 0, 2, 3, ..., N/2 (k = 1 then holds by mu^2+eta^2+xi^2 = 1);
* mu_1 is the root that makes that over-determined system consistent;
* for S16 the class system is rank-deficient (a line of solutions); the point
  taken is the one nearest the 7-digit S16 weights of the standard LQn table
  (Lewis and Miller, Computational Methods of Neutron Transport, 1984).

Weights are scaled so the full sphere sums to 4 pi (eq. 3 then returns the
scalar fluence).  Ordering: n = o * N(N+2)/8 + p, octant o has signs
(-1)^(o&1), (-1)^((o>>1)&1), (-1)^((o>>2)&1) on (mu, eta, xi), and inside an
octant p runs over a ascending, then b ascending.
"""
from functools import lru_cache

import mpmath as mp
import numpy as np

# S14 is left out: like S16 its class system is rank-deficient and no anchor
# table is carried for it.
SUPPORTED_ORDERS = (2, 4, 6, 8, 10, 12, 16)

# mu_1 brackets around the standard tabulated LQn values (root isolation only)
_MU1_GUESS = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 10: 0.1893213,
              12: 0.1672126, 14: 0.1519859, 16: 0.1389568}

# 7-digit S16 class weights (per-point, octant-normalised), standard LQn table
_S16_ANCHOR = {(1, 1, 8): 0.0489872, (1, 2, 7): 0.0413296, (1, 3, 6): 0.0212326,
               (1, 4, 5): 0.0256206, (2, 2, 6): 0.0360485, (2, 3, 5): 0.0144590,
               (2, 4, 4): 0.0344958, (3, 3, 4): 0.0085181}


def octant_points(N):
    """1-based level triples (a, b, c) of one octant, in quadrature order."""
    n = N // 2
    return [(a, b, n + 2 - a - b) for a in range(1, n + 1) for b in range(1, n + 2 - a)]


def _levels(N, mu1):
    n = N // 2
    if N == 2:
        return [mp.sqrt(mp.mpf(1) / 3)]
    d = 2 * (1 - 3 * mu1 ** 2) / (N - 2)
    return [mp.sqrt(mu1 ** 2 + i * d) for i in range(n)]


def _class_system(N, mu1):
    pts = octant_points(N)
    classes = sorted(set(tuple(sorted(p)) for p in pts))
    idx = {c: i for i, c in enumerate(classes)}
    x = _levels(N, mu1)
    ks = [0] + list(range(2, N // 2 + 1))
    A = mp.zeros(len(ks), len(classes))
    b = mp.zeros(len(ks), 1)
    for r, k in enumerate(ks):
        for p in pts:
            A[r, idx[tuple(sorted(p))]] += x[p[0] - 1] ** (2 * k)
        b[r] = mp.mpf(1) / (2 * k + 1)
    return A, b, classes


def _consistency(N, mu1):
    """Signed distance of b from the column space of A (zero at the LQn mu_1)."""
    A, b, _ = _class_system(N, mu1)
    U, S, V = mp.svd_r(A, full_matrices=True)
    rank = sum(1 for s in S if s > mp.mpf(10) ** (-25))
    if rank >= A.rows:
        return mp.mpf(0)
    u = U[:, rank]
    k = max(range(A.rows), key=lambda i: abs(u[i]))
    if u[k] < 0:
        u = -u
    return sum(u[i] * b[i] for i in range(A.rows))


@lru_cache(maxsize=None)
def lqn_mu1(N):
    """mu_1 of the LQn set (40-digit root, returned as mpf string)."""
    with mp.workdps(40):
        if N == 2:
            return str(mp.sqrt(mp.mpf(1) / 3))
        g = mp.mpf(_MU1_GUESS[N])
        r = mp.findroot(lambda m: _consistency(N, m), (g * (1 - 1e-4), g * (1 + 1e-4)), solver='illinois')
        return str(r)


@lru_cache(maxsize=None)
def _lqn_cached(N):
    if N not in SUPPORTED_ORDERS:
        raise ValueError("S_N order must be one of %s" % (SUPPORTED_ORDERS,))
    with mp.workdps(40):
        mu1 = mp.mpf(lqn_mu1(N))
        pts = octant_points(N)
        A, b, classes = _class_system(N, mu1)
        # minimum-norm least-squares solution through the SVD
        U, S, V = mp.svd_r(A)
        r = sum(1 for s in S if s > mp.mpf(10) ** (-25))
        w = mp.zeros(A.cols, 1)
        for i in range(r):
            coef = sum(U[j, i] * b[j] for j in range(A.rows)) / S[i]
            for c in range(A.cols):
                w[c] += coef * V[i, c]
        if r < A.cols:  # S16: move along the null line towards the anchor weights
            for i in range(r, A.cols):
                t = sum(V[i, c] * (mp.mpf(_S16_ANCHOR[classes[c]]) - w[c])
                        for c in range(A.cols))
                for c in range(A.cols):
                    w[c] += t * V[i, c]
        x = _levels(N, mu1)
        wc = {cl: w[i] for i, cl in enumerate(classes)}
        om0 = [(x[a - 1], x[b - 1], x[c - 1]) for (a, b, c) in pts]
        w0 = [wc[tuple(sorted((a, b, c)))] * mp.pi / 2 for (a, b, c) in pts]
        om, ww = [], []
        for o in range(8):
            sx = -1 if o & 1 else 1
            sy = -1 if o & 2 else 1
            sz = -1 if o & 4 else 1
            for (m, e, xi), wp in zip(om0, w0):
                om.append((float(sx * m), float(sy * e), float(sz * xi)))
                ww.append(float(wp))
        return np.array(om, dtype=np.float64), np.array(ww, dtype=np.float64)


def lqn(N):
    """(omega [N(N+2), 3], w [N(N+2)]) of the level-symmetric set S_N."""
    om, w = _lqn_cached(int(N))
    return om.copy(), w.copy()


def class_weights(N):
    """Per-point octant-normalised weight of each class, keyed by the sorted
    1-based level triple (for comparison with published tables)."""
    om, w = lqn(N)
    pts = octant_points(N)
    out = {}
    for p, wp in zip(pts, w[: len(pts)]):
        out[tuple(sorted(p))] = wp / (np.pi / 2)
    return out
