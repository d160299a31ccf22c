/*
 * Plain FP64 CPU oracle for the discrete-ordinates source-iteration step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or helper with the HIP library; the two agree only because
 * both follow the paper.
 *
 * What it computes (paper section II.A, eqs. 1-7; section II.B, eqs. 8-22):
 *   - multigroup discrete-ordinates equation (eq. 2) on a uniform i,j,k voxel
 *     mesh with vacuum boundaries, diamond-difference (DD) cells (named in
 *     section IV), source iteration inside each group, downscatter between
 *     groups;
 *   - the first-collision-source split (eqs. 4-7): the uncollided fluence is
 *     traced along straight rays from the point source (exact path lengths),
 *     its first-collision source drives the collided S_N solve;
 *   - scalar fluence by the quadrature sum of eq. 3, generalised to the
 *     Legendre moments needed by a P_L scattering kernel;
 *   - the sub-sweep (hyperplane) plane sizes of eqs. 9-22 and the voxel
 *     enumeration of Table 1, used as an alternative sweep order;
 *   - the adjoint of the converged discrete solve and the gradient of a
 *     linear fluence functional with respect to per-voxel density.
 *
 * The paper does not fix the quadrature set, the DD negative-flux fixup, the
 * iteration criterion or the anisotropic first-collision source; the readings
 * taken here are stated at each function.  Parity unpinned: none (every
 * exported function is pinned by a CPU test against analytic values, a brute
 * force dense solve, a library routine or finite differences).
 *
 * Deliberately plain: no blocking, no fusion.  The only parallelism is an
 * OpenMP loop over the eight octants (each with its own moment accumulator,
 * summed in fixed octant order, so results do not depend on the thread
 * count) and over independent rays in the ray trace.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MEM 3
#define ORC_ERR_NOT_CONVERGED 5

#define ORC_LMAX 15

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;             /* cm */
    const uint8_t *material;       /* [V], v = i + nx*(j + ny*k) */
    const double *density;         /* [V] or NULL (all ones) */
    int n_mat, G;
    const double *sigma_t;         /* [n_mat][G]  cm^-1, g = 0 highest energy */
    int L;
    const double *sigma_s;         /* [n_mat][L+1][G (to)][G (from)]          */
    int n_dir;
    const double *omega;           /* [n_dir][3] unit directions               */
    const double *w;               /* [n_dir] weights, sum 4 pi                */
    int fixup;                     /* 0 pure DD, 1 set-to-zero                 */
} orc_problem;

typedef struct {
    double pos[3], axis[3], half_angle;  /* half_angle >= pi: isotropic point */
    const double *spectrum;              /* [G] photons per source particle   */
    const double *q_vol;                 /* [G][V] volumetric isotropic source
                                            (test hook) or NULL              */
    double fan_normal[3];                /* fan beam: normal of its plane     */
    double fan_half_thickness;           /* > 0: fan beam, half_angle in the
                                            plane; 0: cone                   */
} orc_source;

typedef struct {
    double tol;
    int max_iters;
    const int *fixed_iters;        /* [G] exact iteration counts, or NULL      */
    int sweep_order;               /* 0 nested upwind loops, 1 sub-sweep planes */
    int verbose;                   /* 1: a line on stderr as each group ends    */
    int stop_rule;                 /* forward groups: 0 relative L2 change of
                                      phi_00 < tol; 1 estimated pointwise error
                                      < tol (see group_si).  Adjoint: 0.      */
    int cell_single;               /* forward solve without the fixup: 1 runs
                                      every DD cell in single precision
                                      (CELL_DD_SINGLE), a model of that
                                      rounding; moments stay double          */
} orc_opts;

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for later calls (n >= 1); results do not depend on it. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics (Schmidt semi-normalised, no Condon-Shortley     */
/* phase, polar axis z, azimuth atan2(eta, mu)), index lm = l*l + l + m.     */
/* With this normalisation P_l(W.W') = sum_m R_lm(W) R_lm(W') (addition      */
/* theorem), which is how the Legendre kernel of eq. 1 enters in moments.    */
/* ------------------------------------------------------------------------ */
void orc_harmonics(int L, double mu, double eta, double xi, double *R)
{
    double P[ORC_LMAX + 1][ORC_LMAX + 1];
    double s = sqrt(mu * mu + eta * eta);
    double phi = atan2(eta, mu);
    P[0][0] = 1.0;
    for (int m = 1; m <= L; ++m) P[m][m] = (2.0 * m - 1.0) * s * P[m - 1][m - 1];
    for (int m = 0; m < L; ++m) P[m + 1][m] = (2.0 * m + 1.0) * xi * P[m][m];
    for (int m = 0; m <= L; ++m)
        for (int l = m + 2; l <= L; ++l)
            P[l][m] = ((2.0 * l - 1.0) * xi * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
    for (int l = 0; l <= L; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double ratio = 1.0;  /* (l-|m|)! / (l+|m|)! */
            for (int t = l - am + 1; t <= l + am; ++t) ratio /= (double)t;
            double norm = sqrt((am == 0 ? 1.0 : 2.0) * ratio);
            double ang = m >= 0 ? cos(m * phi) : sin(am * phi);
            R[l * l + l + m] = norm * P[l][am] * ang;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Sub-sweeps (section II.B).  Plane S of an nx*ny*nz mesh holds the voxels   */
/* with ix+iy+iz = S inside the bounds of eq. 8; its size is eq. 9 built from */
/* the triangular numbers of eqs. 10-22.                                      */
/* ------------------------------------------------------------------------ */
static long tri(long d) { return d * (d + 1) / 2; }
static long pos0(long a) { return a > 0 ? a : 0; }

long orc_plane_count(int S, int nx, int ny, int nz)
{
    long Cs = (long)(S + 1) * (S + 2) / 2;                       /* eq. 10 */
    long Lx = tri(pos0(S + 1 - nx));                             /* eqs. 11, 17 */
    long Ly = tri(pos0(S + 1 - ny));                             /* eqs. 12, 18 */
    long Lz = tri(pos0(S + 1 - nz));                             /* eqs. 13, 19 */
    long Gxy = tri(pos0(S + 1 - nx - ny));                       /* eqs. 14, 20 */
    long Gyz = tri(pos0(S + 1 - ny - nz));                       /* eqs. 15, 21 */
    long Gxz = tri(pos0(S + 1 - nx - nz));                       /* eqs. 16, 22 */
    return Cs - Lx - Ly - Lz + Gxy + Gyz + Gxz;                  /* eq. 9 */
}

/* Voxels of plane S in the order of Table 1: ix descending, then iy
 * descending (iz = S - ix - iy).  Writes 3 ints per voxel, returns count. */
long orc_plane_enumerate(int S, int nx, int ny, int nz, int *ijk)
{
    long c = 0;
    for (int ix = S; ix >= 0; --ix) {
        for (int iy = S - ix; iy >= 0; --iy) {
            int iz = S - ix - iy;
            if (ix < nx && iy < ny && iz < nz) {
                if (ijk) { ijk[3 * c] = ix; ijk[3 * c + 1] = iy; ijk[3 * c + 2] = iz; }
                ++c;
            }
        }
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Diamond-difference cell.  Balance with the DD closure psi_out = 2 psi -    */
/* psi_in on each axis, c_a = 2|Omega_a| / Delta_a.  Optional set-to-zero     */
/* fixup: an axis whose outflow goes negative gets psi_out = 0 and the cell   */
/* balance is re-solved, at most three passes.  Returns psi.                  */
/*                                                                            */
/* Cell modes:                                                                */
/*  CELL_DD      pure diamond difference                                      */
/*  CELL_FIXUP   with the fixup; if mask is given, the set of fixed axes is   */
/*               recorded there (bit a set: axis a fixed)                     */
/*  CELL_FROZEN  the fixup's cell with the fixed set read from mask: a linear */
/*               map of (q, inflows), equal to CELL_FIXUP where that set was  */
/*               recorded                                                     */
/*  CELL_TRANS   the transpose of the CELL_FROZEN cell, in the face variables */
/*               of a sweep along -Omega: psi = (q + sum_{a free} c_a in_a) / */
/*               (sig + sum_{a free} c_a), out_a = 2 psi - in_a on free axes  */
/*               and psi on fixed ones.  (Reverse-mode differentiation of the */
/*               frozen cell with the adjoint face values scaled by 2/c_a.)   */
/* ------------------------------------------------------------------------ */
enum { CELL_DD = 0, CELL_FIXUP = 1, CELL_FROZEN = 2, CELL_TRANS = 3, CELL_DD_SINGLE = 4 };

/* CELL_DD_SINGLE: the pure DD cell evaluated in IEEE single precision (the
 * source, cross section, coefficients and inflows rounded to float first,
 * every operation in float), a model of what single-precision rounding does
 * to the solve; the result and outflows are floats held in doubles. */
static double dd_cell_single(double q, double sig, const double c[3], const double in[3], double out[3])
{
    const float c0 = (float)c[0], c1 = (float)c[1], c2 = (float)c[2];
    const float i0 = (float)in[0], i1 = (float)in[1], i2 = (float)in[2];
    float num = (float)q;
    num = num + c0 * i0;
    num = num + c1 * i1;
    num = num + c2 * i2;
    float den = (float)sig;
    den = den + c0;
    den = den + c1;
    den = den + c2;
    const float psi = num / den;
    out[0] = (double)(2.0f * psi - i0);
    out[1] = (double)(2.0f * psi - i1);
    out[2] = (double)(2.0f * psi - i2);
    return (double)psi;
}

/* the cell with the axes in `fixed` (bit a) fixed */
static double dd_cell_fixed(double q, double sig, const double c[3], const double in[3], int fixed,
                            double out[3])
{
    double num = q, den = sig;
    for (int a = 0; a < 3; ++a) {
        if (fixed >> a & 1) num += 0.5 * c[a] * in[a];
        else { num += c[a] * in[a]; den += c[a]; }
    }
    double psi = num / den;
    for (int a = 0; a < 3; ++a) out[a] = (fixed >> a & 1) ? 0.0 : 2.0 * psi - in[a];
    return psi;
}

static double dd_cell(double q, double sig, const double c[3], const double in[3],
                      int mode, unsigned char *mask, double out[3], long *nneg)
{
    if (mode == CELL_TRANS) {
        const int fixed = *mask;
        double num = q, den = sig;
        for (int a = 0; a < 3; ++a)
            if (!(fixed >> a & 1)) { num += c[a] * in[a]; den += c[a]; }
        double psi = num / den;
        for (int a = 0; a < 3; ++a) out[a] = (fixed >> a & 1) ? psi : 2.0 * psi - in[a];
        return psi;
    }
    if (mode == CELL_DD_SINGLE) return dd_cell_single(q, sig, c, in, out);
    if (mode == CELL_FROZEN && *mask) return dd_cell_fixed(q, sig, c, in, *mask, out);
    double psi = (q + c[0] * in[0] + c[1] * in[1] + c[2] * in[2]) / (sig + c[0] + c[1] + c[2]);
    for (int a = 0; a < 3; ++a) out[a] = 2.0 * psi - in[a];
    if (mode == CELL_FROZEN) return psi;
    if (out[0] < 0.0 || out[1] < 0.0 || out[2] < 0.0) ++*nneg;
    int fixed = 0;
    if (mode == CELL_FIXUP) {
        for (int pass = 0; pass < 3; ++pass) {
            int grew = 0;
            for (int a = 0; a < 3; ++a)
                if (!(fixed >> a & 1) && out[a] < 0.0) { fixed |= 1 << a; grew = 1; }
            if (!grew) break;
            psi = dd_cell_fixed(q, sig, c, in, fixed, out);
        }
        if (mask) *mask = (unsigned char)fixed;
    }
    return psi;
}

/* One transport sweep of direction omega over the whole mesh: psi = T^-1 Q
 * with vacuum inflow on every face.  sig[v] is the total cross section of the
 * voxel (density already applied).  oxyz (optional) receives the outflow on
 * the downwind x, y and z faces of every voxel ([3][V]).  Upwind neighbours
 * are always visited first, in either order. */
static void sweep_dir(const orc_problem *p, const double om[3], const double *sig,
                      const double *Q, double *psi, double *ox, double *oy, double *oz,
                      int order, int mode, unsigned char *mask, long *nneg)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    const double c[3] = {2.0 * fabs(om[0]) / p->dx, 2.0 * fabs(om[1]) / p->dy, 2.0 * fabs(om[2]) / p->dz};
    const int sx = om[0] > 0 ? 1 : -1, sy = om[1] > 0 ? 1 : -1, sz = om[2] > 0 ? 1 : -1;
    long cnt = 0;
#define VISIT(i, j, k)                                                                 \
    do {                                                                               \
        long v_ = (long)(i) + (long)nx * ((j) + (long)ny * (k));                       \
        double in_[3], out_[3];                                                        \
        int iu_ = (i) - sx, ju_ = (j) - sy, ku_ = (k) - sz;                            \
        in_[0] = (iu_ >= 0 && iu_ < nx) ? ox[v_ - sx] : 0.0;                           \
        in_[1] = (ju_ >= 0 && ju_ < ny) ? oy[v_ - (long)sy * nx] : 0.0;                \
        in_[2] = (ku_ >= 0 && ku_ < nz) ? oz[v_ - (long)sz * nx * ny] : 0.0;           \
        psi[v_] = dd_cell(Q[v_], sig[v_], c, in_, mode, mask ? mask + v_ : NULL, out_, &cnt); \
        ox[v_] = out_[0]; oy[v_] = out_[1]; oz[v_] = out_[2];                          \
    } while (0)
    if (order == 0) {
        for (int kk = 0; kk < nz; ++kk) {
            int k = sz > 0 ? kk : nz - 1 - kk;
            for (int jj = 0; jj < ny; ++jj) {
                int j = sy > 0 ? jj : ny - 1 - jj;
                for (int ii = 0; ii < nx; ++ii) {
                    int i = sx > 0 ? ii : nx - 1 - ii;
                    VISIT(i, j, k);
                }
            }
        }
    } else {
        /* the paper's sub-sweeps: plane S (octant-relative indices) in the
         * voxel order of Table 1 */
        int *ijk = (int *)malloc(sizeof(int) * 3 * (size_t)nx * ny * nz);
        for (int S = 0; S <= nx + ny + nz - 3; ++S) {
            long n = orc_plane_enumerate(S, nx, ny, nz, ijk);
            for (long t = 0; t < n; ++t) {
                int ir = ijk[3 * t], jr = ijk[3 * t + 1], kr = ijk[3 * t + 2];
                int i = sx > 0 ? ir : nx - 1 - ir;
                int j = sy > 0 ? jr : ny - 1 - jr;
                int k = sz > 0 ? kr : nz - 1 - kr;
                VISIT(i, j, k);
            }
        }
        free(ijk);
    }
#undef VISIT
    if (nneg) *nneg += cnt;
}

/* Exported single sweep, for tests (DD transpose, sweep order, balance). */
int orc_sweep(const orc_problem *p, const double om[3], const double *sig, const double *Q,
              double *psi, double *oxyz, int order, long *nneg)
{
    long V = (long)p->nx * p->ny * p->nz;
    double *o = oxyz ? oxyz : (double *)malloc(sizeof(double) * 3 * V);
    if (!o) return ORC_ERR_MEM;
    long cnt = 0;
    sweep_dir(p, om, sig, Q, psi, o, o + V, o + 2 * V, order, p->fixup ? CELL_FIXUP : CELL_DD, NULL, &cnt);
    if (nneg) *nneg = cnt;
    if (!oxyz) free(o);
    return ORC_OK;
}

/* Exported single sweep with an explicit cell mode and fixed-axis mask [V]
 * (recorded by CELL_FIXUP, read by CELL_FROZEN and CELL_TRANS), for tests. */
int orc_sweep_mode(const orc_problem *p, const double om[3], const double *sig, const double *Q,
                   double *psi, double *oxyz, int mode, unsigned char *mask)
{
    long V = (long)p->nx * p->ny * p->nz;
    if (mode < CELL_DD || mode > CELL_DD_SINGLE || ((mode == CELL_FROZEN || mode == CELL_TRANS) && !mask))
        return ORC_ERR_ARG;
    double *o = oxyz ? oxyz : (double *)malloc(sizeof(double) * 3 * V);
    if (!o) return ORC_ERR_MEM;
    long cnt = 0;
    sweep_dir(p, om, sig, Q, psi, o, o + V, o + 2 * V, 0, mode, mask, &cnt);
    if (!oxyz) free(o);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Ray tracing for the uncollided fluence (eq. 4 without scattering has the   */
/* closed solution exp(-tau)/(4 pi r^2) along the straight path).  Exact      */
/* path lengths through the voxel grid: all parametric crossings of the      */
/* segment xs -> xe with the grid planes, merged in increasing order; each    */
/* piece is charged to the voxel holding its midpoint (outside = vacuum).     */
/* Accumulates rho*length per material into lam[n_mat].                       */
/* ------------------------------------------------------------------------ */
static int axis_crossings(double a0, double a1, double d, int n, double *out)
{
    int c = 0;
    double da = a1 - a0;
    if (da == 0.0) return 0;
    if (da > 0) {
        for (int q = 0; q <= n; ++q) {
            double al = (q * d - a0) / da;
            if (al > 0.0 && al < 1.0) out[c++] = al;
        }
    } else {
        for (int q = n; q >= 0; --q) {
            double al = (q * d - a0) / da;
            if (al > 0.0 && al < 1.0) out[c++] = al;
        }
    }
    return c;
}

void orc_ray_material_path(const orc_problem *p, const double xs[3], const double xe[3], double *lam)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    int cap = nx + ny + nz + 8;
    double *ax = (double *)malloc(sizeof(double) * 4 * (size_t)cap);
    double *ay = ax + cap, *az = ay + cap, *all = az + cap;
    int cx = axis_crossings(xs[0], xe[0], p->dx, nx, ax);
    int cy = axis_crossings(xs[1], xe[1], p->dy, ny, ay);
    int cz = axis_crossings(xs[2], xe[2], p->dz, nz, az);
    /* three-way merge of increasing lists, bracketed by 0 and 1 */
    int n = 0, a = 0, b = 0, e = 0;
    all[n++] = 0.0;
    while (a < cx || b < cy || e < cz) {
        double va = a < cx ? ax[a] : 2.0, vb = b < cy ? ay[b] : 2.0, ve = e < cz ? az[e] : 2.0;
        if (va <= vb && va <= ve) all[n++] = ax[a++];
        else if (vb <= ve) all[n++] = ay[b++];
        else all[n++] = az[e++];
    }
    all[n++] = 1.0;
    double r = sqrt((xe[0] - xs[0]) * (xe[0] - xs[0]) + (xe[1] - xs[1]) * (xe[1] - xs[1]) +
                    (xe[2] - xs[2]) * (xe[2] - xs[2]));
    for (int m = 0; m < p->n_mat; ++m) lam[m] = 0.0;
    for (int t = 0; t + 1 < n; ++t) {
        double a0 = all[t], a1 = all[t + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        double px = xs[0] + am * (xe[0] - xs[0]);
        double py = xs[1] + am * (xe[1] - xs[1]);
        double pz = xs[2] + am * (xe[2] - xs[2]);
        int i = (int)floor(px / p->dx), j = (int)floor(py / p->dy), k = (int)floor(pz / p->dz);
        if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) continue;
        long v = (long)i + (long)nx * (j + (long)ny * k);
        double rho = p->density ? p->density[v] : 1.0;
        lam[p->material[v]] += rho * (a1 - a0) * r;
    }
    free(ax);
}

/* Calls fn(v, length) for every voxel piece along xs -> xe (used by the
 * gradient back-projection). */
static void ray_visit(const orc_problem *p, const double xs[3], const double xe[3],
                      void (*fn)(void *, long, double), void *ctx)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz;
    int cap = nx + ny + nz + 8;
    double *ax = (double *)malloc(sizeof(double) * 4 * (size_t)cap);
    double *ay = ax + cap, *az = ay + cap, *all = az + cap;
    int cx = axis_crossings(xs[0], xe[0], p->dx, nx, ax);
    int cy = axis_crossings(xs[1], xe[1], p->dy, ny, ay);
    int cz = axis_crossings(xs[2], xe[2], p->dz, nz, az);
    int n = 0, a = 0, b = 0, e = 0;
    all[n++] = 0.0;
    while (a < cx || b < cy || e < cz) {
        double va = a < cx ? ax[a] : 2.0, vb = b < cy ? ay[b] : 2.0, ve = e < cz ? az[e] : 2.0;
        if (va <= vb && va <= ve) all[n++] = ax[a++];
        else if (vb <= ve) all[n++] = ay[b++];
        else all[n++] = az[e++];
    }
    all[n++] = 1.0;
    double r = sqrt((xe[0] - xs[0]) * (xe[0] - xs[0]) + (xe[1] - xs[1]) * (xe[1] - xs[1]) +
                    (xe[2] - xs[2]) * (xe[2] - xs[2]));
    for (int t = 0; t + 1 < n; ++t) {
        double a0 = all[t], a1 = all[t + 1];
        if (!(a1 > a0)) continue;
        double am = 0.5 * (a0 + a1);
        int i = (int)floor((xs[0] + am * (xe[0] - xs[0])) / p->dx);
        int j = (int)floor((xs[1] + am * (xe[1] - xs[1])) / p->dy);
        int k = (int)floor((xs[2] + am * (xe[2] - xs[2])) / p->dz);
        if (i < 0 || i >= nx || j < 0 || j >= ny || k < 0 || k >= nz) continue;
        fn(ctx, (long)i + (long)nx * (j + (long)ny * k), (a1 - a0) * r);
    }
    free(ax);
}

/* Uncollided fluence of one point/cone/fan source at every voxel centre, per
 * group, and the unit direction source -> voxel.  Voxel centre of (i,j,k) is
 * ((i+1/2)dx, (j+1/2)dy, (k+1/2)dz).  The cone holds the voxels whose
 * direction makes an angle <= half_angle with the axis (inclusive); inside it
 * the source emits spectrum[g]/(4 pi) per steradian.  A fan: in the frame
 * e1 = axis, e3 = the fan normal made orthogonal to e1, e2 = e3 x e1, the
 * direction's elevation asin(d.e3 / r) is within +-fan_half_thickness and its
 * in-plane angle atan2(|d.e2|, d.e1) at most half_angle. */
static int in_fan(const orc_source *s, const double d[3], double r)
{
    double e1[3], e2[3], e3[3];
    double an = sqrt(s->axis[0] * s->axis[0] + s->axis[1] * s->axis[1] + s->axis[2] * s->axis[2]);
    for (int t = 0; t < 3; ++t) e1[t] = s->axis[t] / an;
    double na = s->fan_normal[0] * e1[0] + s->fan_normal[1] * e1[1] + s->fan_normal[2] * e1[2];
    for (int t = 0; t < 3; ++t) e3[t] = s->fan_normal[t] - na * e1[t];
    double l = sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
    for (int t = 0; t < 3; ++t) e3[t] /= l;
    e2[0] = e3[1] * e1[2] - e3[2] * e1[1];
    e2[1] = e3[2] * e1[0] - e3[0] * e1[2];
    e2[2] = e3[0] * e1[1] - e3[1] * e1[0];
    double x = d[0] * e1[0] + d[1] * e1[1] + d[2] * e1[2];
    double y = d[0] * e2[0] + d[1] * e2[1] + d[2] * e2[2];
    double z = d[0] * e3[0] + d[1] * e3[1] + d[2] * e3[2];
    double elev = asin(fmin(1.0, fmax(-1.0, z / r)));
    return fabs(elev) <= s->fan_half_thickness && atan2(fabs(y), x) <= s->half_angle;
}

int orc_raytrace(const orc_problem *p, const orc_source *s, double *phi_u, double *omega_s)
{
    const int nx = p->nx, ny = p->ny, nz = p->nz, G = p->G;
    const long V = (long)nx * ny * nz;
    double mind = p->dx < p->dy ? p->dx : p->dy;
    if (p->dz < mind) mind = p->dz;
    double an = sqrt(s->axis[0] * s->axis[0] + s->axis[1] * s->axis[1] + s->axis[2] * s->axis[2]);
    int iso = s->half_angle >= M_PI;
    if (!iso && !(an > 0.0)) return ORC_ERR_ARG;
    double cosh_ = cos(s->half_angle);
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (long v = 0; v < V; ++v) {
        int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((long)nx * ny));
        double c[3] = {(i + 0.5) * p->dx, (j + 0.5) * p->dy, (k + 0.5) * p->dz};
        double d[3] = {c[0] - s->pos[0], c[1] - s->pos[1], c[2] - s->pos[2]};
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        if (r < 1e-6 * mind) { bad = 1; continue; }
        if (omega_s) { omega_s[3 * v] = d[0] / r; omega_s[3 * v + 1] = d[1] / r; omega_s[3 * v + 2] = d[2] / r; }
        int inside = iso || (s->fan_half_thickness > 0.0
                                 ? in_fan(s, d, r)
                                 : (d[0] * s->axis[0] + d[1] * s->axis[1] + d[2] * s->axis[2]) >= r * an * cosh_);
        if (!inside) {
            for (int g = 0; g < G; ++g) phi_u[(long)g * V + v] = 0.0;
            continue;
        }
        double lam[256];
        orc_ray_material_path(p, s->pos, c, lam);
        for (int g = 0; g < G; ++g) {
            double tau = 0.0;
            for (int m = 0; m < p->n_mat; ++m) tau += p->sigma_t[m * G + g] * lam[m];
            phi_u[(long)g * V + v] = s->spectrum[g] * exp(-tau) / (4.0 * M_PI * r * r);
        }
    }
    return bad ? ORC_ERR_ARG : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Moment <-> direction matrices.  Scattering source of eq. 2 in moment form: */
/*   Q_n = sum_lm (2l+1)/(4 pi) R_lm(W_n) S_lm,   S_lm = sigma_{s,l} phi_lm,  */
/*   phi_lm = sum_n w_n R_lm(W_n) psi_n  (eq. 3 is the lm = 00 row).          */
/* By the addition theorem this equals the direct sum over n' in eq. 2.       */
/* ------------------------------------------------------------------------ */
static void build_md(const orc_problem *p, double *M, double *D)
{
    int Nm = (p->L + 1) * (p->L + 1);
    double R[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
    for (int n = 0; n < p->n_dir; ++n) {
        orc_harmonics(p->L, p->omega[3 * n], p->omega[3 * n + 1], p->omega[3 * n + 2], R);
        for (int l = 0; l <= p->L; ++l)
            for (int m = -l; m <= l; ++m) {
                int lm = l * l + l + m;
                M[(long)n * Nm + lm] = (2.0 * l + 1.0) / (4.0 * M_PI) * R[lm];
                D[(long)lm * p->n_dir + n] = p->w[n] * R[lm];
            }
    }
}

void orc_moment_matrices(const orc_problem *p, double *M, double *D) { build_md(p, M, D); }

static int octant_of(const double om[3])
{
    return (om[0] < 0 ? 1 : 0) | (om[1] < 0 ? 2 : 0) | (om[2] < 0 ? 4 : 0);
}

/* One source iteration sweep of all directions: Q_n from the moments S,
 * sweep each direction, accumulate the new moments.  Direction order inside
 * an octant is the caller's order; octants are summed in order 0..7.
 * If reverse != 0 every direction is swept along -Omega_n (adjoint).  If
 * psi_keep is not NULL the angular fluence of every direction is stored
 * ([n_dir][V]).  mode is the cell mode; masks ([n_dir][V], or NULL) the
 * fixed-axis sets it records or reads. */
static int sweep_all(const orc_problem *p, const double *M, const double *D, const double *sig,
                     const double *S, double *phi_new, int order, int reverse,
                     double *psi_keep, long *nneg_total, int mode, unsigned char *masks)
{
    const long V = (long)p->nx * p->ny * p->nz;
    const int Nm = (p->L + 1) * (p->L + 1), Nd = p->n_dir;
    double *part = (double *)calloc((size_t)8 * Nm * V, sizeof(double));
    if (!part) return ORC_ERR_MEM;
    int fail = 0;
    long nneg = 0;
#pragma omp parallel for schedule(static, 1) reduction(| : fail) reduction(+ : nneg)
    for (int o = 0; o < 8; ++o) {
        double *Q = (double *)malloc(sizeof(double) * 5 * V);
        if (!Q) { fail = 1; continue; }
        double *psi = Q + V, *ox = psi + V, *oy = ox + V, *oz = oy + V;
        double *acc = part + (long)o * Nm * V;
        for (int n = 0; n < Nd; ++n) {
            const double *om = p->omega + 3 * n;
            if (octant_of(om) != o) continue;
            for (long v = 0; v < V; ++v) {
                double q = 0.0;
                for (int lm = 0; lm < Nm; ++lm) q += M[(long)n * Nm + lm] * S[(long)lm * V + v];
                Q[v] = q;
            }
            double omr[3] = {om[0], om[1], om[2]};
            if (reverse) { omr[0] = -om[0]; omr[1] = -om[1]; omr[2] = -om[2]; }
            long c = 0;
            sweep_dir(p, omr, sig, Q, psi, ox, oy, oz, order, mode, masks ? masks + (long)n * V : NULL, &c);
            nneg += c;
            if (psi_keep) memcpy(psi_keep + (long)n * V, psi, sizeof(double) * V);
            for (int lm = 0; lm < Nm; ++lm) {
                double dn = D[(long)lm * Nd + n];
                double *a = acc + (long)lm * V;
                for (long v = 0; v < V; ++v) a[v] += dn * psi[v];
            }
        }
        free(Q);
    }
    if (fail) { free(part); return ORC_ERR_MEM; }
    for (long x = 0; x < (long)Nm * V; ++x) {
        double s = 0.0;
        for (int o = 0; o < 8; ++o) s += part[(long)o * Nm * V + x];
        phi_new[x] = s;
    }
    free(part);
    if (nneg_total) *nneg_total += nneg;
    return ORC_OK;
}

static double relchange(const double *a_new, const double *a_old, long V)
{
    double num = 0.0, den = 0.0;
    for (long v = 0; v < V; ++v) {
        double d = a_new[v] - a_old[v];
        num += d * d;
        den += a_new[v] * a_new[v];
    }
    if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
    return sqrt(num) / sqrt(den);
}

/* sigma_{s,l}^{g'->g} at material m */
static double sgs(const orc_problem *p, int m, int l, int g, int gp)
{
    const int G = p->G;
    return p->sigma_s[(((long)m * (p->L + 1) + l) * G + g) * G + gp];
}

/* Source iteration in group g on the external moments F ([Nm][V]); result
 * moments in phi ([Nm][V], zero initial guess).  Returns the status and
 * writes iterations and final relative change. */
/* Stop rule 1: the largest change of phi_00 relative to the total scalar
 * fluence phi_u + phi_00, over the voxels whose total is at least 1e-6 of the
 * previous iterate's largest |total| (floor_ref).  Returns that change and
 * writes this iterate's largest |total| for the next call. */
static double pointwise_change(const double *phi_new, const double *phi_old, const double *phiu, long V,
                               double floor_ref, double *max_total)
{
    double d = 0.0, mx = 0.0;
    for (long v = 0; v < V; ++v) {
        double t = fabs((phiu ? phiu[v] : 0.0) + phi_new[v]);
        if (t > mx) mx = t;
        if (t > 0.0 && t >= 1e-6 * floor_ref) {
            double e = fabs(phi_new[v] - phi_old[v]) / t;
            if (e > d) d = e;
        }
    }
    *max_total = mx;
    return d;
}

/* Source iteration in group g.  rule: the stop rule (0 or 1, see orc_opts);
 * phiu_g: the group's uncollided fluence (rule 1; NULL = zero). */
static int group_si(const orc_problem *p, const orc_opts *o, int g, const double *M, const double *D,
                    const double *sig, const double *F, double *phi, int reverse, int *iters,
                    double *resid, long *nneg, int mode, unsigned char *masks, int rule, const double *phiu_g)
{
    const long V = (long)p->nx * p->ny * p->nz;
    const int Nm = (p->L + 1) * (p->L + 1);
    double *S = (double *)malloc(sizeof(double) * 2 * Nm * V);
    if (!S) return ORC_ERR_MEM;
    double *phin = S + (long)Nm * V;
    memset(phi, 0, sizeof(double) * Nm * V);
    int it = 0, st = ORC_OK;
    double r = 0.0;
    int target = o->fixed_iters ? o->fixed_iters[g] : -1;
    /* rule 1 state: largest |total| of the current iterate (not needed for
     * the first change, which never stops the iteration) and the previous L2
     * change */
    double mtot = 0.0, r_prev = 0.0;
    while (1) {
        if (target >= 0 && it >= target) break;
        for (int l = 0; l <= p->L; ++l)
            for (int m = -l; m <= l; ++m) {
                int lm = l * l + l + m;
                for (long v = 0; v < V; ++v) {
                    double rho = p->density ? p->density[v] : 1.0;
                    S[(long)lm * V + v] = F[(long)lm * V + v] +
                                          rho * sgs(p, p->material[v], l, g, g) * phi[(long)lm * V + v];
                }
            }
        int e = sweep_all(p, M, D, sig, S, phin, o->sweep_order, reverse, NULL, nneg, mode, masks);
        if (e) { st = e; break; }
        r = relchange(phin, phi, V);
        double mnew = 0.0;
        double d = rule == 1 ? pointwise_change(phin, phi, phiu_g, V, mtot, &mnew) : 0.0;
        memcpy(phi, phin, sizeof(double) * Nm * V);
        ++it;
        if (target >= 0) continue;
        if (rule == 1) {
            /* the iteration shrinks the change by about rho per step, so the
             * error left after this step is about d rho / (1 - rho) */
            double rho = (it >= 2 && r_prev > 0.0) ? r / r_prev : 1.0;
            double est = rho < 1.0 ? d * rho / (1.0 - rho) : INFINITY;
            if (o->verbose >= 2)
                fprintf(stderr, "oracle: g %d it %d r %.3e d %.3e rho %.4f est %.3e\n", g, it, r, d, rho, est);
            mtot = mnew;
            r_prev = r;
            if (r == 0.0 || est < o->tol) break;
        } else if (r < o->tol) break;
        if (it >= o->max_iters) { st = ORC_ERR_NOT_CONVERGED; break; }
    }
    free(S);
    if (iters) iters[g] = it;
    if (resid) resid[g] = r;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Forward solve of one source (eqs. 2-7).                                    */
/*  phi_total [G][V] = phi_u + collided scalar fluence (required)             */
/*  phi_u     [G][V] uncollided (optional)                                    */
/*  phi_c     [G][Nm][V] collided moments (optional)                          */
/* Groups are solved in order g = 0 (highest energy) .. G-1; group g gets the */
/* downscatter of every converged group g' < g.                               */
/* ------------------------------------------------------------------------ */
static void group_source(const orc_problem *p, int g, const orc_source *s, const double *phiu,
                         const double *oms, const double *phic_all, double *F)
{
    const long V = (long)p->nx * p->ny * p->nz;
    const int Nm = (p->L + 1) * (p->L + 1), G = p->G;
    double R[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
    for (long v = 0; v < V; ++v) {
        int m = p->material[v];
        double rho = p->density ? p->density[v] : 1.0;
        /* first-collision source (eq. 5): the uncollided angular fluence is a
         * delta in the direction source -> voxel, so its moments are
         * phi_u * R_lm(Omega_s) */
        if (oms) orc_harmonics(p->L, oms[3 * v], oms[3 * v + 1], oms[3 * v + 2], R);
        for (int l = 0; l <= p->L; ++l)
            for (int mm = -l; mm <= l; ++mm) {
                int lm = l * l + l + mm;
                double f = 0.0;
                if (oms)
                    for (int gp = 0; gp <= g; ++gp) f += sgs(p, m, l, g, gp) * phiu[(long)gp * V + v] * R[lm];
                for (int gp = 0; gp < g; ++gp)
                    f += sgs(p, m, l, g, gp) * phic_all[((long)gp * Nm + lm) * V + v];
                F[(long)lm * V + v] = rho * f;
            }
        if (s->q_vol) F[v] += s->q_vol[(long)g * V + v];
    }
    (void)G;
}

int orc_solve(const orc_problem *p, const orc_source *s, const orc_opts *o, double *phi_total,
              double *phi_u_out, double *phi_c_out, int *iters, double *resid, long *nneg)
{
    const long V = (long)p->nx * p->ny * p->nz;
    const int Nm = (p->L + 1) * (p->L + 1), G = p->G, Nd = p->n_dir;
    if (p->L > ORC_LMAX || p->n_mat > 256 || V <= 0) return ORC_ERR_ARG;
    if (o->cell_single && p->fixup) return ORC_ERR_ARG;  /* the single-precision model is pure DD */
    double *M = (double *)malloc(sizeof(double) * 2 * (size_t)Nd * Nm);
    double *phiu = (double *)calloc((size_t)G * V, sizeof(double));
    double *oms = s->q_vol ? NULL : (double *)malloc(sizeof(double) * 3 * V);
    double *phic = phi_c_out ? phi_c_out : (double *)malloc(sizeof(double) * (size_t)G * Nm * V);
    double *F = (double *)malloc(sizeof(double) * (size_t)Nm * V);
    double *sig = (double *)malloc(sizeof(double) * V);
    if (!M || !phiu || (!oms && !s->q_vol) || !phic || !F || !sig) return ORC_ERR_MEM;
    double *D = M + (long)Nd * Nm;
    build_md(p, M, D);
    int st = ORC_OK;
    if (!s->q_vol) st = orc_raytrace(p, s, phiu, oms);
    if (nneg) *nneg = 0;
    for (int g = 0; g < G && (st == ORC_OK || st == ORC_ERR_NOT_CONVERGED); ++g) {
        for (long v = 0; v < V; ++v)
            sig[v] = (p->density ? p->density[v] : 1.0) * p->sigma_t[p->material[v] * G + g];
        group_source(p, g, s, phiu, oms, phic, F);
        int e = group_si(p, o, g, M, D, sig, F, phic + (long)g * Nm * V, 0, iters, resid, nneg,
                         p->fixup ? CELL_FIXUP : o->cell_single ? CELL_DD_SINGLE : CELL_DD, NULL, o->stop_rule,
                         s->q_vol ? NULL : phiu + (long)g * V);
        if (e == ORC_ERR_NOT_CONVERGED) st = e;
        else if (e) st = e;
        if (o->verbose) {
            fprintf(stderr, "oracle: group %d of %d done (%d source iterations)\n", g + 1, G, iters ? iters[g] : -1);
            fflush(stderr);
        }
    }
    for (int g = 0; g < G; ++g)
        for (long v = 0; v < V; ++v) {
            phi_total[(long)g * V + v] = phiu[(long)g * V + v] + phic[(long)g * Nm * V + v];
            if (phi_u_out) phi_u_out[(long)g * V + v] = phiu[(long)g * V + v];
        }
    free(M); free(phiu); free(oms); free(F); free(sig);
    if (!phi_c_out) free(phic);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the converged discrete forward solve and gradient              */
/* of J = sum_g sum_v W^g(v) phi_total^g(v) with respect to the per-voxel     */
/* density rho(v), which scales sigma_t and every sigma_{s,l} at v.           */
/*                                                                            */
/* Discrete adjoint: the transpose of the DD sweep along W equals the DD      */
/* sweep along -W with the same coefficients.  With the set-to-zero fixup    */
/* the forward solve is piecewise linear; it is linearised with every cell's */
/* set of fixed axes frozen at the converged forward solution (recorded by a */
/* forward sweep of each group from its converged moments), and the adjoint  */
/* sweep uses the transposed frozen cell (CELL_TRANS).  chi^g (adjoint        */
/* angular fluence, per unit weight) solves, for g = G-1 .. 0, source         */
/* iteration with                                                             */
/*   Qa_n = W^g + sum_lm M[n,lm] rho (sigma_{s,l}^{g->g} phia_lm^g            */
/*                              + sum_{g''>g} sigma_{s,l}^{g->g''} phia^g'')  */
/* swept along -W_n, phia_lm = sum_n w_n R_lm(W_n) chi_n.                     */
/* Gradient (collision, scattering and first-collision terms, then the ray   */
/* back-projection of the uncollided term):                                   */
/*   dJ/drho(v) = sum_g [ -sigma_t^g sum_n w_n chi_n psi_n                    */
/*     + sum_lm (2l+1)/(4pi) phia_lm^g sum_{g'<=g} sigma_{s,l}^{g'->g}        */
/*              (phic_lm^{g'} + phiu^{g'} R_lm(Omega_s)) ]                    */
/*     - sum_g sum_v' Gu^g(v') phiu^g(v') sigma_t^g[m(v)] len(v; ray to v')   */
/*   Gu^g(v') = W^g(v') + rho(v') sum_{g''>=g} sum_lm (2l+1)/(4pi)            */
/*              sigma_{s,l}^{g->g''} R_lm(Omega_s(v')) phia_lm^{g''}(v')      */
/* psi^g is recomputed by one forward sweep from the converged moments.      */
/* Also returns J and the reciprocity value <W,phiu> + sum w chi . M F_fc.    */
/* ------------------------------------------------------------------------ */
typedef struct { const orc_problem *p; double *grad; const double *B; } bp_ctx;
static void bp_fn(void *c_, long v, double len)
{
    bp_ctx *c = (bp_ctx *)c_;
    c->grad[v] -= c->B[c->p->material[v]] * len;
}

int orc_adjoint(const orc_problem *p, const orc_source *s, const orc_opts *o, const double *W,
                double *J_out, double *recip_out, double *grad, int *iters_fwd, int *iters_adj)
{
    const long V = (long)p->nx * p->ny * p->nz;
    const int Nm = (p->L + 1) * (p->L + 1), G = p->G, Nd = p->n_dir;
    const int fmode = p->fixup ? CELL_FIXUP : CELL_DD, amode = p->fixup ? CELL_TRANS : CELL_DD;
    unsigned char *masks = p->fixup ? (unsigned char *)malloc((size_t)Nd * V) : NULL;
    if (p->fixup && !masks) return ORC_ERR_MEM;
    double *phit = (double *)malloc(sizeof(double) * (size_t)G * V);
    double *phiu = (double *)malloc(sizeof(double) * (size_t)G * V);
    double *phic = (double *)malloc(sizeof(double) * (size_t)G * Nm * V);
    double *phia = (double *)malloc(sizeof(double) * (size_t)G * Nm * V);
    double *oms = (double *)malloc(sizeof(double) * 3 * V);
    double *M = (double *)malloc(sizeof(double) * 2 * (size_t)Nd * Nm);
    double *F = (double *)malloc(sizeof(double) * (size_t)Nm * V);
    double *Fa = (double *)malloc(sizeof(double) * (size_t)Nm * V);
    double *sig = (double *)malloc(sizeof(double) * V);
    double *psi = (double *)malloc(sizeof(double) * (size_t)Nd * V);
    double *chi = (double *)malloc(sizeof(double) * (size_t)Nd * V);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)Nm * V);
    if (!phit || !phiu || !phic || !phia || !oms || !M || !F || !Fa || !sig || !psi || !chi || !tmp)
        return ORC_ERR_MEM;
    double *D = M + (long)Nd * Nm;
    build_md(p, M, D);
    orc_source s2 = *s;
    s2.q_vol = NULL;
    int st = orc_solve(p, &s2, o, phit, phiu, phic, iters_fwd, NULL, NULL);
    if (st && st != ORC_ERR_NOT_CONVERGED) return st;
    orc_raytrace(p, &s2, phiu, oms);
    double J = 0.0;
    for (long x = 0; x < (long)G * V; ++x) J += W[x] * phit[x];
    *J_out = J;
    for (long v = 0; v < V; ++v) grad[v] = 0.0;
    double recip = 0.0;
    for (long x = 0; x < (long)G * V; ++x) recip += W[x] * phiu[x];
    double R[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
    /* adjoint groups, lowest energy first */
    for (int g = G - 1; g >= 0; --g) {
        for (long v = 0; v < V; ++v)
            sig[v] = (p->density ? p->density[v] : 1.0) * p->sigma_t[p->material[v] * G + g];
        /* adjoint external moments: W^g enters as an isotropic angular source
         * of unit intensity per direction, i.e. moment 00 equal to 4 pi W */
        for (int l = 0; l <= p->L; ++l)
            for (int mm = -l; mm <= l; ++mm) {
                int lm = l * l + l + mm;
                for (long v = 0; v < V; ++v) {
                    double rho = p->density ? p->density[v] : 1.0;
                    double f = 0.0;
                    for (int gpp = g + 1; gpp < G; ++gpp)
                        f += sgs(p, p->material[v], l, gpp, g) * phia[((long)gpp * Nm + lm) * V + v];
                    Fa[(long)lm * V + v] = rho * f;
                }
            }
        for (long v = 0; v < V; ++v) Fa[v] += 4.0 * M_PI * W[(long)g * V + v];
        if (masks) {
            /* fixed-axis sets of the converged forward solution of group g */
            group_source(p, g, &s2, phiu, oms, phic, F);
            for (int l = 0; l <= p->L; ++l)
                for (int mm = -l; mm <= l; ++mm) {
                    int lm = l * l + l + mm;
                    for (long v = 0; v < V; ++v) {
                        double rho = p->density ? p->density[v] : 1.0;
                        tmp[(long)lm * V + v] = F[(long)lm * V + v] +
                            rho * sgs(p, p->material[v], l, g, g) * phic[((long)g * Nm + lm) * V + v];
                    }
                }
            double *scratch = (double *)malloc(sizeof(double) * (size_t)Nm * V);
            if (!scratch) return ORC_ERR_MEM;
            sweep_all(p, M, D, sig, tmp, scratch, 0, 0, NULL, NULL, fmode, masks);
            free(scratch);
        }
        int e = group_si(p, o, g, M, D, sig, Fa, phia + (long)g * Nm * V, 1, iters_adj, NULL, NULL, amode, masks,
                         0, NULL);
        if (e && e != ORC_ERR_NOT_CONVERGED) return e;
    }
    for (int g = 0; g < G; ++g) {
        for (long v = 0; v < V; ++v)
            sig[v] = (p->density ? p->density[v] : 1.0) * p->sigma_t[p->material[v] * G + g];
        /* recompute psi^g from the converged moments, and chi^g from phia^g */
        group_source(p, g, &s2, phiu, oms, phic, F);
        for (int l = 0; l <= p->L; ++l)
            for (int mm = -l; mm <= l; ++mm) {
                int lm = l * l + l + mm;
                for (long v = 0; v < V; ++v) {
                    double rho = p->density ? p->density[v] : 1.0;
                    int m = p->material[v];
                    tmp[(long)lm * V + v] = F[(long)lm * V + v] + rho * sgs(p, m, l, g, g) * phic[((long)g * Nm + lm) * V + v];
                    double f = 0.0;
                    for (int gpp = g + 1; gpp < G; ++gpp)
                        f += sgs(p, m, l, gpp, g) * phia[((long)gpp * Nm + lm) * V + v];
                    Fa[(long)lm * V + v] = rho * (f + sgs(p, m, l, g, g) * phia[((long)g * Nm + lm) * V + v]);
                }
            }
        for (long v = 0; v < V; ++v) Fa[v] += 4.0 * M_PI * W[(long)g * V + v];
        double *scratch = (double *)malloc(sizeof(double) * (size_t)Nm * V);
        sweep_all(p, M, D, sig, tmp, scratch, 0, 0, psi, NULL, fmode, masks);
        sweep_all(p, M, D, sig, Fa, scratch, 0, 1, chi, NULL, amode, masks);
        free(scratch);
        /* reciprocity: <chi, M F_fc> with F_fc the first-collision part */
        for (long v = 0; v < V; ++v) {
            int m = p->material[v];
            double rho = p->density ? p->density[v] : 1.0;
            double ffc[(ORC_LMAX + 1) * (ORC_LMAX + 1)];
            orc_harmonics(p->L, oms[3 * v], oms[3 * v + 1], oms[3 * v + 2], R);
            for (int l = 0; l <= p->L; ++l)
                for (int mm = -l; mm <= l; ++mm) {
                    int lm = l * l + l + mm;
                    double f = 0.0;
                    for (int gp = 0; gp <= g; ++gp) f += sgs(p, m, l, g, gp) * phiu[(long)gp * V + v];
                    ffc[lm] = rho * f * R[lm];
                }
            for (int n = 0; n < Nd; ++n) {
                double q = 0.0;
                for (int lm = 0; lm < Nm; ++lm) q += M[(long)n * Nm + lm] * ffc[lm];
                recip += p->w[n] * chi[(long)n * V + v] * q;
            }
        }
        /* collision and scattering terms */
        for (long v = 0; v < V; ++v) {
            int m = p->material[v];
            double cw = 0.0;
            for (int n = 0; n < Nd; ++n) cw += p->w[n] * chi[(long)n * V + v] * psi[(long)n * V + v];
            double gv = -p->sigma_t[m * G + g] * cw;
            orc_harmonics(p->L, oms[3 * v], oms[3 * v + 1], oms[3 * v + 2], R);
            for (int l = 0; l <= p->L; ++l)
                for (int mm = -l; mm <= l; ++mm) {
                    int lm = l * l + l + mm;
                    double f = 0.0;
                    for (int gp = 0; gp <= g; ++gp)
                        f += sgs(p, m, l, g, gp) * (phic[((long)gp * Nm + lm) * V + v] + phiu[(long)gp * V + v] * R[lm]);
                    gv += (2.0 * l + 1.0) / (4.0 * M_PI) * phia[((long)g * Nm + lm) * V + v] * f;
                }
            grad[v] += gv;
        }
    }
    /* back-projection of the uncollided term along every ray */
    double *B = (double *)malloc(sizeof(double) * (size_t)p->n_mat);
    for (long vp = 0; vp < V; ++vp) {
        int mp = p->material[vp];
        double rhop = p->density ? p->density[vp] : 1.0;
        orc_harmonics(p->L, oms[3 * vp], oms[3 * vp + 1], oms[3 * vp + 2], R);
        for (int m = 0; m < p->n_mat; ++m) B[m] = 0.0;
        int any = 0;
        for (int g = 0; g < G; ++g) {
            double pu = phiu[(long)g * V + vp];
            if (pu == 0.0) continue;
            any = 1;
            double Gu = W[(long)g * V + vp];
            for (int gpp = g; gpp < G; ++gpp)
                for (int l = 0; l <= p->L; ++l)
                    for (int mm = -l; mm <= l; ++mm) {
                        int lm = l * l + l + mm;
                        Gu += rhop * (2.0 * l + 1.0) / (4.0 * M_PI) * sgs(p, mp, l, gpp, g) * R[lm] *
                              phia[((long)gpp * Nm + lm) * V + vp];
                    }
            for (int m = 0; m < p->n_mat; ++m) B[m] += Gu * pu * p->sigma_t[m * G + g];
        }
        if (!any) continue;
        int i = (int)(vp % p->nx), j = (int)((vp / p->nx) % p->ny), k = (int)(vp / ((long)p->nx * p->ny));
        double c[3] = {(i + 0.5) * p->dx, (j + 0.5) * p->dy, (k + 0.5) * p->dz};
        bp_ctx ctx = {p, grad, B};
        ray_visit(p, s->pos, c, bp_fn, &ctx);
    }
    free(B);
    if (recip_out) *recip_out = recip;
    free(phit); free(phiu); free(phic); free(phia); free(oms); free(M); free(F); free(Fa);
    free(sig); free(psi); free(chi); free(tmp); free(masks);
    return st;
}
