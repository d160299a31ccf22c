// HIP kernels of one discrete-ordinates source iteration, written for gfx950
// (CDNA4, wave64).  See internal.h for the pencil voxel layout.
//
// Per group g (paper section II.A, eq. 2) one iteration is
//   k_m2d    scattering source: S_lm = F_lm + rho sigma_{s,l}^{g->g} phi_lm,
//            Q_n = sum_lm (2l+1)/(4 pi) R_lm(Omega_n) S_lm
//   k_sweep  diamond-difference transport sweep of every direction (sweep.hip)
//            (section II.B: voxels with i+j+k = S are independent)
//   k_d2m    moments phi_lm = sum_n w_n R_lm(Omega_n) psi_n (eq. 3 for lm = 00)
//            accumulated in FP64, plus the residual partial sums
//   k_resid  relative change of phi_00 in FP64, convergence flag
// and before the iterations k_group_source builds F (first-collision source
// of eq. 5 from the ray-traced uncollided fluence, plus downscatter from the
// converged higher groups).
//
// Contractions use the octant reflection symmetry of the level-symmetric set:
// Omega_{o,p} = (s_x mu_p, s_y eta_p, s_z xi_p), and R_lm changes sign under a
// reflection of axis a exactly when its parity class has bit a.  So
//   Q_{o,p} = sum_c chi_c(o) T_{c,p},   T_{c,p} = sum_{lm in c} M0[p][lm] S_lm
//   phi_lm  = sum_p D0[p][lm] psit_{c(lm),p},   psit_{c,p} = sum_o chi_c(o) psi_{o,p}
// with chi_c(o) = (-1)^popcount(c & o): an 8-point Walsh-Hadamard transform,
// eight times fewer multiplies than the dense N(N+2) x (L+1)^2 product.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "internal.h"

namespace dsn {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int lm_l(int lm)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    return l;
}

// parity class of the real harmonic (l, m): bit0 odd under x -> -x,
// bit1 odd under y -> -y, bit2 odd under z -> -z
__host__ __device__ constexpr int lm_class(int lm)
{
    const int l = lm_l(lm), m = lm - l * l - l, am = m < 0 ? -m : m;
    const int xo = m >= 0 ? (am & 1) : ((am & 1) ^ 1);
    const int yo = m < 0 ? 1 : 0;
    const int zo = (l + am) & 1;
    return xo | (yo << 1) | (zo << 2);
}

// l and parity class of every moment index, as compile-time tables: kernels
// loop over lm with a constant trip count so the moment arrays stay in
// registers (a loop bound that depends on an outer index would not be fully
// unrolled, and the arrays would go to scratch).
struct LmTables {
    int l[(kMaxL + 1) * (kMaxL + 1)];
    int cls[(kMaxL + 1) * (kMaxL + 1)];
};
__host__ __device__ constexpr LmTables make_lm_tables()
{
    LmTables t{};
    for (int lm = 0; lm < (kMaxL + 1) * (kMaxL + 1); ++lm) {
        t.l[lm] = lm_l(lm);
        t.cls[lm] = lm_class(lm);
    }
    return t;
}

template <typename T>
__device__ __forceinline__ void fwht8(T x[8])
{
#pragma unroll
    for (int h = 1; h < 8; h <<= 1)
#pragma unroll
        for (int i = 0; i < 8; i += 2 * h)
#pragma unroll
            for (int j = i; j < i + h; ++j) {
                const T a = x[j], b = x[j + h];
                x[j] = a + b;
                x[j + h] = a - b;
            }
}

// Real harmonics R_lm (Schmidt semi-normalised, no Condon-Shortley phase),
// written through P_l^m(xi) = (1-xi^2)^(m/2) P~_l^m(xi) and
// (mu + i eta)^m = s^m e^{i m phi}, so no azimuth angle is formed.
template <int L>
__device__ __forceinline__ void harmonics(double mu, double eta, double xi, double *R)
{
    double C[L + 1], S[L + 1];
    C[0] = 1.0;
    S[0] = 0.0;
#pragma unroll
    for (int m = 1; m <= L; ++m) {
        C[m] = C[m - 1] * mu - S[m - 1] * eta;
        S[m] = S[m - 1] * mu + C[m - 1] * eta;
    }
    double P[L + 1][L + 1];
#pragma unroll
    for (int m = 0; m <= L; ++m) {
        double dfac = 1.0;
#pragma unroll
        for (int t = 3; t <= 2 * L; t += 2)
            if (t <= 2 * m - 1) dfac *= (double)t;
        P[m][m] = dfac;
#pragma unroll
        for (int l = 1; l <= L; ++l) {
            if (l == m + 1) P[l][m] = (2.0 * m + 1.0) * xi * P[m][m];
            else if (l >= m + 2)
                P[l][m] = ((2.0 * l - 1.0) * xi * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
        }
    }
    constexpr LmTables tab = make_lm_tables();
#pragma unroll
    for (int lm = 0; lm < (L + 1) * (L + 1); ++lm) {
        const int l = tab.l[lm], m = lm - l * l - l, am = m < 0 ? -m : m;
        double ratio = 1.0;
#pragma unroll
        for (int t = 1; t <= 2 * L; ++t)
            if (t >= l - am + 1 && t <= l + am) ratio /= (double)t;
        R[lm] = sqrt((am == 0 ? 1.0 : 2.0) * ratio) * P[l][am] * (m >= 0 ? C[am] : S[am]);
    }
}

__device__ __forceinline__ void pencil_coords(const Geom &g, long v, int &i, int &j, int &k)
{
    const int lane = (int)(v & 63);
    const long row = v >> 6;
    i = (int)(row % g.nx);
    const long pen = row / g.nx;
    const int J = (int)(pen % g.NJ), K = (int)(pen / g.NJ);
    j = J * kCB + (lane & 7);
    k = K * kCB + (lane >> 3);
}

__device__ __forceinline__ long pencil_index(const Geom &g, int i, int j, int k)
{
    const int J = j >> 3, K = k >> 3;
    return ((long)(K * g.NJ + J) * g.nx + i) * 64 + (j & 7) + ((k & 7) << 3);
}


// ---------------------------------------------------------------------------
// set-up: natural-order voxel data -> pencil order (ghosts padded)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_voxels_to_pencils(Geom g, const uint8_t *mat_nat,
                                                           const double *dens_nat, uint8_t *mat,
                                                           double *dens)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    if (v >= g.Vp) return;
    int i, j, k;
    pencil_coords(g, v, i, j, k);
    if (j >= g.ny || k >= g.nz) {
        mat[v] = kGhost;
        dens[v] = 0.0;
        return;
    }
    const long vn = i + (long)g.nx * (j + (long)g.ny * k);
    mat[v] = mat_nat[vn];
    dens[v] = dens_nat ? dens_nat[vn] : 1.0;
}

// ---------------------------------------------------------------------------
// a0: uncollided fluence by exact ray tracing (eq. 4 without scattering).
// One thread per voxel centre; the segment source -> centre is cut at every
// grid plane (crossings merged in increasing order as they are generated),
// each piece is charged to the voxel holding its midpoint.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_raytrace(SolveArgs<T> a0)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    const SolveArgs<T> a = at_source(a0, blockIdx.y);
    if (v >= a.g.Vp) return;
    const double sx0 = a.src_par[0], sy0 = a.src_par[1], sz0 = a.src_par[2];
    const double ax = a.src_par[3], ay = a.src_par[4], az = a.src_par[5];
    const double cos_half = a.src_par[6];
    const int iso = a.src_par[7] != 0.0;
    const double fnx = a.src_par[8], fny = a.src_par[9], fnz = a.src_par[10], sin_thick = a.src_par[11];
    const double *spec = a.src_spec;
    const Geom &gm = a.g;
    const long Vp = gm.Vp;
    int i, j, k;
    pencil_coords(gm, v, i, j, k);
    if (j >= gm.ny || k >= gm.nz) {
        for (int gg = 0; gg < a.G; ++gg) a.phiu[gg * Vp + v] = 0.0;
        a.oms[v] = 1.0;
        a.oms[Vp + v] = 0.0;
        a.oms[2 * Vp + v] = 0.0;
        return;
    }
    const double x0[3] = {sx0, sy0, sz0};
    const double x1[3] = {(i + 0.5) * gm.dx, (j + 0.5) * gm.dy, (k + 0.5) * gm.dz};
    const double h[3] = {gm.dx, gm.dy, gm.dz};
    const int nn[3] = {gm.nx, gm.ny, gm.nz};
    double d[3];
    for (int t = 0; t < 3; ++t) d[t] = x1[t] - x0[t];
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    a.oms[v] = d[0] / r;
    a.oms[Vp + v] = d[1] / r;
    a.oms[2 * Vp + v] = d[2] / r;
    const double an = sqrt(ax * ax + ay * ay + az * az);
    bool inside;
    if (iso) {
        inside = true;
    } else if (sin_thick < 0.0) {  // cone: angle to the axis
        inside = (d[0] * ax + d[1] * ay + d[2] * az) >= r * an * cos_half;
    } else {  // fan: out of the plane by at most the half thickness, in-plane angle to the axis
        const double t = d[0] * fnx + d[1] * fny + d[2] * fnz;
        const double pin = sqrt(fmax(r * r - t * t, 0.0));
        inside = fabs(t) <= r * sin_thick && (d[0] * ax + d[1] * ay + d[2] * az) >= pin * an * cos_half;
    }
    if (!inside) {
        for (int gg = 0; gg < a.G; ++gg) a.phiu[gg * Vp + v] = 0.0;
        return;
    }
    double lam[kMaxMat];
#pragma unroll
    for (int t = 0; t < kMaxMat; ++t) lam[t] = 0.0;
    int q[3], st[3];
    double al[3];
    for (int t = 0; t < 3; ++t) {
        al[t] = 2.0;
        st[t] = 0;
        q[t] = 0;
        if (d[t] > 0.0) {
            st[t] = 1;
            q[t] = (int)fmax(0.0, floor(x0[t] / h[t]));
        } else if (d[t] < 0.0) {
            st[t] = -1;
            q[t] = (int)fmin((double)nn[t], ceil(x0[t] / h[t]));
        }
        if (st[t] != 0) {
            while (q[t] >= 0 && q[t] <= nn[t]) {
                const double c = (q[t] * h[t] - x0[t]) / d[t];
                if (c > 0.0) {
                    if (c < 1.0) al[t] = c;
                    break;
                }
                q[t] += st[t];
            }
        }
    }
    double acur = 0.0;
    for (;;) {
        double an_ = fmin(al[0], fmin(al[1], al[2]));
        const bool last = an_ >= 1.0;
        if (last) an_ = 1.0;
        if (an_ > acur) {
            const double am = 0.5 * (acur + an_);
            const int ii = (int)floor((x0[0] + am * d[0]) / h[0]);
            const int jj = (int)floor((x0[1] + am * d[1]) / h[1]);
            const int kk = (int)floor((x0[2] + am * d[2]) / h[2]);
            if (ii >= 0 && ii < nn[0] && jj >= 0 && jj < nn[1] && kk >= 0 && kk < nn[2]) {
                const long vn = ii + (long)nn[0] * (jj + (long)nn[1] * kk);
                const int m = a.mat_nat[vn];
                const double rho = a.dens_nat ? a.dens_nat[vn] : 1.0;
                const double seg = rho * ((an_ - acur) * r);
#pragma unroll
                for (int t = 0; t < kMaxMat; ++t) lam[t] += (t == m) ? seg : 0.0;
            }
        }
        if (last) break;
        for (int t = 0; t < 3; ++t) {
            if (al[t] == an_) {
                q[t] += st[t];
                if (q[t] < 0 || q[t] > nn[t]) {
                    al[t] = 2.0;
                } else {
                    const double c = (q[t] * h[t] - x0[t]) / d[t];
                    al[t] = c < 1.0 ? c : 2.0;
                }
            }
        }
        acur = an_;
    }
    for (int gg = 0; gg < a.G; ++gg) {
        double tau = 0.0;
#pragma unroll
        for (int t = 0; t < kMaxMat; ++t)
            if (t < a.nmat) tau += a.xs_t[t * a.G + gg] * lam[t];
        a.phiu[gg * Vp + v] = spec[gg] * exp(-tau) / (4.0 * M_PI * r * r);
    }
}

// ---------------------------------------------------------------------------
// a5 + first-collision source: external moments of group g, the group's
// total cross section per voxel, zero initial flux.
//   F_lm = rho [ sum_{g'<=g} sigma_{s,l}^{g'->g} phiu^{g'} R_lm(Omega_s)
//              + sum_{g'<g}  sigma_{s,l}^{g'->g} phic_lm^{g'} ]
// For sources acting together (a.usum set) the first-collision part reads the
// summed uncollided moments sum_s phiu_s^{g'} R_lm(Omega_s) instead.
// ---------------------------------------------------------------------------
// Streamed arrays (angular fluence, moments, external source) are read and
// written non-temporally when NT is set (the runtime sets it when they
// exceed the last-level cache), else as ordinary accesses.
template <bool NT, typename X>
__device__ __forceinline__ X ld_stream(const X *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename X>
__device__ __forceinline__ void st_stream(X v, X *p)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Stores of angular data through LDS, block-cooperative.  A block of 256
// voxels that lies inside one pencil (pencil-major psi: psi_index) sees each
// direction as one contiguous row of 256 values.  For direction index p the
// threads put their 8 octant values in an LDS tile [8][256] at their own
// voxel, and wave w then writes octant rows 2w and 2w + 1 (rows o * D + p of
// the block's run) in 16-byte accesses: whole 2 KB rows instead of one
// 8-byte store per voxel and direction (FP64; FP32 psi is faster with the
// plain per-voxel stores).
typedef unsigned U4 __attribute__((ext_vector_type(4)));

template <typename T, bool NT>
__device__ __forceinline__ void store_rows(T *blk, long PL, int D, int p, T (*tile)[256])
{
    constexpr int VL = 16 / (int)sizeof(T);  // values per 16-byte access
    constexpr int NI = 256 / (64 * VL);      // accesses per row and lane
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        U4 *row = (U4 *)(blk + (long)((2 * w + h) * D + p) * PL);
#pragma unroll
        for (int i = 0; i < NI; ++i)
            st_stream<NT>(*(const U4 *)&tile[2 * w + h][(i * 64 + lane) * VL], row + i * 64 + lane);
    }
}

// Whether block bx (voxels 256 bx ..) lies inside one pencil, which every
// block does when nx is a multiple of 4.  Uniform over the block.
__device__ __forceinline__ bool block_in_pencil(const Geom &g, unsigned bx)
{
    const long PL = (long)g.nx * 64, v0 = bx * 256L;
    return v0 + 256 <= g.Vp && v0 / PL == (v0 + 255) / PL;
}

// Directional source of one voxel from its source moments S (registers):
// Q_{o,p} = sum_c chi_c(o) sum_{lm in c} M0[p][lm] S_lm, written over psi.
// coop (uniform over the block, which then lies inside one pencil): stores
// through the LDS tiles stage[p & 1], one barrier per direction index p (a
// tile is written again two indices later, after every thread has passed the
// barrier of the index in between).
template <typename T, int L, bool NT>
__device__ __forceinline__ void expand_moments(const SolveArgs<T> &a, long v, const T (&S)[(L + 1) * (L + 1)],
                                               bool coop, T (*stage)[8][256])
{
    constexpr int Nm = (L + 1) * (L + 1);
    constexpr LmTables tab = make_lm_tables();
    const int D = a.D;
    const long PL = (long)a.g.nx * 64;
    // M0 is read-only for the whole launch: read through the constant address
    // space, its uniform rows are scalar loads.  As plain global loads beside
    // the psi stores they were vector loads, and each wait for a row also
    // waited for every store issued before it (one counter for both).
    const __attribute__((address_space(4))) T *M0 = (const __attribute__((address_space(4))) T *)a.M0;
    T *blk = a.psi + psi_index(a.g, a.Nd, v - threadIdx.x);
    T *out = a.psi + psi_index(a.g, a.Nd, v);
    for (int p = 0; p < D; ++p) {
        T t[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) t[c] = T(0);
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) t[tab.cls[lm]] += M0[p * Nm + lm] * S[lm];
        fwht8(t);
        if (coop) {
            T(*tile)[256] = stage[p & 1];
#pragma unroll
            for (int o = 0; o < 8; ++o) tile[o][threadIdx.x] = t[o];
            __syncthreads();
            store_rows<T, NT>(blk, PL, D, p, tile);
        } else {
#pragma unroll
            for (int o = 0; o < 8; ++o) st_stream<NT>(t[o], &out[(long)(o * D + p) * PL]);
        }
    }
}

// EXPAND: also form the group's first directional source (the moments start
// at zero, so S = F) while F is in registers, instead of a separate k_m2d.
template <typename T, int L, bool EXPAND, bool NT>
__global__ __launch_bounds__(256) void k_group_source(SolveArgs<T> a0, int g, int zero_phi)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long v = blockIdx.x * 256L + threadIdx.x;
    const SolveArgs<T> a = at_source(a0, blockIdx.y);
    const long Vp = a.g.Vp;
    if (v >= Vp) return;
    __shared__ T stage[2][8][256];
    const int G = a.G;
    const int m = a.mat[v];
    double f[Nm];
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) f[lm] = 0.0;
    T sg = T(0);
    if (m != kGhost) {
        const double rho = a.dens[v];
        constexpr LmTables tab = make_lm_tables();
        const double *xs = a.xs_s + (long)m * (L + 1) * G * G + (long)g * G;
        if (a.usum) {
            for (int gp = 0; gp <= g; ++gp) {
                double c[L + 1];
#pragma unroll
                for (int l = 0; l <= L; ++l) c[l] = xs[(long)l * G * G + gp];
                const double *u = a.usum + (long)gp * Nm * Vp + v;
#pragma unroll
                for (int lm = 0; lm < Nm; ++lm) f[lm] += c[tab.l[lm]] * u[(long)lm * Vp];
            }
        } else {
            double R[Nm];
            harmonics<L>(a.oms[v], a.oms[Vp + v], a.oms[2 * Vp + v], R);
            for (int gp = 0; gp <= g; ++gp) {
                const double pu = a.phiu[gp * Vp + v];
                if (pu == 0.0) continue;
                double c[L + 1];
#pragma unroll
                for (int l = 0; l <= L; ++l) c[l] = xs[(long)l * G * G + gp] * pu;
#pragma unroll
                for (int lm = 0; lm < Nm; ++lm) f[lm] += c[tab.l[lm]] * R[lm];
            }
        }
        for (int gp = 0; gp < g; ++gp) {
            double c[L + 1];
#pragma unroll
            for (int l = 0; l <= L; ++l) c[l] = xs[(long)l * G * G + gp];
            const double *ph = a.phic + (long)gp * Nm * Vp + v;
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) f[lm] += c[tab.l[lm]] * ld_stream<NT>(&ph[(long)lm * Vp]);
        }
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) f[lm] *= rho;
        sg = (T)(rho * a.xs_t[m * G + g]);
    }
    if (blockIdx.y == 0) a.sig[v] = sg;  // shared by the batch
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) {
        st_stream<NT>((T)f[lm], &a.F[lm * Vp + v]);
        if (zero_phi) st_stream<NT>(0.0, &a.phic[((long)g * Nm + lm) * Vp + v]);
    }
    if constexpr (EXPAND) {
        T S[Nm];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) S[lm] = (T)(f[lm] + 0.0);  // as F + sigma_s * phi with phi = 0
        expand_moments<T, L, NT>(a, v, S, sizeof(T) == 8 && block_in_pencil(a.g, blockIdx.x), stage);
    }
}

// Sources acting together: per group, the summed uncollided fluence
// pusum = sum_s phiu_s and moments usum_lm = sum_s phiu_s R_lm(Omega_s) of
// sources 0 .. nsrc-1 (their ray traces in a0's per-source buffers).
template <typename T, int L>
__global__ __launch_bounds__(256) void k_sum_uncollided(SolveArgs<T> a0, int nsrc, double *usum, double *pusum)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = a0.g.Vp;
    if (v >= Vp) return;
    for (int g = 0; g < a0.G; ++g) {
        double acc[Nm];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) acc[lm] = 0.0;
        double pt = 0.0;
        for (int k = 0; k < nsrc; ++k) {
            const SolveArgs<T> b = at_source(a0, k);
            const double pu = b.phiu[(long)g * Vp + v];
            if (pu == 0.0) continue;
            double R[Nm];
            harmonics<L>(b.oms[v], b.oms[Vp + v], b.oms[2 * Vp + v], R);
            pt += pu;
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) acc[lm] += pu * R[lm];
        }
        pusum[(long)g * Vp + v] = pt;
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) usum[((long)g * Nm + lm) * Vp + v] = acc[lm];
    }
}

__global__ void k_ctl_init(Ctl *ctl0, int G, int nsrc, int g, int target, int max_iters, double tol,
                           int stag_stop, int rule)
{
    if (blockIdx.x != 0 || (int)threadIdx.x >= nsrc) return;
    Ctl *ctl = ctl0 + (long)threadIdx.x * G;
    Ctl c;
    c.iters = 0;
    c.done = target == 0 ? 1 : 0;
    c.target = target;
    c.max_iters = max_iters;
    c.stag_stop = stag_stop;
    c.stag = 0;
    c.status = 0;
    c.rule = rule;
    c.tol = tol;
    c.r = 0.0;
    c.r_prev = 0.0;
    c.tmax = 0.0;
    c.est = INFINITY;
    c.rmin = INFINITY;
    ctl[g] = c;
}

// ---------------------------------------------------------------------------
// a1: scattering source assembly and moment -> direction contraction
// ---------------------------------------------------------------------------
// Source moments S_lm = F_lm + rho sigma_{s,l}^{g->g} phi_lm of voxel v and
// their expansion Q_n = sum_lm M(n, lm) S_lm over every direction, written
// into psi.  phi(lm) gives the group's current moments; coop and stage as
// for expand_moments.
template <typename T, int L, bool NT, typename PHI>
__device__ __forceinline__ void expand_source(const SolveArgs<T> &a, int g, long v, PHI phi, bool coop,
                                              T (*stage)[8][256])
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long Vp = a.g.Vp;
    const int G = a.G;
    const int m = a.mat[v];
    constexpr LmTables tab = make_lm_tables();
    T S[Nm];
    if (m == kGhost) {
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) S[lm] = T(0);
    } else {
        const double rho = a.dens[v];
        double sl[L + 1];
#pragma unroll
        for (int l = 0; l <= L; ++l) sl[l] = rho * a.xs_s[(((long)m * (L + 1) + l) * G + g) * G + g];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm)
            S[lm] = (T)((double)ld_stream<NT>(&a.F[lm * Vp + v]) + sl[tab.l[lm]] * phi(lm));
    }
    expand_moments<T, L, NT>(a, v, S, coop, stage);
}

template <typename T, int L>
__global__ __launch_bounds__(256) void k_m2d(SolveArgs<T> a0, int g)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const SolveArgs<T> a = at_source(a0, blockIdx.y);
    if (a.ctl[g].done) return;
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = a.g.Vp;
    if (v >= Vp) return;
    __shared__ T stage[2][8][256];
    const double *ph = a.phic + (long)g * Nm * Vp + v;
    expand_source<T, L, false>(a, g, v, [&](int lm) { return ph[(long)lm * Vp]; },
                               sizeof(T) == 8 && block_in_pencil(a.g, blockIdx.x), stage);
}

// ---------------------------------------------------------------------------
// a3 + a4: direction -> moment quadrature in FP64 and residual partial sums
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ double wave_max(double x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    return x;
}

// EXPAND: also form the next iteration's directional source from the new
// moments (the work of k_m2d, while the moments are still in registers), so
// an iteration is one sweep and one pass over psi.
// Residual partials of each block: the sums of (phi00_new - phi00_old)^2 and
// phi00_new^2, and for the pointwise rule the largest |total| = |phi_u +
// phi00_new| and the largest |phi00_new - phi00_old| / |total| over voxels
// whose |total| reaches 1e-6 of the previous iterate's largest.  Maxima do not
// depend on the order of reduction.
template <typename T, int L, bool EXPAND, bool NT>
__device__ __forceinline__ void d2m_body(const SolveArgs<T> &a, int g, unsigned bx)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const Ctl &cg = a.ctl[g];
    if (cg.done) return;
    const int rule = cg.rule;
    const double floor_t = 1e-6 * cg.tmax;
    const long v = bx * 256L + threadIdx.x;
    const long Vp = a.g.Vp;
    const int D = a.D;
    double d2 = 0.0, n2 = 0.0, tm = 0.0, dm = 0.0;
    constexpr LmTables tab = make_lm_tables();
    __shared__ T stage[2][8][256];
    const bool coop = sizeof(T) == 8 && block_in_pencil(a.g, bx);
    if (v < Vp) {
        double acc[Nm];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) acc[lm] = 0.0;
        const T *in = a.psi + psi_index(a.g, a.Nd, v);
        const long PL = (long)a.g.nx * 64;  // direction stride of pencil-major psi
        const double *D0 = a.D0;
        for (int p = 0; p < D; ++p) {
            double x[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) x[o] = (double)ld_stream<NT>(&in[(long)(o * D + p) * PL]);
            fwht8(x);
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) acc[lm] += D0[p * Nm + lm] * x[tab.cls[lm]];
        }
        double *ph = a.phic + (long)g * Nm * Vp + v;
        const double old = ld_stream<NT>(&ph[0]);
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) st_stream<NT>(acc[lm], &ph[(long)lm * Vp]);
        const double dd = acc[0] - old;
        d2 = dd * dd;
        n2 = acc[0] * acc[0];
        if (rule == 1) {
            const double t = fabs(a.phiu[(long)g * Vp + v] + acc[0]);
            tm = t;
            if (t > 0.0 && t >= floor_t) dm = fabs(dd) / t;
        }
        if (EXPAND) expand_source<T, L, NT>(a, g, v, [&](int lm) { return acc[lm]; }, coop, stage);
    }
    __shared__ double red[4][4];
    d2 = wave_sum(d2);
    n2 = wave_sum(n2);
    tm = wave_max(tm);
    dm = wave_max(dm);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = d2; red[1][w] = n2; red[2][w] = tm; red[3][w] = dm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double *pb = a.part + 4 * bx;
        pb[0] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        pb[1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        pb[2] = fmax(fmax(red[2][0], red[2][1]), fmax(red[2][2], red[2][3]));
        pb[3] = fmax(fmax(red[3][0], red[3][1]), fmax(red[3][2], red[3][3]));
    }
}

template <typename T, int L, bool EXPAND, bool NT>
__global__ __launch_bounds__(256) void k_d2m(SolveArgs<T> a0, int g)
{
    d2m_body<T, L, EXPAND, NT>(at_source(a0, blockIdx.y), g, blockIdx.x);
}

// The moments of every (problem, source) pair of a fused batch in one
// launch: blockIdx.z = problem (its argument block in tab), blockIdx.y =
// source, blockIdx.x = voxel block; blocks past a smaller problem's voxels
// or sources leave at once.
template <typename T, int L, bool EXPAND, bool NT>
__global__ __launch_bounds__(256) void k_d2m_multi(const SolveArgs<T> *tab, int g)
{
    const SolveArgs<T> &a0 = tab[blockIdx.z];
    if ((long)blockIdx.x * 256 >= a0.g.Vp || (int)blockIdx.y >= a0.S) return;
    d2m_body<T, L, EXPAND, NT>(at_source(a0, blockIdx.y), g, blockIdx.x);
}

// Convergence test of one group (section II.C leaves the criterion open).
// r = ||phi00_new - phi00_old||_2 / ||phi00_new||_2 (0/0 = 0).  Rule 0 stops
// when r < tol.  Rule 1 stops when the estimated per-voxel error left,
// est = d rho / (1 - rho), drops below tol: d is the largest change of phi_00
// relative to the voxel's total fluence (voxels above 1e-6 of the previous
// iterate's largest total) and rho = r / r_prev estimates the factor by which
// source iteration shrinks the change per step, so the changes still to come
// sum to about d rho / (1 - rho).  The first iterate (no rho yet) never stops
// rule 1 unless r = 0.
__device__ __forceinline__ void resid_body(Ctl *ctl, int g, const double *part, int nblk)
{
    if (ctl[g].done) return;
    double s0 = 0.0, s1 = 0.0, tm = 0.0, dm = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        s0 += part[4 * b];
        s1 += part[4 * b + 1];
        tm = fmax(tm, part[4 * b + 2]);
        dm = fmax(dm, part[4 * b + 3]);
    }
    __shared__ double red[4][4];
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    tm = wave_max(tm);
    dm = wave_max(dm);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = s0; red[1][w] = s1; red[2][w] = tm; red[3][w] = dm; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    s0 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    s1 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    tm = fmax(fmax(red[2][0], red[2][1]), fmax(red[2][2], red[2][3]));
    dm = fmax(fmax(red[3][0], red[3][1]), fmax(red[3][2], red[3][3]));
    Ctl c = ctl[g];
    double r;
    if (s1 == 0.0) r = s0 == 0.0 ? 0.0 : INFINITY;
    else r = sqrt(s0) / sqrt(s1);
    c.iters += 1;
    c.r_prev = c.r;
    c.r = r;
    bool conv = r < c.tol;
    if (c.rule == 1) {
        const double rho = (c.iters >= 2 && c.r_prev > 0.0) ? r / c.r_prev : 1.0;
        c.est = rho < 1.0 ? dm * rho / (1.0 - rho) : INFINITY;
        c.tmax = tm;
        conv = r == 0.0 || c.est < c.tol;
    }
    if (c.target >= 0) {
        if (c.iters >= c.target) c.done = 1;
    } else if (!isfinite(r)) {
        c.done = 1;
        c.status = 6;
    } else if (conv) {
        c.done = 1;
        c.status = 0;
    } else {
        // stagnation (the FP32 rounding floor): three iterations in a row
        // that do not improve on the smallest value so far of the quantity
        // the rule tests (r, or est for rule 1)
        const double m = c.rule == 1 ? c.est : r;
        if (m < c.rmin) {
            c.rmin = m;
            c.stag = 0;
        } else if (c.stag_stop && ++c.stag >= 3) {
            c.done = 1;
            c.status = 7;
        }
        if (!c.done && c.iters >= c.max_iters) { c.done = 1; c.status = 5; }
    }
    ctl[g] = c;
}

__global__ __launch_bounds__(256) void k_resid(Ctl *ctl0, int G, long str_part, int g, const double *part0,
                                              int nblk)
{
    resid_body(ctl0 + (long)blockIdx.x * G, g, part0 + blockIdx.x * str_part, nblk);
}

// The convergence test of every (problem, source) pair of a fused batch:
// blockIdx.y = problem, blockIdx.x = source.
template <typename T>
__global__ __launch_bounds__(256) void k_resid_multi(const SolveArgs<T> *tab, int g)
{
    const SolveArgs<T> &a = tab[blockIdx.y];
    if ((int)blockIdx.x >= a.S) return;
    resid_body(a.ctl + (long)blockIdx.x * a.G, g, a.part + blockIdx.x * a.str_part, (int)((a.g.Vp + 255) / 256));
}

// ---------------------------------------------------------------------------
// a6: total fluence of group g into the caller's natural-order buffers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Absorbed dose, the quantity the fluence is computed for (paper sections I
// and IV): dose[s][v] = sum_g phi[s][g][v] k[m(v)][g], with k the caller's
// fluence-to-dose factor per material and group.  One thread per voxel in
// natural order; each group's read is a coalesced row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dose(const uint8_t *mat, long V, int G, const double *phi, const double *k,
                                              double *dose)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    if (v >= V) return;
    const long s = blockIdx.y;
    const double *ph = phi + s * G * V + v;
    const double *km = k + (long)mat[v] * G;
    double acc = 0.0;
    for (int g = 0; g < G; ++g) acc += ph[(long)g * V] * km[g];
    dose[s * V + v] = acc;
}

template <typename T>
__global__ __launch_bounds__(256) void k_finalize(SolveArgs<T> a0, int g, double *phi_total0, double *phi_unc0)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    const SolveArgs<T> a = at_source(a0, blockIdx.y);
    const Geom &gm = a.g;
    double *phi_total = phi_total0 + (long)blockIdx.y * a.G * gm.V;
    double *phi_unc = phi_unc0 ? phi_unc0 + (long)blockIdx.y * a.G * gm.V : nullptr;
    if (v >= gm.V) return;
    const int i = (int)(v % gm.nx), j = (int)((v / gm.nx) % gm.ny), k = (int)(v / ((long)gm.nx * gm.ny));
    const long vp = pencil_index(gm, i, j, k);
    const double pu = a.phiu[(long)g * gm.Vp + vp];
    phi_total[(long)g * gm.V + v] = pu + a.phic[(long)g * a.Nm * gm.Vp + vp];
    if (phi_unc) phi_unc[(long)g * gm.V + v] = pu;
}

// ---------------------------------------------------------------------------
// Adjoint of the converged discrete solve and density gradient (pure DD).
//
// With W the detector weights of J = sum_g sum_v W^g(v) phi_total^g(v), the
// adjoint angular fluence chi^g (per unit quadrature weight) solves, from the
// lowest-energy group up, source iteration along -Omega_n with source
//   Qa_n = W^g + sum_lm (2l+1)/(4 pi) R_lm(Omega_n) rho
//          (sigma_{s,l}^{g->g} phia_lm^g + sum_{g''>g} sigma_{s,l}^{g->g''} phia_lm^{g''})
// i.e. external moments Fa_00 = 4 pi W^g plus the adjoint downscatter, and
// phia_lm = sum_n w_n R_lm(Omega_n) chi_n.  The gradient is
//   dJ/drho(v) = sum_g [ -sigma_t^g sum_n w_n chi_n psi_n
//                + sum_lm (2l+1)/(4pi) phia_lm^g sum_{g'<=g} sigma_{s,l}^{g'->g}
//                  (phic_lm^{g'} + phiu^{g'} R_lm(Omega_s)) ]
//              - sum_{v'} B_{m(v)}(v') len(v; source -> centre of v')
//   B_m(v') = sum_g Gu^g(v') phiu^g(v') sigma_t^g[m],
//   Gu^g(v') = W^g(v') + rho sum_{g''>=g} sum_lm (2l+1)/(4pi)
//              sigma_{s,l}^{g->g''} R_lm(Omega_s) phia_lm^{g''}
// (the last line is the derivative of the uncollided fluence through the
// optical depth of every ray, back-projected along the ray).
// ---------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(256) void k_adj_source(SolveArgs<T> a, int g, const double *W, int zero_phi)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = a.g.Vp;
    if (v >= Vp) return;
    const int G = a.G;
    const int m = a.mat[v];
    double f[Nm];
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) f[lm] = 0.0;
    T sg = T(0);
    if (m != kGhost) {
        const double rho = a.dens[v];
        constexpr LmTables tab = make_lm_tables();
        for (int gpp = g + 1; gpp < G; ++gpp) {
            double c[L + 1];
#pragma unroll
            for (int l = 0; l <= L; ++l) c[l] = a.xs_s[(((long)m * (L + 1) + l) * G + gpp) * G + g];
            const double *ph = a.phic + (long)gpp * Nm * Vp + v;
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) f[lm] += c[tab.l[lm]] * ph[(long)lm * Vp];
        }
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) f[lm] *= rho;
        int i, j, k;
        pencil_coords(a.g, v, i, j, k);
        f[0] += 4.0 * M_PI * W[(long)g * a.g.V + i + (long)a.g.nx * (j + (long)a.g.ny * k)];
        sg = (T)(rho * a.xs_t[m * G + g]);
    }
    a.sig[v] = sg;
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) {
        a.F[lm * Vp + v] = (T)f[lm];
        if (zero_phi) a.phic[((long)g * Nm + lm) * Vp + v] = 0.0;
    }
}

// collision, scattering and first-collision terms of group g
template <typename T, int L>
__global__ __launch_bounds__(256) void k_grad_accum(SolveArgs<T> fw, SolveArgs<T> ad, int g, double *grad)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = fw.g.Vp;
    if (v >= Vp) return;
    const int m = fw.mat[v];
    if (m == kGhost) return;
    const int G = fw.G, Nd = fw.Nd;
    double cw = 0.0;
    const long pv = psi_index(fw.g, Nd, v), PL = (long)fw.g.nx * 64;
    for (int n = 0; n < Nd; ++n)
        cw += fw.wdir[n] * (double)ad.psi[pv + n * PL] * (double)fw.psi[pv + n * PL];
    double gv = -fw.xs_t[m * G + g] * cw;
    double R[Nm], f[Nm];
    harmonics<L>(fw.oms[v], fw.oms[Vp + v], fw.oms[2 * Vp + v], R);
    constexpr LmTables tab = make_lm_tables();
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) f[lm] = 0.0;
    for (int gp = 0; gp <= g; ++gp) {
        double c[L + 1];
#pragma unroll
        for (int l = 0; l <= L; ++l) c[l] = fw.xs_s[(((long)m * (L + 1) + l) * G + g) * G + gp];
        const double pu = fw.phiu[(long)gp * Vp + v];
        const double *ph = fw.phic + (long)gp * Nm * Vp + v;
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) f[lm] += c[tab.l[lm]] * (ph[(long)lm * Vp] + pu * R[lm]);
    }
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm)
        gv += (2.0 * tab.l[lm] + 1.0) / (4.0 * M_PI) * ad.phic[((long)g * Nm + lm) * Vp + v] * f[lm];
    int i, j, k;
    pencil_coords(fw.g, v, i, j, k);
    grad[i + (long)fw.g.nx * (j + (long)fw.g.ny * k)] += gv;
}

// back-projection of the uncollided term: one thread per ray end v'
template <typename T, int L>
__global__ __launch_bounds__(256) void k_backproject(SolveArgs<T> a, const double *phia, const double *W,
                                                     double sx0, double sy0, double sz0, double *grad)
{
    constexpr int Nm = (L + 1) * (L + 1);
    const long v = blockIdx.x * 256L + threadIdx.x;
    const Geom &gm = a.g;
    const long Vp = gm.Vp;
    if (v >= Vp) return;
    const int mp = a.mat[v];
    if (mp == kGhost) return;
    const int G = a.G;
    const double rho = a.dens[v];
    int i, j, k;
    pencil_coords(gm, v, i, j, k);
    const long vn = i + (long)gm.nx * (j + (long)gm.ny * k);
    double R[Nm];
    harmonics<L>(a.oms[v], a.oms[Vp + v], a.oms[2 * Vp + v], R);
    double B[kMaxMat];
#pragma unroll
    for (int t = 0; t < kMaxMat; ++t) B[t] = 0.0;
    bool any = false;
    for (int gg = 0; gg < G; ++gg) {
        const double pu = a.phiu[(long)gg * Vp + v];
        if (pu == 0.0) continue;
        any = true;
        double Gu = W[(long)gg * gm.V + vn];
        constexpr LmTables tab = make_lm_tables();
        for (int gpp = gg; gpp < G; ++gpp) {
            double c[L + 1];
#pragma unroll
            for (int l = 0; l <= L; ++l)
                c[l] = rho * (2.0 * l + 1.0) / (4.0 * M_PI) * a.xs_s[(((long)mp * (L + 1) + l) * G + gpp) * G + gg];
            const double *ph = phia + (long)gpp * Nm * Vp + v;
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) Gu += c[tab.l[lm]] * R[lm] * ph[(long)lm * Vp];
        }
#pragma unroll
        for (int t = 0; t < kMaxMat; ++t)
            if (t < a.nmat) B[t] += Gu * pu * a.xs_t[t * G + gg];
    }
    if (!any) return;
    // walk the ray source -> centre of v' (same plane-crossing traversal as the
    // forward ray trace) and subtract B_m * length from every voxel crossed
    const double x0[3] = {sx0, sy0, sz0};
    const double x1[3] = {(i + 0.5) * gm.dx, (j + 0.5) * gm.dy, (k + 0.5) * gm.dz};
    const double h[3] = {gm.dx, gm.dy, gm.dz};
    const int nn[3] = {gm.nx, gm.ny, gm.nz};
    double d[3];
    for (int t = 0; t < 3; ++t) d[t] = x1[t] - x0[t];
    const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int q[3], st[3];
    double al[3];
    for (int t = 0; t < 3; ++t) {
        al[t] = 2.0;
        st[t] = 0;
        q[t] = 0;
        if (d[t] > 0.0) {
            st[t] = 1;
            q[t] = (int)fmax(0.0, floor(x0[t] / h[t]));
        } else if (d[t] < 0.0) {
            st[t] = -1;
            q[t] = (int)fmin((double)nn[t], ceil(x0[t] / h[t]));
        }
        if (st[t] != 0) {
            while (q[t] >= 0 && q[t] <= nn[t]) {
                const double c = (q[t] * h[t] - x0[t]) / d[t];
                if (c > 0.0) {
                    if (c < 1.0) al[t] = c;
                    break;
                }
                q[t] += st[t];
            }
        }
    }
    double acur = 0.0;
    for (;;) {
        double an_ = fmin(al[0], fmin(al[1], al[2]));
        const bool last = an_ >= 1.0;
        if (last) an_ = 1.0;
        if (an_ > acur) {
            const double am = 0.5 * (acur + an_);
            const int ii = (int)floor((x0[0] + am * d[0]) / h[0]);
            const int jj = (int)floor((x0[1] + am * d[1]) / h[1]);
            const int kk = (int)floor((x0[2] + am * d[2]) / h[2]);
            if (ii >= 0 && ii < nn[0] && jj >= 0 && jj < nn[1] && kk >= 0 && kk < nn[2]) {
                const long vv = ii + (long)nn[0] * (jj + (long)nn[1] * kk);
                atomicAdd(&grad[vv], -B[a.mat_nat[vv]] * ((an_ - acur) * r));
            }
        }
        if (last) break;
        for (int t = 0; t < 3; ++t) {
            if (al[t] == an_) {
                q[t] += st[t];
                if (q[t] < 0 || q[t] > nn[t]) {
                    al[t] = 2.0;
                } else {
                    const double c = (q[t] * h[t] - x0[t]) / d[t];
                    al[t] = c < 1.0 ? c : 2.0;
                }
            }
        }
        acur = an_;
    }
}

// x . y in FP64: per-block partial sums, then one block in fixed order
__global__ __launch_bounds__(256) void k_dot_part(const double *x, const double *y, long n, double *part)
{
    double s = 0.0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) s += x[i] * y[i];
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_dot_final(const double *part, int nblk, double *out)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += part[b];
    __shared__ double red[4];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }

void launch_voxels_to_pencils(const Geom &g, const uint8_t *mat_nat, const double *dens_nat, uint8_t *mat,
                              double *dens, hipStream_t s)
{
    hipLaunchKernelGGL(k_voxels_to_pencils, dim3(nblk(g.Vp)), dim3(256), 0, s, g, mat_nat, dens_nat, mat, dens);
}

template <typename T>
void launch_raytrace(const SolveArgs<T> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_raytrace<T>, dim3(nblk(a.g.Vp), a.S), dim3(256), 0, s, a);
}

#define DSN_DISPATCH_L(L_, EXPR)                \
    switch (L_) {                               \
    case 0: { constexpr int LL = 0; EXPR; } break; \
    case 1: { constexpr int LL = 1; EXPR; } break; \
    case 2: { constexpr int LL = 2; EXPR; } break; \
    case 3: { constexpr int LL = 3; EXPR; } break; \
    case 4: { constexpr int LL = 4; EXPR; } break; \
    default: { constexpr int LL = 5; EXPR; } break; \
    }

template <typename T>
void launch_group_source(const SolveArgs<T> &a, int g, bool expand, hipStream_t s)
{
    const dim3 grid(nblk(a.g.Vp), a.S);
    if (expand && a.stream_nt) {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_group_source<T, LL, true, true>), grid, dim3(256), 0, s, a, g, 1));
    } else if (expand) {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_group_source<T, LL, true, false>), grid, dim3(256), 0, s, a, g, 1));
    } else {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_group_source<T, LL, false, false>), grid, dim3(256), 0, s, a, g, 1));
    }
}

template <typename T>
void launch_sum_uncollided(const SolveArgs<T> &a, int nsrc, double *usum, double *pusum, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_sum_uncollided<T, LL>), dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, nsrc,
                                           usum, pusum));
}

// same, keeping the group's converged moments (gradient recomputation)
template <typename T>
void launch_group_source_keep(const SolveArgs<T> &a, int g, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_group_source<T, LL, false, false>), dim3(nblk(a.g.Vp), a.S), dim3(256), 0,
                                           s, a, g, 0));
}

void launch_ctl_init(Ctl *ctl, int G, int nsrc, int g, int target, int max_iters, double tol, int stag_stop,
                     int rule, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(1024), 0, s, ctl, G, nsrc, g, target, max_iters, tol, stag_stop,
                       rule);
}

template <typename T>
int launch_m2d(const SolveArgs<T> &a, int g, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_m2d<T, LL>), dim3(nblk(a.g.Vp), a.S), dim3(256), 0, s, a, g));
    return 1;
}

template <typename T>
int launch_d2m(const SolveArgs<T> &a, int g, bool expand, hipStream_t s)
{
    const unsigned nb = nblk(a.g.Vp);
    if (expand && a.stream_nt) {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m<T, LL, true, true>), dim3(nb, a.S), dim3(256), 0, s, a, g));
    } else if (expand) {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m<T, LL, true, false>), dim3(nb, a.S), dim3(256), 0, s, a, g));
    } else {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m<T, LL, false, false>), dim3(nb, a.S), dim3(256), 0, s, a, g));
    }
    hipLaunchKernelGGL(k_resid, dim3(a.S), dim3(256), 0, s, a.ctl, a.G, a.str_part, g, (const double *)a.part, (int)nb);
    return 2;
}

// Moments, residual partials, next directional source and convergence test
// of every (problem, source) pair of a fused batch: two launches.  tab: the
// problems' argument blocks on the device; a: any one of them (host), for
// the moment order; vp_max, s_max: the largest padded voxel count and
// source count among them; nt: non-temporal streams.
template <typename T>
int launch_d2m_multi(const SolveArgs<T> *tab, const SolveArgs<T> &a, int n, long vp_max, int s_max, bool nt, int g,
                     hipStream_t s)
{
    const dim3 grid(nblk(vp_max), s_max, n);
    if (nt) {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m_multi<T, LL, true, true>), grid, dim3(256), 0, s, tab, g));
    } else {
        DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m_multi<T, LL, true, false>), grid, dim3(256), 0, s, tab, g));
    }
    hipLaunchKernelGGL(k_resid_multi<T>, dim3(s_max, n), dim3(256), 0, s, tab, g);
    return 2;
}

template <typename T>
void launch_finalize(const SolveArgs<T> &a, int g, double *phi_total, double *phi_unc, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize<T>, dim3(nblk(a.g.V), a.S), dim3(256), 0, s, a, g, phi_total, phi_unc);
}

template <typename T>
void launch_adj_source(const SolveArgs<T> &a, int g, const double *W, int zero_phi, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_adj_source<T, LL>), dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, g, W,
                                           zero_phi));
}

template <typename T>
void launch_m2d_always(const SolveArgs<T> &a, int g, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_m2d<T, LL>), dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, g));
}

template <typename T>
void launch_grad_accum(const SolveArgs<T> &fw, const SolveArgs<T> &ad, int g, double *grad, hipStream_t s)
{
    DSN_DISPATCH_L(fw.L, hipLaunchKernelGGL((k_grad_accum<T, LL>), dim3(nblk(fw.g.Vp)), dim3(256), 0, s, fw, ad,
                                            g, grad));
}

template <typename T>
void launch_backproject(const SolveArgs<T> &fw, const double *phia, const double *W, const double pos[3],
                        double *grad, hipStream_t s)
{
    DSN_DISPATCH_L(fw.L, hipLaunchKernelGGL((k_backproject<T, LL>), dim3(nblk(fw.g.Vp)), dim3(256), 0, s, fw, phia,
                                            W, pos[0], pos[1], pos[2], grad));
}

void launch_dose(const uint8_t *mat, long V, int G, const double *phi, const double *k, int n, double *dose,
                 hipStream_t s)
{
    hipLaunchKernelGGL(k_dose, dim3(nblk(V), n), dim3(256), 0, s, mat, V, G, phi, k, dose);
}

void launch_dot(const double *x, const double *y, long n, double *part, int nb, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(256), 0, s, x, y, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, s, (const double *)part, nb, out);
}

#define DSN_INST_ADJ(T)                                                                                      \
    template void launch_group_source_keep<T>(const SolveArgs<T> &, int, hipStream_t);                      \
    template void launch_adj_source<T>(const SolveArgs<T> &, int, const double *, int, hipStream_t);        \
    template void launch_m2d_always<T>(const SolveArgs<T> &, int, hipStream_t);                             \
    template void launch_grad_accum<T>(const SolveArgs<T> &, const SolveArgs<T> &, int, double *, hipStream_t); \
    template void launch_backproject<T>(const SolveArgs<T> &, const double *, const double *, const double *, \
                                        double *, hipStream_t);
DSN_INST_ADJ(float)
DSN_INST_ADJ(double)

template void launch_raytrace<float>(const SolveArgs<float> &, hipStream_t);
template void launch_raytrace<double>(const SolveArgs<double> &, hipStream_t);
template void launch_group_source<float>(const SolveArgs<float> &, int, bool, hipStream_t);
template void launch_group_source<double>(const SolveArgs<double> &, int, bool, hipStream_t);
template void launch_sum_uncollided<float>(const SolveArgs<float> &, int, double *, double *, hipStream_t);
template void launch_sum_uncollided<double>(const SolveArgs<double> &, int, double *, double *, hipStream_t);
template int launch_m2d<float>(const SolveArgs<float> &, int, hipStream_t);
template int launch_m2d<double>(const SolveArgs<double> &, int, hipStream_t);
template int launch_d2m<float>(const SolveArgs<float> &, int, bool, hipStream_t);
template int launch_d2m<double>(const SolveArgs<double> &, int, bool, hipStream_t);
template int launch_d2m_multi<float>(const SolveArgs<float> *, const SolveArgs<float> &, int, long, int, bool, int,
                                     hipStream_t);
template int launch_d2m_multi<double>(const SolveArgs<double> *, const SolveArgs<double> &, int, long, int, bool, int,
                                      hipStream_t);
template void launch_finalize<float>(const SolveArgs<float> &, int, double *, double *, hipStream_t);
template void launch_finalize<double>(const SolveArgs<double> &, int, double *, double *, hipStream_t);

}  // namespace dsn
