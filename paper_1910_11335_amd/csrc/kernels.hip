// HIP kernels of one discrete-ordinates source iteration, written for gfx950
// (CDNA4, wave64).  See internal.h for the pencil voxel layout.
//
// Per group g (paper section II.A, eq. 2) one iteration is
//   k_m2d    scattering source: S_lm = F_lm + rho sigma_{s,l}^{g->g} phi_lm,
//            Q_n = sum_lm (2l+1)/(4 pi) R_lm(Omega_n) S_lm
//   k_sweep  diamond-difference transport sweep of every direction
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
        for (int t = 2 * m - 1; t > 1; t -= 2) dfac *= (double)t;
        P[m][m] = dfac;
        if (m + 1 <= L) P[m + 1][m] = (2.0 * m + 1.0) * xi * P[m][m];
#pragma unroll
        for (int l = m + 2; l <= L; ++l)
            P[l][m] = ((2.0 * l - 1.0) * xi * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
    }
#pragma unroll
    for (int l = 0; l <= L; ++l)
#pragma unroll
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            double ratio = 1.0;
            for (int t = l - am + 1; t <= l + am; ++t) ratio /= (double)t;
            const double nrm = sqrt((am == 0 ? 1.0 : 2.0) * ratio);
            R[l * l + l + m] = nrm * P[l][am] * (m >= 0 ? C[am] : S[am]);
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

template <typename T>
__device__ __forceinline__ T dd_div(T num, T den)
{
    return num / den;
}
template <>
__device__ __forceinline__ float dd_div<float>(float num, float den)
{
    return num * __builtin_amdgcn_rcpf(den);
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
__global__ __launch_bounds__(256) void k_raytrace(SolveArgs<T> a, double sx0, double sy0, double sz0,
                                                  double ax, double ay, double az, double cos_half,
                                                  int iso, const double *spec)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    if (v >= a.g.Vp) return;
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
    const bool inside = iso || (d[0] * ax + d[1] * ay + d[2] * az) >= r * an * cos_half;
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
// ---------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(256) void k_group_source(SolveArgs<T> a, int g)
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
        double R[Nm];
        harmonics<L>(a.oms[v], a.oms[Vp + v], a.oms[2 * Vp + v], R);
        for (int gp = 0; gp <= g; ++gp) {
            const double pu = a.phiu[gp * Vp + v];
            if (pu == 0.0) continue;
#pragma unroll
            for (int l = 0; l <= L; ++l) {
                const double c = a.xs_s[(((long)m * (L + 1) + l) * G + g) * G + gp] * pu;
#pragma unroll
                for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm) f[lm] += c * R[lm];
            }
        }
        for (int gp = 0; gp < g; ++gp) {
#pragma unroll
            for (int l = 0; l <= L; ++l) {
                const double c = a.xs_s[(((long)m * (L + 1) + l) * G + g) * G + gp];
                if (c == 0.0) continue;
#pragma unroll
                for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm)
                    f[lm] += c * a.phic[((long)gp * Nm + lm) * Vp + v];
            }
        }
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) f[lm] *= rho;
        sg = (T)(rho * a.xs_t[m * G + g]);
    }
    a.sig[v] = sg;
#pragma unroll
    for (int lm = 0; lm < Nm; ++lm) {
        a.F[lm * Vp + v] = f[lm];
        a.phic[((long)g * Nm + lm) * Vp + v] = 0.0;
    }
}

__global__ void k_ctl_init(Ctl *ctl, int g, int target, int max_iters, double tol, int stag_stop)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Ctl c;
    c.iters = 0;
    c.done = target == 0 ? 1 : 0;
    c.target = target;
    c.max_iters = max_iters;
    c.stag_stop = stag_stop;
    c.stag = 0;
    c.status = 0;
    c.pad = 0;
    c.tol = tol;
    c.r = 0.0;
    c.r_prev = 0.0;
    ctl[g] = c;
}

// ---------------------------------------------------------------------------
// a1: scattering source assembly and moment -> direction contraction
// ---------------------------------------------------------------------------
template <typename T, int L>
__global__ __launch_bounds__(256) void k_m2d(SolveArgs<T> a, int g)
{
    constexpr int Nm = (L + 1) * (L + 1);
    if (a.ctl[g].done) return;
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = a.g.Vp;
    if (v >= Vp) return;
    const int G = a.G, D = a.D;
    const int m = a.mat[v];
    T S[Nm];
    if (m == kGhost) {
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) S[lm] = T(0);
    } else {
        const double rho = a.dens[v];
#pragma unroll
        for (int l = 0; l <= L; ++l) {
            const double sl = rho * a.xs_s[(((long)m * (L + 1) + l) * G + g) * G + g];
#pragma unroll
            for (int lm = l * l; lm < (l + 1) * (l + 1); ++lm)
                S[lm] = (T)(a.F[lm * Vp + v] + sl * a.phic[((long)g * Nm + lm) * Vp + v]);
        }
    }
    const T *M0 = a.M0;
    T *out = a.psi + v;
    for (int p = 0; p < D; ++p) {
        T t[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) t[c] = T(0);
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) t[lm_class(lm)] += M0[p * Nm + lm] * S[lm];
        fwht8(t);
#pragma unroll
        for (int o = 0; o < 8; ++o) out[(long)(o * D + p) * Vp] = t[o];
    }
}

// ---------------------------------------------------------------------------
// a2: diamond-difference transport sweep.
//
// One wave = one direction x one pencil (8 x 8 columns of voxels spanning the
// x extent).  Lane (j, k) marches along x with a diagonal skew: at step s it
// updates the voxel with i_r + j_r + k_r = s (octant-relative indices), i.e.
// each step is one sub-sweep plane (section II.B) restricted to the pencil.
// The x inflow stays in a register; y and z inflows are the neighbouring
// lanes' outflows of the previous step (cross-lane permute), or the upstream
// pencil's outgoing face on the pencil boundary.
//
// Memory: the skew makes one step touch 15 different 64-voxel rows, so rows
// are staged through LDS rings and every global access moves whole rows:
//   - Q rows (per wave, RQ slots) are loaded one 8-step chunk ahead into
//     registers, committed to LDS, overwritten in place by psi, and written
//     back as whole rows once all 64 lanes have passed them;
//   - sigma rows are shared by the WPB waves (directions of one octant) of the
//     block, RS slots;
//   - face inflow/outflow rows (8 values each) likewise, RF slots.
// Row r (octant-relative) is needed by steps r .. r+14, so chunk c (steps
// 8c .. 8c+7) needs rows 8c-14 .. 8c+7 and completes rows 8c-14 .. 8c-7.
// One barrier per chunk orders the shared sigma ring (RS = 32 keeps a slot
// free until every wave has left the chunk that last read it).
// Pencils on one diagonal (J_r + K_r = diag) of every octant run in one launch.
// ---------------------------------------------------------------------------
template <typename T, bool FIXUP, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_sweep(SolveArgs<T> a, int g, int diag, int Jlo, int P)
{
    constexpr int RQ = 24, RS = 32, RF = 16, CH = 8;
    __shared__ T sQ[WPB][RQ][64];
    __shared__ T sS[RS][64];
    __shared__ T sFYi[WPB][RF][8], sFZi[WPB][RF][8], sFYo[WPB][RF][8], sFZo[WPB][RF][8];
    if (a.ctl[g].done) return;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int D = a.D, ngrp = D / WPB;
    int item = blockIdx.x;
    const int qd = item % P;
    item /= P;
    const int dg = item % ngrp, o = item / ngrp;
    const int n = o * D + dg * WPB + w;
    const int sx = (o & 1) ? -1 : 1, sy = (o & 2) ? -1 : 1, sz = (o & 4) ? -1 : 1;
    const int NJ = a.g.NJ, NK = a.g.NK, nx = a.g.nx;
    const int Jr = Jlo + qd, Kr = diag - Jr;
    const int J = sy > 0 ? Jr : NJ - 1 - Jr, K = sz > 0 ? Kr : NK - 1 - Kr;
    const int jl = lane & 7, kl = lane >> 3;
    const int jr = sy > 0 ? jl : 7 - jl, kr = sz > 0 ? kl : 7 - kl;
    const int srcY = (lane - sy) & 63, srcZ = (lane - 8 * sz) & 63;
    const T cx = a.cdir[3 * n], cy = a.cdir[3 * n + 1], cz = a.cdir[3 * n + 2];
    const long Vp = a.g.Vp;
    const long pen = (long)K * NJ + J;
    T *psiG = a.psi + (long)n * Vp + pen * nx * 64;
    const T *sigG = a.sig + pen * nx * 64;
    const long fb = (long)n * NJ * NK * nx * 8;
    T *fYo = a.faceY + fb + pen * nx * 8;
    T *fZo = a.faceZ + fb + pen * nx * 8;
    const T *fYi = Jr > 0 ? a.faceY + fb + ((long)K * NJ + (J - sy)) * nx * 8 : nullptr;
    const T *fZi = Kr > 0 ? a.faceZ + fb + ((long)(K - sz) * NJ + J) * nx * 8 : nullptr;
    auto phys = [&](int r) { return sx > 0 ? r : nx - 1 - r; };

    T pq[CH], ps[CH], pfy = T(0), pfz = T(0);
    auto prefetch = [&](int c) {
        const int r0 = CH * c;
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int r = r0 + b;
            if (r < nx) {
                pq[b] = psiG[(long)phys(r) * 64 + lane];
                if (b % WPB == w) ps[b] = sigG[(long)phys(r) * 64 + lane];
            }
        }
        const int r = r0 + (lane >> 3);
        pfy = T(0);
        pfz = T(0);
        if (r < nx) {
            if (fYi) pfy = fYi[(long)phys(r) * 8 + (lane & 7)];
            if (fZi) pfz = fZi[(long)phys(r) * 8 + (lane & 7)];
        }
    };
    auto commit = [&](int c) {
        const int r0 = CH * c;
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int r = r0 + b;
            if (r < nx) {
                sQ[w][r % RQ][lane] = pq[b];
                if (b % WPB == w) sS[r % RS][lane] = ps[b];
            }
        }
        const int r = r0 + (lane >> 3);
        if (r < nx) {
            sFYi[w][r % RF][lane & 7] = pfy;
            sFZi[w][r % RF][lane & 7] = pfz;
        }
    };

    T px = T(0), oy = T(0), oz = T(0);
    const int nchunks = (nx + 6 + CH - 1) / CH + 1;
    prefetch(0);
    for (int c = 0; c < nchunks; ++c) {
        commit(c);
        prefetch(c + 1);
        if (WPB > 1) __syncthreads();
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int ir = CH * c + b - jr - kr;
            const bool act = ir >= 0 && ir < nx;
            T iny = __shfl(oy, srcY);
            T inz = __shfl(oz, srcZ);
            if (act) {
                const int sq = ir % RQ, sf = ir % RF;
                const T q = sQ[w][sq][lane];
                const T sg = sS[ir % RS][lane];
                if (jr == 0) iny = sFYi[w][sf][kl];
                if (kr == 0) inz = sFZi[w][sf][jl];
                T p = dd_div<T>(q + cx * px + cy * iny + cz * inz, sg + cx + cy + cz);
                T ox_ = T(2) * p - px, oy_ = T(2) * p - iny, oz_ = T(2) * p - inz;
                if (FIXUP && (ox_ < T(0) || oy_ < T(0) || oz_ < T(0))) {
                    // set-to-zero: fixed axes get zero outflow, balance re-solved
                    bool fx = false, fyx = false, fzx = false;
#pragma unroll
                    for (int pass = 0; pass < 3; ++pass) {
                        bool grew = false;
                        if (!fx && ox_ < T(0)) { fx = true; grew = true; }
                        if (!fyx && oy_ < T(0)) { fyx = true; grew = true; }
                        if (!fzx && oz_ < T(0)) { fzx = true; grew = true; }
                        if (!grew) break;
                        T num = q, den = sg;
                        if (fx) num += T(0.5) * cx * px; else { num += cx * px; den += cx; }
                        if (fyx) num += T(0.5) * cy * iny; else { num += cy * iny; den += cy; }
                        if (fzx) num += T(0.5) * cz * inz; else { num += cz * inz; den += cz; }
                        p = dd_div<T>(num, den);
                        ox_ = fx ? T(0) : T(2) * p - px;
                        oy_ = fyx ? T(0) : T(2) * p - iny;
                        oz_ = fzx ? T(0) : T(2) * p - inz;
                    }
                }
                sQ[w][sq][lane] = p;
                if (jr == 7) sFYo[w][sf][kl] = oy_;
                if (kr == 7) sFZo[w][sf][jl] = oz_;
                px = ox_;
                oy = oy_;
                oz = oz_;
            }
        }
        // rows 8c-14 .. 8c-7 are complete: write them back as whole rows
#pragma unroll
        for (int b = 0; b < CH; ++b) {
            const int r = CH * c - 14 + b;
            if (r >= 0 && r < nx) psiG[(long)phys(r) * 64 + lane] = sQ[w][r % RQ][lane];
        }
        const int r = CH * c - 14 + (lane >> 3);
        if (r >= 0 && r < nx) {
            fYo[(long)phys(r) * 8 + (lane & 7)] = sFYo[w][r % RF][lane & 7];
            fZo[(long)phys(r) * 8 + (lane & 7)] = sFZo[w][r % RF][lane & 7];
        }
    }
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

template <typename T, int L>
__global__ __launch_bounds__(256) void k_d2m(SolveArgs<T> a, int g)
{
    constexpr int Nm = (L + 1) * (L + 1);
    if (a.ctl[g].done) return;
    const long v = blockIdx.x * 256L + threadIdx.x;
    const long Vp = a.g.Vp;
    const int D = a.D;
    double d2 = 0.0, n2 = 0.0;
    if (v < Vp) {
        double acc[Nm];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) acc[lm] = 0.0;
        const T *in = a.psi + v;
        const double *D0 = a.D0;
        for (int p = 0; p < D; ++p) {
            double x[8];
#pragma unroll
            for (int o = 0; o < 8; ++o) x[o] = (double)in[(long)(o * D + p) * Vp];
            fwht8(x);
#pragma unroll
            for (int lm = 0; lm < Nm; ++lm) acc[lm] += D0[p * Nm + lm] * x[lm_class(lm)];
        }
        double *ph = a.phic + (long)g * Nm * Vp + v;
        const double old = ph[0];
#pragma unroll
        for (int lm = 0; lm < Nm; ++lm) ph[(long)lm * Vp] = acc[lm];
        const double dd = acc[0] - old;
        d2 = dd * dd;
        n2 = acc[0] * acc[0];
    }
    __shared__ double red[2][4];
    d2 = wave_sum(d2);
    n2 = wave_sum(n2);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = d2; red[1][w] = n2; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        a.part[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

__global__ __launch_bounds__(256) void k_resid(Ctl *ctl, int g, const double *part, int nblk)
{
    if (ctl[g].done) return;
    double s0 = 0.0, s1 = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        s0 += part[2 * b];
        s1 += part[2 * b + 1];
    }
    __shared__ double red[2][4];
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = s0; red[1][w] = s1; }
    __syncthreads();
    if (threadIdx.x != 0) return;
    s0 = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    s1 = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    Ctl c = ctl[g];
    double r;
    if (s1 == 0.0) r = s0 == 0.0 ? 0.0 : INFINITY;
    else r = sqrt(s0) / sqrt(s1);
    c.iters += 1;
    c.r_prev = c.r;
    c.r = r;
    if (c.target >= 0) {
        if (c.iters >= c.target) c.done = 1;
    } else if (isnan(r)) {
        c.done = 1;
        c.status = 6;
    } else if (r < c.tol) {
        c.done = 1;
        c.status = 0;
    } else {
        if (c.stag_stop && c.iters > 1 && r >= c.r_prev) {
            if (++c.stag >= 3) { c.done = 1; c.status = 7; }
        } else {
            c.stag = 0;
        }
        if (!c.done && c.iters >= c.max_iters) { c.done = 1; c.status = 5; }
    }
    ctl[g] = c;
}

// ---------------------------------------------------------------------------
// a6: total fluence of group g into the caller's natural-order buffers
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_finalize(SolveArgs<T> a, int g, double *phi_total, double *phi_unc)
{
    const long v = blockIdx.x * 256L + threadIdx.x;
    const Geom &gm = a.g;
    if (v >= gm.V) return;
    const int i = (int)(v % gm.nx), j = (int)((v / gm.nx) % gm.ny), k = (int)(v / ((long)gm.nx * gm.ny));
    const long vp = pencil_index(gm, i, j, k);
    const double pu = a.phiu[(long)g * gm.Vp + vp];
    phi_total[(long)g * gm.V + v] = pu + a.phic[(long)g * a.Nm * gm.Vp + vp];
    if (phi_unc) phi_unc[(long)g * gm.V + v] = pu;
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
void launch_raytrace(const SolveArgs<T> &a, const double pos[3], const double axis[3], double cos_half, int iso,
                     const double *spec, hipStream_t s)
{
    hipLaunchKernelGGL(k_raytrace<T>, dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, pos[0], pos[1], pos[2], axis[0],
                       axis[1], axis[2], cos_half, iso, spec);
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
void launch_group_source(const SolveArgs<T> &a, int g, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_group_source<T, LL>), dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, g));
}

void launch_ctl_init(Ctl *ctl, int g, int target, int max_iters, double tol, int stag_stop, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_init, dim3(1), dim3(64), 0, s, ctl, g, target, max_iters, tol, stag_stop);
}

template <typename T>
int launch_m2d(const SolveArgs<T> &a, int g, hipStream_t s)
{
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_m2d<T, LL>), dim3(nblk(a.g.Vp)), dim3(256), 0, s, a, g));
    return 1;
}

// Waves per block: directions of one octant that share a pencil's sigma rows.
inline int sweep_wpb(int D, bool fp64)
{
    if (D % 4 == 0 && !fp64) return 4;
    if (D % 2 == 0) return 2;
    return 1;
}

template <typename T, bool FIXUP, int WPB>
static void launch_sweep_diags(const SolveArgs<T> &a, int g, hipStream_t s)
{
    const int NJ = a.g.NJ, NK = a.g.NK;
    for (int d = 0; d <= NJ + NK - 2; ++d) {
        const int Jlo = d - (NK - 1) > 0 ? d - (NK - 1) : 0;
        const int Jhi = d < NJ - 1 ? d : NJ - 1;
        const int P = Jhi - Jlo + 1;
        const unsigned blocks = (unsigned)(P * 8 * (a.D / WPB));
        hipLaunchKernelGGL((k_sweep<T, FIXUP, WPB>), dim3(blocks), dim3(64 * WPB), 0, s, a, g, d, Jlo, P);
    }
}

template <typename T>
int launch_sweeps(const SolveArgs<T> &a, int g, int fixup, hipStream_t s)
{
    const int wpb = sweep_wpb(a.D, sizeof(T) == 8);
    if (fixup) {
        if (wpb == 4) launch_sweep_diags<T, true, 4>(a, g, s);
        else if (wpb == 2) launch_sweep_diags<T, true, 2>(a, g, s);
        else launch_sweep_diags<T, true, 1>(a, g, s);
    } else {
        if (wpb == 4) launch_sweep_diags<T, false, 4>(a, g, s);
        else if (wpb == 2) launch_sweep_diags<T, false, 2>(a, g, s);
        else launch_sweep_diags<T, false, 1>(a, g, s);
    }
    return a.g.NJ + a.g.NK - 1;
}

template <typename T>
int launch_d2m(const SolveArgs<T> &a, int g, hipStream_t s)
{
    const unsigned nb = nblk(a.g.Vp);
    DSN_DISPATCH_L(a.L, hipLaunchKernelGGL((k_d2m<T, LL>), dim3(nb), dim3(256), 0, s, a, g));
    hipLaunchKernelGGL(k_resid, dim3(1), dim3(256), 0, s, a.ctl, g, (const double *)a.part, (int)nb);
    return 2;
}

template <typename T>
void launch_finalize(const SolveArgs<T> &a, int g, double *phi_total, double *phi_unc, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize<T>, dim3(nblk(a.g.V)), dim3(256), 0, s, a, g, phi_total, phi_unc);
}

template void launch_raytrace<float>(const SolveArgs<float> &, const double *, const double *, double, int,
                                     const double *, hipStream_t);
template void launch_raytrace<double>(const SolveArgs<double> &, const double *, const double *, double, int,
                                      const double *, hipStream_t);
template void launch_group_source<float>(const SolveArgs<float> &, int, hipStream_t);
template void launch_group_source<double>(const SolveArgs<double> &, int, hipStream_t);
template int launch_m2d<float>(const SolveArgs<float> &, int, hipStream_t);
template int launch_m2d<double>(const SolveArgs<double> &, int, hipStream_t);
template int launch_sweeps<float>(const SolveArgs<float> &, int, int, hipStream_t);
template int launch_sweeps<double>(const SolveArgs<double> &, int, int, hipStream_t);
template int launch_d2m<float>(const SolveArgs<float> &, int, hipStream_t);
template int launch_d2m<double>(const SolveArgs<double> &, int, hipStream_t);
template void launch_finalize<float>(const SolveArgs<float> &, int, double *, double *, hipStream_t);
template void launch_finalize<double>(const SolveArgs<double> &, int, double *, double *, hipStream_t);

}  // namespace dsn
