// Level-symmetric S_N quadrature, derived on the host in extended precision.
//
// The paper (section II.E) uses S2..S8 sets with N(N+2) directions and the
// weights of eq. 3 but prints no values.  This library takes the
// level-symmetric LQn family and re-derives it from its moment conditions:
//   levels      mu_i^2 = mu_1^2 + (i-1) 2(1 - 3 mu_1^2)/(N-2), i = 1..N/2
//   points      (mu_a, mu_b, mu_c), a+b+c = N/2+2 (1-based), one octant
//   weights     one per permutation class, sum_p w_p mu_p^(2k) = 1/(2k+1)
//               for k = 0, 2, ..., N/2 (per octant, weights summing to 1)
//   mu_1        the value making that over-determined system consistent:
//               a sign change of det[A | b] (S4..S12) or of the Cramer
//               determinant with the last class column replaced by b (S16,
//               whose class matrix has rank 7 everywhere)
//   S16 weights the system leaves a line of solutions; the point nearest the
//               7-digit weights of the standard LQn table is taken
//               (projection onto the affine solution set).
// Everything runs in long double (64-bit mantissa); the result is rounded to
// double once.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "quadrature.h"

namespace dsn {
namespace {

typedef long double ld;
typedef std::vector<std::vector<ld>> Mat;

struct Tri { int a, b, c; };

std::vector<Tri> octant_points(int N)
{
    const int n = N / 2;
    std::vector<Tri> p;
    for (int a = 1; a <= n; ++a)
        for (int b = 1; b <= n + 1 - a; ++b) p.push_back({a, b, n + 2 - a - b});
    return p;
}

Tri sorted3(Tri t)
{
    int v[3] = {t.a, t.b, t.c};
    std::sort(v, v + 3);
    return {v[0], v[1], v[2]};
}

bool operator<(const Tri &x, const Tri &y)
{
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    return x.c < y.c;
}

std::vector<ld> levels_sq(int N, ld mu1)
{
    const int n = N / 2;
    std::vector<ld> x(n);
    if (N == 2) { x[0] = 1.0L / 3.0L; return x; }
    const ld d = 2.0L * (1.0L - 3.0L * mu1 * mu1) / (ld)(N - 2);
    for (int i = 0; i < n; ++i) x[i] = mu1 * mu1 + (ld)i * d;
    return x;
}

// Moment system A w = b over the permutation classes.
void class_system(int N, ld mu1, Mat &A, std::vector<ld> &b, std::vector<Tri> &classes)
{
    std::vector<Tri> pts = octant_points(N);
    std::map<Tri, int> idx;
    for (const Tri &p : pts) idx.emplace(sorted3(p), 0);
    classes.clear();
    for (auto &kv : idx) { kv.second = (int)classes.size(); classes.push_back(kv.first); }
    std::vector<int> ks = {0};
    for (int k = 2; k <= N / 2; ++k) ks.push_back(k);
    std::vector<ld> x = levels_sq(N, mu1);
    A.assign(ks.size(), std::vector<ld>(classes.size(), 0.0L));
    b.assign(ks.size(), 0.0L);
    for (size_t r = 0; r < ks.size(); ++r) {
        for (const Tri &p : pts) A[r][idx[sorted3(p)]] += std::pow(x[p.a - 1], (ld)ks[r]);
        b[r] = 1.0L / (ld)(2 * ks[r] + 1);
    }
}

// Determinant by Gaussian elimination with partial pivoting.
ld det(Mat M)
{
    const int n = (int)M.size();
    ld d = 1.0L;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0L) return 0.0L;
        if (piv != c) { std::swap(M[piv], M[c]); d = -d; }
        d *= M[c][c];
        for (int r = c + 1; r < n; ++r) {
            ld f = M[r][c] / M[c][c];
            for (int k = c; k < n; ++k) M[r][k] -= f * M[c][k];
        }
    }
    return d;
}

// Solves the square system M x = y (partial pivoting); false if singular.
bool solve(Mat M, std::vector<ld> y, std::vector<ld> &x)
{
    const int n = (int)M.size();
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
        if (M[piv][c] == 0.0L) return false;
        std::swap(M[piv], M[c]);
        std::swap(y[piv], y[c]);
        for (int r = c + 1; r < n; ++r) {
            ld f = M[r][c] / M[c][c];
            for (int k = c; k < n; ++k) M[r][k] -= f * M[c][k];
            y[r] -= f * y[c];
        }
    }
    x.assign(n, 0.0L);
    for (int r = n - 1; r >= 0; --r) {
        ld s = y[r];
        for (int k = r + 1; k < n; ++k) s -= M[r][k] * x[k];
        x[r] = s / M[r][r];
    }
    return true;
}

ld consistency(int N, ld mu1)
{
    Mat A;
    std::vector<ld> b;
    std::vector<Tri> cl;
    class_system(N, mu1, A, b, cl);
    const size_t rows = A.size(), cols = cl.size();
    if (rows == cols + 1) {
        for (size_t r = 0; r < rows; ++r) A[r].push_back(b[r]);
        return det(A);
    }
    // square, rank-deficient: Cramer determinant with the last column <- b
    for (size_t r = 0; r < rows; ++r) A[r][cols - 1] = b[r];
    return det(A);
}

// 7-digit S16 class weights (per point, octant sum 1) of the standard LQn
// table; only used to pick a point on the S16 solution line.
ld s16_anchor(const Tri &t)
{
    static const struct { int a, b, c; double w; } tab[] = {
        {1, 1, 8, 0.0489872}, {1, 2, 7, 0.0413296}, {1, 3, 6, 0.0212326}, {1, 4, 5, 0.0256206},
        {2, 2, 6, 0.0360485}, {2, 3, 5, 0.0144590}, {2, 4, 4, 0.0344958}, {3, 3, 4, 0.0085181}};
    for (const auto &e : tab)
        if (e.a == t.a && e.b == t.b && e.c == t.c) return (ld)e.w;
    return 0.0L;
}

}  // namespace

bool lqn_supported(int N)
{
    return N == 2 || N == 4 || N == 6 || N == 8 || N == 10 || N == 12 || N == 16;
}

bool lqn_build(int N, std::vector<double> &omega, std::vector<double> &w, std::string &err)
{
    if (!lqn_supported(N)) { err = "S_N order must be one of 2,4,6,8,10,12,16"; return false; }
    std::vector<Tri> pts = octant_points(N);
    ld mu1 = std::sqrt(1.0L / 3.0L);
    std::vector<ld> cw;  // per-class weight (octant sum 1)
    std::vector<Tri> classes;
    if (N == 2) {
        classes = {sorted3(pts[0])};
        cw = {1.0L};
    } else {
        // bracket around the standard tabulated values, then bisect
        static const std::map<int, double> guess = {{4, 0.3500212}, {6, 0.2666355}, {8, 0.2182179},
                                                    {10, 0.1893213}, {12, 0.1672126}, {16, 0.1389568}};
        ld g = (ld)guess.at(N);
        ld lo = g * (1.0L - 1e-4L), hi = g * (1.0L + 1e-4L);
        ld flo = consistency(N, lo), fhi = consistency(N, hi);
        if (!((flo < 0) != (fhi < 0))) { err = "LQn mu_1 root not bracketed"; return false; }
        for (int it = 0; it < 200; ++it) {
            ld mid = 0.5L * (lo + hi);
            if (mid <= lo || mid >= hi) break;
            ld fm = consistency(N, mid);
            if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else hi = mid;
        }
        mu1 = 0.5L * (lo + hi);
        Mat A;
        std::vector<ld> b;
        class_system(N, mu1, A, b, classes);
        const size_t nc = classes.size();
        if (A.size() == nc + 1) {
            Mat S(A.begin(), A.begin() + nc);
            std::vector<ld> y(b.begin(), b.begin() + nc);
            if (!solve(S, y, cw)) { err = "LQn weight system singular"; return false; }
        } else {
            // rank-deficient square system: drop one dependent row r, then
            // w = a + Ar^T (Ar Ar^T)^-1 (br - Ar a), the nearest solution to a
            std::vector<ld> a(nc);
            for (size_t c = 0; c < nc; ++c) a[c] = s16_anchor(classes[c]);
            bool ok = false;
            for (int r = (int)A.size() - 1; r >= 0 && !ok; --r) {
                Mat Ar;
                std::vector<ld> br;
                for (int q = 0; q < (int)A.size(); ++q)
                    if (q != r) { Ar.push_back(A[q]); br.push_back(b[q]); }
                const size_t m = Ar.size();
                Mat G(m, std::vector<ld>(m, 0.0L));
                std::vector<ld> rhs(m, 0.0L);
                for (size_t i = 0; i < m; ++i) {
                    for (size_t j = 0; j < m; ++j)
                        for (size_t c = 0; c < nc; ++c) G[i][j] += Ar[i][c] * Ar[j][c];
                    rhs[i] = br[i];
                    for (size_t c = 0; c < nc; ++c) rhs[i] -= Ar[i][c] * a[c];
                }
                std::vector<ld> lam;
                if (!solve(G, rhs, lam)) continue;
                std::vector<ld> wt(a);
                for (size_t c = 0; c < nc; ++c)
                    for (size_t i = 0; i < m; ++i) wt[c] += Ar[i][c] * lam[i];
                // accept only if the full system is satisfied
                ld res = 0.0L;
                for (size_t q = 0; q < A.size(); ++q) {
                    ld s = -b[q];
                    for (size_t c = 0; c < nc; ++c) s += A[q][c] * wt[c];
                    res = std::max(res, std::fabs(s));
                }
                if (res < 1e-15L) { cw = wt; ok = true; }
            }
            if (!ok) { err = "S16 weight projection failed"; return false; }
        }
    }
    std::vector<ld> x = levels_sq(N, mu1);
    std::map<Tri, ld> wmap;
    for (size_t c = 0; c < classes.size(); ++c) wmap[classes[c]] = cw[c];
    const int D = (int)pts.size();
    omega.assign((size_t)8 * D * 3, 0.0);
    w.assign((size_t)8 * D, 0.0);
    const ld half_pi = 1.5707963267948966192313216916397514L;
    for (int o = 0; o < 8; ++o) {
        const ld s[3] = {(o & 1) ? -1.0L : 1.0L, (o & 2) ? -1.0L : 1.0L, (o & 4) ? -1.0L : 1.0L};
        for (int p = 0; p < D; ++p) {
            const int n = o * D + p;
            omega[3 * n + 0] = (double)(s[0] * std::sqrt(x[pts[p].a - 1]));
            omega[3 * n + 1] = (double)(s[1] * std::sqrt(x[pts[p].b - 1]));
            omega[3 * n + 2] = (double)(s[2] * std::sqrt(x[pts[p].c - 1]));
            w[n] = (double)(wmap[sorted3(pts[p])] * half_pi);
        }
    }
    return true;
}

}  // namespace dsn
