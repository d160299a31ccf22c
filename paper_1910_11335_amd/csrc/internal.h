// Internal declarations shared by the library's kernels and its host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsn {

// Voxels are stored on the device in "pencil" order: the (j, k) plane is cut
// into 8 x 8 column blocks; a pencil is one column block over the full x
// extent, and inside it voxel (i, j, k) sits at row i, lane (j & 7) + 8 (k & 7):
//   v' = ((K * NJ + J) * nx + i) * 64 + (j & 7) + 8 * (k & 7),  J = j/8, K = k/8.
// ny and nz are padded up to multiples of 8 with ghost voxels (no material,
// zero source, zero cross section) that only ever carry zero fluence.
constexpr int kCB = 8;
constexpr int kLanes = 64;
constexpr uint8_t kGhost = 0xFF;
constexpr int kMaxMat = 16;
constexpr int kMaxL = 5;

struct Geom {
    int nx, ny, nz;     // real mesh
    int NJ, NK;         // pencils along y and z
    long Vp;            // padded voxel count = NJ * NK * nx * 64
    long V;             // real voxel count
    double dx, dy, dz;
};

// Per-group iteration state kept on the device so that converged groups make
// every later kernel of the same group return at once.
struct Ctl {
    int iters;      // source iterations done
    int done;       // 1: stop iterating
    int target;     // fixed iteration count, or -1
    int max_iters;
    int stag_stop;  // stop after 3 iterations without a new smallest residual
    int stag;       // iterations since the smallest residual so far
    int status;     // 0 converged/fixed, 5 max_iters, 6 NaN or infinite, 7 stagnated
    int rule;       // 0: stop when r < tol; 1: stop when the estimated per-voxel error est < tol
    double tol;
    double r;       // last relative L2 change of phi_00
    double r_prev;
    double tmax;    // largest |phi_u + phi_00| of the last iterate (rule 1)
    double est;     // rule 1: estimated per-voxel error left after the last iterate
    double rmin;    // smallest r (rule 1: est) so far, for the stagnation stop
};

// Angular arrays (psi, which holds the directional source Q until the sweep
// overwrites it) are pencil-major: pencil after pencil (8 x 8 columns along
// x, nx * 64 voxels in the voxel order of every per-voxel array), that
// pencil's nx * 64 values of direction 0, then of direction 1, and so on.
// One pencil-direction is one contiguous run (what a sweep wave streams) and
// a pencil's Nd runs are adjacent (what the moments pass streams).
// psi_run: first value of pencil pen, direction n; psi_index: value (0, v),
// so that value (n, v) sits at psi_index + n * nx * 64.
__host__ __device__ inline long psi_run(long pen, int Nd, int n, int nx)
{
    return (pen * Nd + n) * ((long)nx * 64);
}
__host__ __device__ inline long psi_index(const Geom &g, int Nd, long v)
{
    const long PL = (long)g.nx * 64;
    return v + (v / PL) * (long)(Nd - 1) * PL;
}

constexpr int kSrcPar = 12;  // doubles of source parameters per source

// Per-solve argument block for the kernels (all device pointers).
template <typename T>
struct SolveArgs {
    Geom g;
    int G, L, Nm, Nd, D, nmat;
    const uint8_t *mat;       // [Vp] pencil order, kGhost for ghosts
    const double *dens;       // [Vp]
    const uint8_t *mat_nat;   // [V] natural order (ray trace)
    const double *dens_nat;   // [V] natural order, or null
    const double *xs_t;       // [nmat][G]
    const double *xs_s;       // [nmat][L+1][G][G]
    const T *M0;              // [D][Nm] (2l+1)/(4 pi) R_lm(Omega_{0,p})
    const double *D0;         // [D][Nm] w_p R_lm(Omega_{0,p})
    const T *cdir;            // [Nd][3] 2|Omega_a|/Delta_a
    double *phiu;             // [G][Vp] uncollided fluence
    double *oms;              // [3][Vp] unit direction source -> voxel
    double *phic;             // [G][Nm][Vp] collided moments, all groups
    T *F;                     // [Nm][Vp] external moments of the current group (they only enter the
                              // directional source, which is formed in T)
    const double *usum;       // [G][Nm][Vp] summed uncollided moments of sources acting together, or null
    T *sig;                   // [Vp] rho * sigma_t of the current group
    T *psi;                   // [NJ*NK][Nd][nx*64] Q, then psi, in place (pencil-major: psi_index)
    unsigned long long *faceY, *faceZ;  // [Nd][NJ*NK][nx][8][words]: tagged face values
    double *part;             // [n_blocks][4] residual partials: two sums (L2), two maxima (rule 1)
    Ctl *ctl;                 // [G]
    // persistent sweep work queue
    int *sweep_ctr;           // [3]: next ticket, abort flag, epoch of the current sweep
    int *face_par;            // [S]: sign-bit parity of the next sweep's face words
    const int *sweep_dstart;  // [NJ+NK] first ticket of each pencil diagonal (+ total)
    int sweep_nitems;
    int sweep_grid;           // blocks launched
    int sweep_wpb;            // waves per block: directions of an octant sharing a pencil item
    int sweep_xcd;            // > 0: per-XCD ticket queues (octant o on XCD o mod sweep_xcd), faces in L2
    int sweep_relay;          // > 0: column-relay sweep with this many roles (pencils handed over in LDS)
    int sweep_mode;           // cell mode: 0 DD, 1 fixup, 2 fixup recording the fixed axes into mask,
                              // 3 transposed fixup cell with the fixed axes read from mask (adjoint)
    uint8_t *mask;            // [Nd][Vp] fixed-axis sets (modes 2 and 3), else null
    int sweep_spin_limit;     // polls before a wait gives up
    int sig_from_mat;         // 1: sigma_t = xs_t[material] (no density), the sweep reads the material byte
    int stream_nt;            // 1: the angular fluence of a launch exceeds the last-level cache, so its
                              // streamed arrays are read and written non-temporally
    int rev;                  // 1: sweep every direction along -Omega (adjoint)
    const double *wdir;       // [Nd] quadrature weights (gradient)
    // source batch: S independent sources of this problem advance together;
    // every per-source array above is [S][...] with these element strides
    int S;
    long str_psi, str_phic, str_phiu, str_oms, str_F, str_face, str_part;
    const double *src_par;    // [S][kSrcPar]: position xyz, axis xyz, cos(half angle), isotropic flag,
                              // fan-plane unit normal xyz (orthogonal to the axis), sin(fan half thickness)
                              // (< 0: a cone, no fan)
    const double *src_spec;   // [S][G]
    // several problems (meshes) in one sweep launch: their own argument
    // blocks, and the merged ticket order over them.  seg holds nseg + 1
    // segment starts (ascending tickets; the last is the total), then nseg
    // codes (problem << 16 | pencil diagonal).  Segments go diagonal by
    // diagonal over all problems, so every item's upstream items (the
    // previous diagonal of its own problem) hold smaller tickets.
    const SolveArgs<T> *multi;  // [nmulti], or null
    int nmulti;
    const int *seg;
    int nseg;
};

// The sweep runs as column-relay items: relay roles set, a forward cell mode
// (pure DD or the fixup) and directions along +Omega.  Other sweeps of a
// handle with such a shape (the adjoint's) use pencil items of the same
// directions per block.
template <typename T>
__host__ __device__ inline bool sweep_uses_col(const SolveArgs<T> &a)
{
    return a.sweep_relay > 0 && (a.sweep_mode == 0 || a.sweep_mode == 1) && !a.rev;
}

// The per-source view of a batched argument block.
template <typename T>
__host__ __device__ inline SolveArgs<T> at_source(SolveArgs<T> a, int s)
{
    if (s) {
        a.psi += s * a.str_psi;
        a.phic += s * a.str_phic;
        a.phiu += s * a.str_phiu;
        a.oms += s * a.str_oms;
        a.F += s * a.str_F;
        a.faceY += s * a.str_face;
        a.faceZ += s * a.str_face;
        a.part += s * a.str_part;
        a.ctl += (long)s * a.G;
        a.src_par += (long)kSrcPar * s;
        a.face_par += s;
        a.src_spec += (long)s * a.G;
    }
    return a;
}

}  // namespace dsn

namespace dsn {

// launchers (kernels.hip)
void launch_voxels_to_pencils(const Geom &g, const uint8_t *mat_nat, const double *dens_nat, uint8_t *mat,
                              double *dens, hipStream_t s);
template <typename T>
void launch_raytrace(const SolveArgs<T> &a, hipStream_t s);
template <typename T>
void launch_group_source(const SolveArgs<T> &a, int g, bool expand, hipStream_t s);
template <typename T>
void launch_sum_uncollided(const SolveArgs<T> &a, int nsrc, double *usum, double *pusum, hipStream_t s);
void launch_ctl_init(Ctl *ctl, int G, int nsrc, int g, int target, int max_iters, double tol, int stag_stop,
                     int rule, hipStream_t s);
template <typename T>
int launch_m2d(const SolveArgs<T> &a, int g, hipStream_t s);
int sweep_wpb(int D, bool fp64);
int sweep_wpb_choices(bool fp64, int *out);  // waves-per-block values built; returns the count (<= 16)
template <typename T>
int sweep_grid(int wpb, int mode, int n_cu);
int sweep_col_choices(bool fp64, int *w_out, int *r_out);  // (directions, roles) of the built column-relay sweeps
template <typename T>
int sweep_grid_col(int w, int r, int mode, int nx, int n_cu);
// ev_before / ev_after (may be null): recorded on s right around the sweep
// kernel itself (after the ticket reset, before the parity flip)
template <typename T>
int launch_sweeps(const SolveArgs<T> &a, int g, hipStream_t s, hipEvent_t ev_before = nullptr,
                  hipEvent_t ev_after = nullptr);
// fused batches: several problems in one sweep launch
int sweep_multi_choices(bool fp64, int *out);
template <typename T>
int sweep_grid_multi(int wpb, int mode, int n_cu);
template <typename T>
int launch_sweep_multi(const SolveArgs<T> &a, const SolveArgs<T> *host_tab, int n, int g, hipStream_t s,
                       hipEvent_t ev_before = nullptr, hipEvent_t ev_after = nullptr);
bool sweep_xcd_supported(bool fp64, int mode, int wpb);  // a per-XCD-queue sweep kernel is built
bool sweep_tagged_faces(bool fp64, int mode, int wpb, int xcd);  // the launch uses tagged (not sign-parity) words
void launch_xcc_probe(int *out, int n, hipStream_t s);    // out[b] = XCD of workgroup b, b < n
void launch_checksum(const void *x, long n_words, unsigned long long *out, hipStream_t s);  // adds to *out
template <typename T>
int launch_d2m(const SolveArgs<T> &a, int g, bool expand, hipStream_t s);
template <typename T>  // every (problem, source) pair of a fused batch
int launch_d2m_multi(const SolveArgs<T> *tab, const SolveArgs<T> &a, int n, long vp_max, int s_max, bool nt, int g,
                     hipStream_t s);
template <typename T>
void launch_finalize(const SolveArgs<T> &a, int g, double *phi_total, double *phi_unc, hipStream_t s);
// adjoint (kernels.hip)
template <typename T>
void launch_group_source_keep(const SolveArgs<T> &a, int g, hipStream_t s);
template <typename T>
void launch_adj_source(const SolveArgs<T> &a, int g, const double *W, int zero_phi, hipStream_t s);
template <typename T>
void launch_m2d_always(const SolveArgs<T> &a, int g, hipStream_t s);
template <typename T>
void launch_grad_accum(const SolveArgs<T> &fw, const SolveArgs<T> &ad, int g, double *grad, hipStream_t s);
template <typename T>
void launch_backproject(const SolveArgs<T> &fw, const double *phia, const double *W, const double pos[3],
                        double *grad, hipStream_t s);
void launch_dot(const double *x, const double *y, long n, double *part, int nblk, double *out, hipStream_t s);
void launch_dose(const uint8_t *mat, long V, int G, const double *phi, const double *k, int n, double *dose,
                 hipStream_t s);

}  // namespace dsn
