// Host runtime and C ABI of the discrete-ordinates library (include/dsn.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "dsn.h"
#include "internal.h"
#include "quadrature.h"

using namespace dsn;

namespace {

thread_local std::string g_err;

dsn_status fail(dsn_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define DSN_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? DSN_ERR_OUT_OF_MEMORY : DSN_ERR_DEVICE,   \
                        std::string(#call) + ": " + hipGetErrorString(e_));                  \
    } while (0)

// Real harmonics on the host (same definition as the device kernels):
// Schmidt semi-normalised, no Condon-Shortley phase, lm = l*l + l + m.
void host_harmonics(int L, double mu, double eta, double xi, double *R)
{
    double C[kMaxL + 1], S[kMaxL + 1], P[kMaxL + 1][kMaxL + 1];
    C[0] = 1.0;
    S[0] = 0.0;
    for (int m = 1; m <= L; ++m) {
        C[m] = C[m - 1] * mu - S[m - 1] * eta;
        S[m] = S[m - 1] * mu + C[m - 1] * eta;
    }
    for (int m = 0; m <= L; ++m) {
        double dfac = 1.0;
        for (int t = 2 * m - 1; t > 1; t -= 2) dfac *= (double)t;
        P[m][m] = dfac;
        if (m + 1 <= L) P[m + 1][m] = (2.0 * m + 1.0) * xi * P[m][m];
        for (int l = m + 2; l <= L; ++l)
            P[l][m] = ((2.0 * l - 1.0) * xi * P[l - 1][m] - (l + m - 1.0) * P[l - 2][m]) / (double)(l - m);
    }
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) {
            const int am = m < 0 ? -m : m;
            double ratio = 1.0;
            for (int t = l - am + 1; t <= l + am; ++t) ratio /= (double)t;
            R[l * l + l + m] = std::sqrt((am == 0 ? 1.0 : 2.0) * ratio) * P[l][am] * (m >= 0 ? C[am] : S[am]);
        }
}

int host_lm_class(int lm)
{
    int l = 0;
    while ((l + 1) * (l + 1) <= lm) ++l;
    const int m = lm - l * l - l, am = m < 0 ? -m : m;
    const int xo = m >= 0 ? (am & 1) : ((am & 1) ^ 1);
    const int yo = m < 0 ? 1 : 0;
    const int zo = (l + am) & 1;
    return xo | (yo << 1) | (zo << 2);
}

bool finite_all(const double *x, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

}  // namespace

// Stage timer: HIP event pairs recorded on the solve stream around each
// stage, summed after the stream is synchronised.
struct StageTimer {
    bool on = false;
    hipStream_t s = 0;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<int> stage_of, iter_of, nl_of;  // per event pair: stage, source iteration (-1: none), launches
    int cur_iter = -1;                          // source iteration being enqueued
    double ms[DSN_NUM_STAGES] = {0, 0, 0, 0};
    int64_t launches[DSN_NUM_STAGES] = {0, 0, 0, 0};

    hipEvent_t next()
    {
        if (used == pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
    size_t begin()
    {
        if (!on) return 0;
        size_t i = used;
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, s);
        return i;
    }
    // a pair of events that the caller records itself, around one kernel
    // inside a stage (the sweep kernel without its small set-up and parity
    // kernels); false with the timer off
    bool pair(int stage, int nl, hipEvent_t &b, hipEvent_t &e)
    {
        if (!on) return false;
        b = next();
        e = next();
        stage_of.push_back(stage);
        iter_of.push_back(cur_iter);
        nl_of.push_back(nl);
        return b && e;
    }
    void end(int stage, size_t i, int nl)
    {
        if (!on) return;
        hipEvent_t e = next();
        if (e) (void)hipEventRecord(e, s);
        stage_of.push_back(stage);
        iter_of.push_back(cur_iter);
        nl_of.push_back(nl);
        (void)i;
    }
    // Call with the stream synchronised.  Iterations from `iters` on were
    // enqueued ahead of the convergence check and found nothing to do: they
    // are dropped, so the totals cover exactly the work done.
    void flush(int iters = 1 << 30)
    {
        if (!on) return;
        for (size_t k = 0; k < stage_of.size(); ++k) {
            if (iter_of[k] >= iters) continue;
            float t = 0.f;
            if (2 * k + 1 < used && hipEventElapsedTime(&t, pool[2 * k], pool[2 * k + 1]) == hipSuccess)
                ms[stage_of[k]] += t;
            launches[stage_of[k]] += nl_of[k];
        }
        stage_of.clear();
        iter_of.clear();
        nl_of.clear();
        used = 0;
    }
    void release()
    {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
        used = 0;
    }
};

// A launch shape of the sweep and its measured time.
struct SweepShape {
    int wpb = 0, blocks = 0, xcd = 0;  // xcd: per-XCD queues (0 = one global queue)
    float ms = 0.f;                    // < 0: its angular fluence differed from the default shape's (not used)
    int relay = 0;                     // > 0: column-relay sweep with wpb directions and this many roles per block
};
constexpr int kMaxWpb = 16;     // waves per block: largest value built is below this
constexpr int kMaxShapes = 64;  // (waves-per-block choices + per-XCD-queue + column-relay variants) x grid {1, 3/4, 1/2}
constexpr int kMaxCol = 8;      // column-relay (directions, roles) choices
constexpr int kCtrInts = 16;    // sweep counter block: ticket, abort flag, epoch, per-XCD tickets
// Polls of an upstream face word before a sweep gives up (about 1-2 us each
// under load, so several seconds): far above any wait of a sweep that
// progresses, also with other problems' sweeps on the GPU at the same time.
constexpr int kDefaultWaitLimit = 1 << 22;

// One captured source iteration (sweep + moments/next source + residual) of
// one group, keyed by everything its kernels were launched with.
struct IterGraph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
};

struct DeviceState {
    bool ready = false;
    std::vector<IterGraph> graphs;  // most recently used last
    hipStream_t capture = nullptr;  // private stream graphs are captured on
    hipStream_t batch_stream = nullptr;  // this problem's stream inside dsn_solve_batch
    int device = -1;
    std::vector<void *> allocs;
    size_t bytes = 0;
    uint8_t *mat_nat = nullptr, *mat = nullptr;
    double *dens_nat = nullptr, *dens = nullptr;
    double *xs_t = nullptr, *xs_s = nullptr, *D0 = nullptr, *phiu = nullptr, *oms = nullptr;
    double *phic = nullptr, *part = nullptr, *spec = nullptr;
    void *F = nullptr;  // T [Nm][Vp]
    void *M0 = nullptr, *cdir = nullptr, *sig = nullptr, *psi = nullptr, *faceY = nullptr, *faceZ = nullptr;
    Ctl *ctl = nullptr;
    Ctl *h_ctl = nullptr;  // pinned host mirror
    int *sweep_ctr = nullptr, *sweep_dstart = nullptr;
    int sweep_nitems = 0, sweep_grid = 0;  // sweep_nitems: items of one source
    // sweep launch shape: waves per block and its resident grid per choice
    int wpb = 0;
    int xcd_nq = 0;   // XCDs, when workgroup i was seen to run on XCD i mod xcd_nq (else 0)
    int xcd_use = 0;  // per-XCD queues in use (0 or xcd_nq)
    int relay = 0;    // column-relay roles in use (0: pencil items)
    // column-relay shapes built: (directions, roles) and their resident grid (0: does not fit)
    int col_w[kMaxCol] = {}, col_r[kMaxCol] = {}, col_grid[kMaxCol] = {};
    int ncol = 0;
    // kind of word the forward face buffers hold: -1 none (all invalid), 0
    // sign-parity, 1 tagged
    int face_tagged = -1;
    int grid_of[kMaxWpb + 1] = {};
    unsigned long long *csum = nullptr;  // autotune checksums
    bool tuned = false, tune_pending = false;
    SweepShape tune_log[kMaxShapes];
    int tune_n = 0;
    // per-source buffers are sized for S_cap sources of a batch
    int S_cap = 0, dstart_S = 0, dstart_wpb = 0;
    double *src_par = nullptr;
    int *face_par = nullptr;
    int S_cap_alloc = 0;  // sources the per-source buffers were sized for
    int wait_limit = 0;   // from the current call's options
    std::vector<void *> src_allocs;
    size_t src_bytes = 0;
    // sources solved together: their ray traces [c_cap][G][Vp], [c_cap][3][Vp], parameters [c_cap][8],
    // spectra [c_cap][G]; the summed uncollided fluence [G][Vp] and moments [G][Nm][Vp]
    double *c_phiu = nullptr, *c_oms = nullptr, *c_par = nullptr, *c_spec = nullptr;
    double *c_pusum = nullptr, *c_usum = nullptr;
    int c_cap = 0;
    std::vector<void *> c_allocs;
    size_t c_bytes = 0;
    // adjoint state (allocated at the first adjoint call)
    bool adj_ready = false;
    double *phia = nullptr, *wdir = nullptr, *phit_tmp = nullptr, *dot_part = nullptr, *dot_out = nullptr;
    double *kdose = nullptr;  // [n_materials][G] fluence-to-dose factors of the last dsn_dose call
    // adjoint with the fixup: fixed-axis sets [Nd][Vp] and the adjoint sweeps' own face words
    uint8_t *mask = nullptr;
    void *afaceY = nullptr, *afaceZ = nullptr;
    void *psi2 = nullptr;
    Ctl *ctl_adj = nullptr, *ctl_free = nullptr;
    StageTimer timer;
};

struct dsn_problem {
    Geom geom;
    int nmat, G, L, Nm, N, Nd, D, fixup, precision;
    bool has_density;
    std::vector<uint8_t> material;
    std::vector<double> density, sigma_t, sigma_s, omega, w, M0, D0, cdir;
    // host staging that dsn_solve_noalloc fills without allocating: the FP32
    // copies of the direction tables, the sweep's diagonal table and the
    // control blocks read back after a solve
    std::vector<float> M0f, cdirf;
    std::vector<int> dstart_host;
    std::vector<Ctl> ctl_host;
    std::vector<double> spec_host;
    double par_host[kSrcPar];
    int flags_host[2];
    DeviceState dev;
};

namespace {

size_t tsize(const dsn_problem *p) { return p->precision == DSN_FP32 ? sizeof(float) : sizeof(double); }

struct Sizes {
    size_t mat, dens, xs_t, xs_s, M0, D0, cdir, phiu, oms, phic, F, sig, psi, face, part, ctl, spec, queue;
    size_t total() const
    {
        return 2 * mat + 2 * dens + xs_t + xs_s + M0 + D0 + cdir + phiu + oms + phic + F + sig + psi + 2 * face +
               part + ctl + spec + queue;
    }
};

// Persistent sweep queue: items = 8 octants x direction groups x pencils
// (relay > 0: x rows of pencils, one item sweeping a whole row).
int sweep_items(const dsn_problem *p, int wpb, int relay = 0)
{
    return 8 * (p->D / wpb) * (relay > 0 ? 1 : p->geom.NJ) * p->geom.NK;
}

// Resident grid of a column-relay shape, 0 if it is not built or does not fit.
int col_grid_of(const DeviceState &d, int w, int r)
{
    for (int i = 0; i < d.ncol; ++i)
        if (d.col_w[i] == w && d.col_r[i] == r) return d.col_grid[i];
    return 0;
}

// First ticket of every pencil diagonal (tickets go diagonal by diagonal, all
// sources of the batch and all direction groups inside each diagonal), plus
// the total.
std::vector<int> diagonal_starts(const dsn_problem *p, int S, int wpb)
{
    const int NJ = p->geom.NJ, NK = p->geom.NK;
    const int ngrp = p->D / wpb;
    std::vector<int> ds(NJ + NK + 1, 0);
    for (int dd = 0; dd <= NJ + NK - 2; ++dd) {
        const int lo = std::max(0, dd - (NK - 1)), hi = std::min(dd, NJ - 1);
        ds[dd + 1] = ds[dd] + (hi - lo + 1) * 8 * ngrp * S;
    }
    ds[NJ + NK] = ds[NJ + NK - 1];
    return ds;
}

Sizes sizes_of(const dsn_problem *p)
{
    const Geom &g = p->geom;
    const size_t ts = tsize(p);
    Sizes s;
    s.mat = (size_t)g.Vp;
    s.dens = (size_t)g.Vp * sizeof(double);
    s.xs_t = (size_t)p->nmat * p->G * sizeof(double);
    s.xs_s = (size_t)p->nmat * (p->L + 1) * p->G * p->G * sizeof(double);
    s.M0 = (size_t)p->D * p->Nm * ts;
    s.D0 = (size_t)p->D * p->Nm * sizeof(double);
    s.cdir = (size_t)p->Nd * 3 * ts;
    s.phiu = (size_t)p->G * g.Vp * sizeof(double);
    s.oms = (size_t)3 * g.Vp * sizeof(double);
    s.phic = (size_t)p->G * p->Nm * g.Vp * sizeof(double);
    s.F = (size_t)p->Nm * g.Vp * ts;
    s.sig = (size_t)g.Vp * ts;
    s.psi = (size_t)p->Nd * g.Vp * ts;
    s.face = (size_t)p->Nd * g.NJ * g.NK * g.nx * 8 * (ts / 4) * sizeof(unsigned long long);
    s.part = (size_t)((g.Vp + 255) / 256) * 4 * sizeof(double);
    s.ctl = (size_t)p->G * sizeof(Ctl);
    s.spec = (size_t)p->G * sizeof(double);
    s.queue = (size_t)(2 + g.NJ + g.NK + 1) * sizeof(int);
    return s;
}

// Device-wide calls (hipDeviceSynchronize, allocation and release) must not
// run while a stream is being captured into a graph, and the problems of a
// batch are driven from several host threads.  Captures hold this gate
// shared; device-wide sections hold it exclusively (re-entrant per thread).
std::shared_mutex g_capture_gate;
thread_local int t_gate_depth = 0;

struct DeviceWide {
    DeviceWide()
    {
        if (t_gate_depth++ == 0) g_capture_gate.lock();
    }
    ~DeviceWide()
    {
        if (--t_gate_depth == 0) g_capture_gate.unlock();
    }
    DeviceWide(const DeviceWide &) = delete;
    DeviceWide &operator=(const DeviceWide &) = delete;
};

dsn_status dev_alloc(DeviceState &d, void **ptr, size_t bytes)
{
    DeviceWide gate;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes ? bytes : 16);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? DSN_ERR_OUT_OF_MEMORY : DSN_ERR_DEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    d.allocs.push_back(q);
    d.bytes += bytes;
    *ptr = q;
    return DSN_OK;
}

void dev_release(DeviceState &d)
{
    DeviceWide gate;
    if (d.device >= 0) (void)hipSetDevice(d.device);
    for (void *q : d.allocs) (void)hipFree(q);
    d.allocs.clear();
    for (void *q : d.src_allocs) (void)hipFree(q);
    d.src_allocs.clear();
    for (void *q : d.c_allocs) (void)hipFree(q);
    d.c_allocs.clear();
    if (d.h_ctl) (void)hipHostFree(d.h_ctl);
    for (IterGraph &x : d.graphs)
        if (x.exec) (void)hipGraphExecDestroy(x.exec);
    if (d.capture) (void)hipStreamDestroy(d.capture);
    if (d.batch_stream) (void)hipStreamDestroy(d.batch_stream);
    d.timer.release();
    d = DeviceState();
}

// Device bytes one source of a batch needs.
size_t per_source_bytes(const dsn_problem *p)
{
    const Sizes s = sizes_of(p);
    return s.phiu + s.oms + s.phic + s.F + s.psi + 2 * s.face + s.part + s.ctl + s.spec + 8 * sizeof(double);
}

// Sources solved together, limited by free device memory (and to 64).
int batch_limit(const dsn_problem *p)
{
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return 1;
    const double avail = 0.8 * (double)(free_b + p->dev.src_bytes);
    const int s = (int)(avail / (double)per_source_bytes(p));
    return std::max(1, std::min(64, s));
}

// Per-source buffers for a batch of S sources; the ticket table of the sweep.
// Every face word becomes one that no sweep accepts: all-ones is a NaN
// payload for the sign-parity words and an epoch no sweep uses for the
// tagged words.  Needed at allocation and after an aborted sweep, which can
// leave words of the current parity behind.
dsn_status invalidate_faces(DeviceState &d, size_t bytes)
{
    DeviceWide gate;
    DSN_HIP(hipDeviceSynchronize());
    DSN_HIP(hipMemset(d.faceY, 0xFF, bytes));
    DSN_HIP(hipMemset(d.faceZ, 0xFF, bytes));
    DSN_HIP(hipMemset(d.face_par, 0, (size_t)d.S_cap_alloc * sizeof(int)));
    DSN_HIP(hipDeviceSynchronize());
    d.face_tagged = -1;
    return DSN_OK;
}

// After a sweep wait timed out: clear the abort flag and the faces so the
// problem stays usable for the next call.
dsn_status recover_from_abort(dsn_problem *p)
{
    DeviceWide gate;
    DeviceState &d = p->dev;
    const int zero2[2] = {0, 0};
    DSN_HIP(hipDeviceSynchronize());
    DSN_HIP(hipMemcpy(d.sweep_ctr, zero2, sizeof(zero2), hipMemcpyHostToDevice));  // ticket, abort flag
    if (d.afaceY) {
        DSN_HIP(hipMemset(d.afaceY, 0xFF, sizes_of(p).face));
        DSN_HIP(hipMemset(d.afaceZ, 0xFF, sizes_of(p).face));
    }
    return invalidate_faces(d, (size_t)d.S_cap_alloc * sizes_of(p).face);
}

// A sweep raised its abort flag: 1 = a dependency wait timed out, 2 = a
// per-XCD queue was not served (the per-XCD queues are then switched off for
// the handle).  The faces are invalidated so the handle stays usable.
dsn_status sweep_failed(dsn_problem *p, int flag)
{
    (void)recover_from_abort(p);
    if (flag == 2) {
        p->dev.xcd_nq = 0;
        p->dev.xcd_use = 0;
        return fail(DSN_ERR_DEVICE, "sweep: a per-XCD ticket queue was not served (results invalid)");
    }
    return fail(DSN_ERR_DEVICE, "sweep dependency wait timed out (results invalid)");
}

dsn_status ensure_batch(dsn_problem *p, int S)
{
    DeviceWide gate;
    DeviceState &d = p->dev;
    if ((double)S * sweep_items(p, 1) >= (double)(1 << 29))
        return fail(DSN_ERR_UNSUPPORTED, "too many sweep items (sources x directions x pencils) in one batch");
    if (S > d.S_cap) {
        (void)hipDeviceSynchronize();
        for (void *q : d.src_allocs) (void)hipFree(q);
        d.src_allocs.clear();
        d.bytes -= d.src_bytes;
        d.src_bytes = 0;
        d.S_cap = 0;
        if (d.h_ctl) (void)hipHostFree(d.h_ctl);
        d.h_ctl = nullptr;
        const Sizes s = sizes_of(p);
        auto alloc = [&](void **ptr, size_t b) -> dsn_status {
            void *q = nullptr;
            hipError_t e = hipMalloc(&q, b ? b : 16);
            if (e != hipSuccess)
                return fail(e == hipErrorOutOfMemory ? DSN_ERR_OUT_OF_MEMORY : DSN_ERR_DEVICE,
                            std::string("hipMalloc: ") + hipGetErrorString(e));
            d.src_allocs.push_back(q);
            d.src_bytes += b;
            d.bytes += b;
            *ptr = q;
            return DSN_OK;
        };
        dsn_status st;
        const size_t n = (size_t)S;
        d.S_cap_alloc = S;
        if ((st = alloc((void **)&d.phiu, n * s.phiu)) || (st = alloc((void **)&d.oms, n * s.oms)) ||
            (st = alloc((void **)&d.phic, n * s.phic)) || (st = alloc((void **)&d.F, n * s.F)) ||
            (st = alloc(&d.psi, n * s.psi)) || (st = alloc(&d.faceY, n * s.face)) ||
            (st = alloc(&d.faceZ, n * s.face)) || (st = alloc((void **)&d.part, n * s.part)) ||
            (st = alloc((void **)&d.ctl, n * s.ctl)) || (st = alloc((void **)&d.spec, n * s.spec)) ||
            (st = alloc((void **)&d.src_par, n * kSrcPar * sizeof(double))) ||
            (st = alloc((void **)&d.face_par, n * sizeof(int))))
            return st;
        if ((st = invalidate_faces(d, n * s.face)) != DSN_OK) return st;
        if (hipHostMalloc((void **)&d.h_ctl, n * s.ctl, hipHostMallocDefault) != hipSuccess)
            return fail(DSN_ERR_OUT_OF_MEMORY, "hipHostMalloc failed");
        d.S_cap = S;
    }
    if (d.dstart_S != S || d.dstart_wpb != d.wpb) {
        const std::vector<int> ds = diagonal_starts(p, S, d.wpb);
        DSN_HIP(hipMemcpy(d.sweep_dstart, ds.data(), ds.size() * sizeof(int), hipMemcpyHostToDevice));
        d.dstart_S = S;
        d.dstart_wpb = d.wpb;
    }
    return DSN_OK;
}

// Ray-trace buffers for n sources solved together (combine_sources), plus
// the one-source iteration buffers.
dsn_status ensure_combined(dsn_problem *p, int n)
{
    dsn_status st = ensure_batch(p, 1);
    if (st != DSN_OK) return st;
    DeviceWide gate;
    DeviceState &d = p->dev;
    if (n <= d.c_cap) return DSN_OK;
    (void)hipDeviceSynchronize();
    for (void *q : d.c_allocs) (void)hipFree(q);
    d.c_allocs.clear();
    d.bytes -= d.c_bytes;
    d.c_bytes = 0;
    d.c_cap = 0;
    const Sizes sz = sizes_of(p);
    const size_t bytes[6] = {(size_t)n * sz.phiu, (size_t)n * sz.oms, (size_t)n * kSrcPar * sizeof(double),
                             (size_t)n * sz.spec, sz.phiu, sz.phic};
    double **dst[6] = {&d.c_phiu, &d.c_oms, &d.c_par, &d.c_spec, &d.c_pusum, &d.c_usum};
    for (int i = 0; i < 6; ++i) {
        void *q = nullptr;
        const hipError_t e = hipMalloc(&q, bytes[i]);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? DSN_ERR_OUT_OF_MEMORY : DSN_ERR_DEVICE,
                        std::string("hipMalloc: ") + hipGetErrorString(e));
        d.c_allocs.push_back(q);
        d.c_bytes += bytes[i];
        d.bytes += bytes[i];
        *dst[i] = (double *)q;
    }
    d.c_cap = n;
    return DSN_OK;
}

dsn_status ensure_device(dsn_problem *p)
{
    DeviceState &d = p->dev;
    if (d.ready) return DSN_OK;
    DeviceWide gate;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(DSN_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    DSN_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    DSN_HIP(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(DSN_ERR_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    d.device = dev;
    const Sizes s = sizes_of(p);
    dsn_status st;
#define ALLOC(ptr, bytes) \
    if ((st = dev_alloc(d, (void **)&(ptr), (bytes))) != DSN_OK) { dev_release(d); return st; }
    ALLOC(d.mat_nat, (size_t)p->geom.V);
    ALLOC(d.mat, s.mat);
    if (p->has_density) ALLOC(d.dens_nat, (size_t)p->geom.V * sizeof(double));
    ALLOC(d.dens, s.dens);
    ALLOC(d.xs_t, s.xs_t);
    ALLOC(d.xs_s, s.xs_s);
    ALLOC(d.M0, s.M0);
    ALLOC(d.D0, s.D0);
    ALLOC(d.cdir, s.cdir);
    ALLOC(d.sig, s.sig);
    d.wpb = sweep_wpb(p->D, p->precision == DSN_FP64);
    d.sweep_nitems = sweep_items(p, d.wpb);
    ALLOC(d.sweep_ctr, kCtrInts * sizeof(int));
    ALLOC(d.csum, 2 * sizeof(unsigned long long));
    ALLOC(d.sweep_dstart, (size_t)std::max(p->geom.NJ + p->geom.NK + 1, 64) * sizeof(int));
#undef ALLOC
    const bool f32 = p->precision == DSN_FP32;
    std::vector<float> M0f(p->M0.begin(), p->M0.end()), cdf(p->cdir.begin(), p->cdir.end());
    hipError_t e = hipSuccess;
    e = e ? e : hipMemcpy(d.mat_nat, p->material.data(), p->geom.V, hipMemcpyHostToDevice);
    if (p->has_density)
        e = e ? e : hipMemcpy(d.dens_nat, p->density.data(), p->geom.V * sizeof(double), hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(d.xs_t, p->sigma_t.data(), s.xs_t, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(d.xs_s, p->sigma_s.data(), s.xs_s, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(d.M0, f32 ? (const void *)M0f.data() : (const void *)p->M0.data(), s.M0,
                          hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(d.D0, p->D0.data(), s.D0, hipMemcpyHostToDevice);
    e = e ? e : hipMemcpy(d.cdir, f32 ? (const void *)cdf.data() : (const void *)p->cdir.data(), s.cdir,
                          hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_release(d);
        return fail(DSN_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    {
        const int zeros[kCtrInts] = {};
        e = e ? e : hipMemcpy(d.sweep_ctr, zeros, sizeof(zeros), hipMemcpyHostToDevice);
        // workgroup -> XCD mapping, for the per-XCD queues: 64 workgroups
        // (the diagonal table, not filled yet, holds the answers) must go
        // round robin over k XCDs; the first one may be any (it depends on
        // the hardware queue the launch goes through)
        if (e == hipSuccess) {
            launch_xcc_probe(d.sweep_dstart, 64, 0);
            int xcc[64];
            e = hipMemcpy(xcc, d.sweep_dstart, sizeof(xcc), hipMemcpyDeviceToHost);
            int k = 0;
            for (int b = 0; b < 64; ++b) k = std::max(k, xcc[b] + 1);
            bool rr = e == hipSuccess && (k == 2 || k == 4 || k == 8);
            for (int b = 0; rr && b < 64; ++b) rr = xcc[b] == (xcc[0] + b) % k;
            d.xcd_nq = rr ? k : 0;
        }
        int wl[kMaxWpb];
        const int nw = sweep_wpb_choices(!f32, wl);
        for (int i = 0; i < nw; ++i)
            if (p->D % wl[i] == 0 && wl[i] <= kMaxWpb)
                d.grid_of[wl[i]] = f32 ? sweep_grid<float>(wl[i], p->fixup, prop.multiProcessorCount)
                                       : sweep_grid<double>(wl[i], p->fixup, prop.multiProcessorCount);  // mode = fixup
        d.sweep_grid = d.grid_of[d.wpb];
        int cw[kMaxCol], cr[kMaxCol];
        const int nc = sweep_col_choices(!f32, cw, cr);
        d.ncol = 0;
        for (int i = 0; i < nc && d.ncol < kMaxCol; ++i) {
            if (p->D % cw[i]) continue;
            const int gr = f32 ? sweep_grid_col<float>(cw[i], cr[i], p->fixup, p->geom.nx, prop.multiProcessorCount)
                               : sweep_grid_col<double>(cw[i], cr[i], p->fixup, p->geom.nx, prop.multiProcessorCount);
            d.col_w[d.ncol] = cw[i];
            d.col_r[d.ncol] = cr[i];
            d.col_grid[d.ncol++] = gr;
        }
    }
    if (e != hipSuccess) {
        dev_release(d);
        return fail(DSN_ERR_DEVICE, std::string("upload: ") + hipGetErrorString(e));
    }
    launch_voxels_to_pencils(p->geom, d.mat_nat, d.dens_nat, d.mat, d.dens, 0);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        dev_release(d);
        return fail(DSN_ERR_DEVICE, std::string("voxel layout: ") + hipGetErrorString(e));
    }
    d.ready = true;
    return ensure_batch(p, 1);
}

template <typename T>
SolveArgs<T> make_args(dsn_problem *p, int S = 1)
{
    DeviceState &d = p->dev;
    SolveArgs<T> a;
    std::memset(&a, 0, sizeof(a));  // padding too: the bytes key the iteration graphs
    a.g = p->geom;
    a.G = p->G;
    a.L = p->L;
    a.Nm = p->Nm;
    a.Nd = p->Nd;
    a.D = p->D;
    a.nmat = p->nmat;
    a.mat = d.mat;
    a.dens = d.dens;
    a.mat_nat = d.mat_nat;
    a.dens_nat = d.dens_nat;
    a.xs_t = d.xs_t;
    a.xs_s = d.xs_s;
    a.M0 = (const T *)d.M0;
    a.D0 = d.D0;
    a.cdir = (const T *)d.cdir;
    a.phiu = d.phiu;
    a.oms = d.oms;
    a.phic = d.phic;
    a.F = (T *)d.F;
    a.usum = nullptr;
    a.sig = (T *)d.sig;
    a.psi = (T *)d.psi;
    a.faceY = (unsigned long long *)d.faceY;
    a.faceZ = (unsigned long long *)d.faceZ;
    a.part = d.part;
    a.ctl = d.ctl;
    a.sweep_ctr = d.sweep_ctr;
    a.sweep_dstart = d.sweep_dstart;
    a.sweep_nitems = d.sweep_nitems;
    a.sweep_grid = d.sweep_grid;
    a.sweep_wpb = d.wpb;
    a.sweep_xcd = d.xcd_use;
    a.sweep_relay = d.relay;
    a.sweep_mode = p->fixup;  // forward: pure DD or with the set-to-zero fixup
    a.mask = nullptr;
    a.sweep_spin_limit = d.wait_limit > 0 ? d.wait_limit : kDefaultWaitLimit;
    a.rev = 0;
    a.sig_from_mat = d.dens_nat == nullptr;
    // MI355X's 256 MB last-level (Infinity) cache holds a small problem's
    // arrays from one pass to the next; past that size they only displace the
    // data the sweep re-reads (face words, material bytes)
    a.stream_nt = (double)S * p->Nd * (double)p->geom.Vp * sizeof(T) > 256.0 * 1024 * 1024 ? 1 : 0;
    a.wdir = d.wdir;
    const Geom &g = p->geom;
    a.S = S;
    a.sweep_nitems = S * d.sweep_nitems;
    a.str_psi = (long)p->Nd * g.Vp;
    a.str_phic = (long)p->G * p->Nm * g.Vp;
    a.str_phiu = (long)p->G * g.Vp;
    a.str_oms = 3L * g.Vp;
    a.str_F = (long)p->Nm * g.Vp;
    a.str_face = (long)p->Nd * g.NJ * g.NK * g.nx * 8 * (long)(sizeof(T) / 4);
    a.str_part = 4L * ((g.Vp + 255) / 256);
    a.src_par = d.src_par;
    a.face_par = d.face_par;
    a.src_spec = d.spec;
    return a;
}

dsn_status check_source(const dsn_problem *p, const dsn_source &s)
{
    const Geom &g = p->geom;
    if (!s.spectrum) return fail(DSN_ERR_INVALID_ARG, "source spectrum is NULL");
    if (!finite_all(s.position, 3) || !finite_all(s.axis, 3) || !std::isfinite(s.half_angle) || s.half_angle < 0)
        return fail(DSN_ERR_INVALID_ARG, "source position/axis/half_angle must be finite, half_angle >= 0");
    for (int gg = 0; gg < p->G; ++gg)
        if (!std::isfinite(s.spectrum[gg]) || s.spectrum[gg] < 0)
            return fail(DSN_ERR_INVALID_ARG, "source spectrum must be finite and >= 0");
    if (s.half_angle < M_PI && !(s.axis[0] * s.axis[0] + s.axis[1] * s.axis[1] + s.axis[2] * s.axis[2] > 0))
        return fail(DSN_ERR_INVALID_ARG, "cone source needs a non-zero axis");
    if (!finite_all(s.fan_normal, 3) || !std::isfinite(s.fan_half_thickness))
        return fail(DSN_ERR_INVALID_ARG, "fan_normal and fan_half_thickness must be finite");
    if (s.fan_half_thickness > 0 && s.half_angle < M_PI) {
        if (s.fan_half_thickness >= M_PI / 2 || s.half_angle >= M_PI / 2)
            return fail(DSN_ERR_INVALID_ARG, "a fan needs half_angle and fan_half_thickness below pi/2");
        const double a2 = s.axis[0] * s.axis[0] + s.axis[1] * s.axis[1] + s.axis[2] * s.axis[2];
        const double n2 = s.fan_normal[0] * s.fan_normal[0] + s.fan_normal[1] * s.fan_normal[1] +
                          s.fan_normal[2] * s.fan_normal[2];
        const double na = s.fan_normal[0] * s.axis[0] + s.fan_normal[1] * s.axis[1] + s.fan_normal[2] * s.axis[2];
        if (!(n2 - na * na / a2 > 1e-12 * n2))
            return fail(DSN_ERR_INVALID_ARG, "fan_normal must not be parallel to the axis");
    }
    // nearest voxel centre must not coincide with the source point
    const double h[3] = {g.dx, g.dy, g.dz};
    const int nn[3] = {g.nx, g.ny, g.nz};
    double r2 = 0.0;
    for (int t = 0; t < 3; ++t) {
        double idx = std::floor(s.position[t] / h[t]);
        idx = std::min(std::max(idx, 0.0), (double)(nn[t] - 1));
        double best = 1e300;
        for (int dd = -1; dd <= 1; ++dd) {
            double c = idx + dd;
            if (c < 0 || c > nn[t] - 1) continue;
            best = std::min(best, std::fabs((c + 0.5) * h[t] - s.position[t]));
        }
        r2 += best * best;
    }
    const double mind = std::min(g.dx, std::min(g.dy, g.dz));
    if (std::sqrt(r2) < 1e-6 * mind)
        return fail(DSN_ERR_INVALID_ARG, "source coincides with a voxel centre");
    return DSN_OK;
}

dsn_status check_opts(const dsn_problem *p, const dsn_solve_opts *o)
{
    if (!o) return fail(DSN_ERR_INVALID_ARG, "opts is NULL");
    if (o->max_iters < 1) return fail(DSN_ERR_INVALID_ARG, "max_iters must be >= 1");
    if (o->fixed_iters) {
        for (int g = 0; g < p->G; ++g)
            if (o->fixed_iters[g] < 0) return fail(DSN_ERR_INVALID_ARG, "fixed_iters must be >= 0");
    } else if (!(o->tol > 0) || !std::isfinite(o->tol)) {
        return fail(DSN_ERR_INVALID_ARG, "tol must be finite and > 0");
    }
    if (o->stagnation_stop != 0 && o->stagnation_stop != 1)
        return fail(DSN_ERR_INVALID_ARG, "stagnation_stop must be 0 or 1");
    if (o->stop_rule != 0 && o->stop_rule != 1) return fail(DSN_ERR_INVALID_ARG, "stop_rule must be 0 or 1");
    if (o->wait_limit < 0) return fail(DSN_ERR_INVALID_ARG, "wait_limit must be >= 0");
    if (o->autotune != 0 && o->autotune != 1) return fail(DSN_ERR_INVALID_ARG, "autotune must be 0 or 1");
    if (o->combine_sources != 0 && o->combine_sources != 1)
        return fail(DSN_ERR_INVALID_ARG, "combine_sources must be 0 or 1");
    if (o->batch_mode != 0 && o->batch_mode != 1) return fail(DSN_ERR_INVALID_ARG, "batch_mode must be 0 or 1");
    return DSN_OK;
}

dsn_status status_of(const Ctl *c, int G)
{
    dsn_status st = DSN_OK;
    for (int g = 0; g < G; ++g) {
        if (c[g].status == 6) return fail(DSN_ERR_NUMERICAL, "residual became NaN or infinite");
        if (c[g].status == 5) st = DSN_ERR_NOT_CONVERGED;
    }
    if (st == DSN_ERR_NOT_CONVERGED) g_err = "max_iters reached before tol";
    return st;
}

// A sweep on the forward face buffers.  Those hold the words of one codec at
// a time: before a sweep that reads the other kind (a launch shape with
// per-XCD queues after one without, a fixed-axis recording sweep after a
// per-XCD one), every word is invalidated on the stream, so neither codec
// can take the other's words for its own.  Sweeps on other face buffers go
// straight through.  Returns -1 if a switch would be needed while the stream
// is capturing (the caller then launches without a graph).
template <typename T>
int sweep_forward_faces(dsn_problem *p, const SolveArgs<T> &a, int g, hipStream_t s, hipEvent_t ev_before = nullptr,
                        hipEvent_t ev_after = nullptr)
{
    DeviceState &d = p->dev;
    if ((void *)a.faceY == d.faceY) {
        // codec of the words; column-relay sweeps (+2) leave the y words
        // alone, so those go stale
        const bool col = sweep_uses_col(a);
        const int tagged = col ? (a.sweep_mode == 0 ? 1 : 0) + 2
                               : sweep_tagged_faces(sizeof(T) == 8, a.sweep_mode, a.sweep_wpb, a.sweep_xcd) ? 1 : 0;
        if (d.face_tagged >= 0 && tagged != d.face_tagged) {
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return -1;
            const size_t bytes = (size_t)d.S_cap_alloc * sizes_of(p).face;
            (void)hipMemsetAsync(d.faceY, 0xFF, bytes, s);
            (void)hipMemsetAsync(d.faceZ, 0xFF, bytes, s);
            (void)hipMemsetAsync(d.face_par, 0, (size_t)d.S_cap_alloc * sizeof(int), s);
        }
        d.face_tagged = tagged;
    }
    return launch_sweeps<T>(a, g, s, ev_before, ev_after);
}

// The steady source iteration of group g as a HIP graph: captured once on a
// private stream (default priority) and replayed on the caller's stream.  All
// state the kernels keep between launches (tickets, sweep epoch, face
// parity, control blocks) lives in device memory, so replays are exact.
// Returns nullptr when capture is not available (the caller launches
// directly).
template <typename T>
hipGraphExec_t iteration_graph(dsn_problem *p, const SolveArgs<T> &a, int g)
{
    DeviceState &d = p->dev;
    std::vector<unsigned char> key(sizeof(SolveArgs<T>) + 3 * sizeof(int));
    std::memcpy(key.data(), &a, sizeof(SolveArgs<T>));
    const int extra[3] = {g, p->fixup, (int)sizeof(T)};
    std::memcpy(key.data() + sizeof(SolveArgs<T>), extra, sizeof(extra));
    for (size_t i = 0; i < d.graphs.size(); ++i)
        if (d.graphs[i].key == key) {
            IterGraph x = d.graphs[i];
            d.graphs.erase(d.graphs.begin() + i);
            d.graphs.push_back(x);
            return x.exec;
        }
    if (!d.capture && hipStreamCreateWithFlags(&d.capture, hipStreamNonBlocking) != hipSuccess) {
        d.capture = nullptr;
        return nullptr;
    }
    std::shared_lock<std::shared_mutex> lk(g_capture_gate, std::defer_lock);
    if (t_gate_depth == 0) lk.lock();
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(d.capture, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    const bool same_faces = sweep_forward_faces<T>(p, a, g, d.capture) >= 0;
    launch_d2m<T>(a, g, true, d.capture);
    const hipError_t ec = hipStreamEndCapture(d.capture, &graph);
    if (!same_faces) {
        if (graph) (void)hipGraphDestroy(graph);
        return nullptr;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = ec == hipSuccess ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) : ec;
    if (graph) (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    constexpr size_t kMaxGraphs = 64;
    if (d.graphs.size() == kMaxGraphs) {
        (void)hipGraphExecDestroy(d.graphs.front().exec);
        d.graphs.erase(d.graphs.begin());
    }
    d.graphs.push_back(IterGraph{key, exec});
    return exec;
}

// Times the sweep's launch shapes on the current group's source and keeps the
// fastest: every built waves-per-block value that divides the directions of
// an octant, with one global ticket queue and - where built and the
// workgroup-to-XCD mapping allows - with per-XCD queues, each with the full
// resident grid, three quarters and half of it; one untimed and two timed
// launches per shape.  The sweep overwrites its source with the angular
// fluence, so the source is formed again from the moments (which no sweep
// changes) before every launch and once more at the end: the iteration that
// follows is unchanged.  Every shape's angular fluence is compared, by an
// order-independent checksum, with the default shape's; a shape that
// differs (or whose waits timed out) is logged with a negative time and not
// used.
template <typename T>
void tune_sweep(dsn_problem *p, SolveArgs<T> &a, int g, hipStream_t s)
{
    DeviceState &d = p->dev;
    d.tune_pending = false;
    d.tune_n = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    for (hipEvent_t &e : ev) ok = ok && hipEventCreate(&e) == hipSuccess;
    SweepShape best{d.wpb, d.sweep_grid, d.xcd_use, 1e30f, d.relay};
    const int S = a.S;
    const long words = (long)S * p->Nd * p->geom.Vp * (long)(sizeof(T) / 4);
    std::vector<int> ds;
    auto use_table = [&](int w) {  // diagonal starts for w waves per block (host copy kept until synced)
        ds = diagonal_starts(p, S, w);
        return hipMemcpyAsync(d.sweep_dstart, ds.data(), ds.size() * sizeof(int), hipMemcpyHostToDevice, s) ==
               hipSuccess;
    };
    auto checksum = [&](int slot, unsigned long long &out) {
        const bool good = hipMemsetAsync(d.csum + slot, 0, sizeof(unsigned long long), s) == hipSuccess;
        launch_checksum(a.psi, words, d.csum + slot, s);
        return good && hipMemcpyAsync(&out, d.csum + slot, sizeof(out), hipMemcpyDeviceToHost, s) == hipSuccess &&
               hipStreamSynchronize(s) == hipSuccess;
    };
    auto shape_args = [&](int w, int blocks, int xcd, int relay) {
        SolveArgs<T> c = a;
        c.sweep_wpb = w;
        c.sweep_nitems = S * sweep_items(p, w, relay);
        c.sweep_grid = blocks;
        c.sweep_xcd = xcd;
        c.sweep_relay = relay;
        return c;
    };
    // reference: the default shape
    unsigned long long ref = 0;
    ok = ok && use_table(d.wpb);
    if (ok) {
        launch_m2d<T>(a, g, s);
        sweep_forward_faces<T>(p, shape_args(d.wpb, d.sweep_grid, 0, 0), g, s);
        ok = checksum(0, ref);
    }
    struct Cand {
        int w, xcd, relay, grid;
    };
    std::vector<Cand> cands;
    int wl[kMaxWpb];
    const int nw = sweep_wpb_choices(sizeof(T) == 8, wl);
    for (int i = 0; i < nw; ++i) {
        const int w = wl[i];
        if (w > kMaxWpb || p->D % w || d.grid_of[w] < 1) continue;
        cands.push_back({w, 0, 0, d.grid_of[w]});
        if (d.xcd_nq > 0 && sweep_xcd_supported(sizeof(T) == 8, p->fixup, w))
            cands.push_back({w, d.xcd_nq, 0, d.grid_of[w]});
    }
    for (int i = 0; i < d.ncol; ++i)
        if (d.col_grid[i] > 0) cands.push_back({d.col_w[i], 0, d.col_r[i], d.col_grid[i]});
    for (size_t ci = 0; ok && ci < cands.size(); ++ci) {
        const int w = cands[ci].w;
        if (!(ok = use_table(w))) break;
        for (int f = 4; ok && f >= 2; --f) {
            const SolveArgs<T> c = shape_args(w, std::max(1, cands[ci].grid * f / 4), cands[ci].xcd, cands[ci].relay);
            launch_m2d<T>(a, g, s);
            sweep_forward_faces<T>(p, c, g, s);
            for (int r = 0; ok && r < 2; ++r) {
                launch_m2d<T>(a, g, s);
                ok = hipEventRecord(ev[2 * r], s) == hipSuccess;
                sweep_forward_faces<T>(p, c, g, s);
                ok = ok && hipEventRecord(ev[2 * r + 1], s) == hipSuccess;
            }
            float ms = 0.f, m1 = 0.f;
            ok = ok && hipEventSynchronize(ev[3]) == hipSuccess && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess &&
                 hipEventElapsedTime(&m1, ev[2], ev[3]) == hipSuccess;
            unsigned long long sum = 0;
            ok = ok && checksum(1, sum);
            int flags[2] = {0, 0};
            ok = ok && hipMemcpy(flags, d.sweep_ctr, sizeof(flags), hipMemcpyDeviceToHost) == hipSuccess;
            if (!ok) break;
            const bool same = sum == ref && !flags[1];
            if (flags[1]) ok = recover_from_abort(p) == DSN_OK;
            const SweepShape x{w, c.sweep_grid, c.sweep_xcd, same ? 0.5f * (ms + m1) : -1.f, c.sweep_relay};
            if (d.tune_n < kMaxShapes) d.tune_log[d.tune_n++] = x;
            if (same && x.ms < best.ms) best = x;
        }
    }
    (void)hipStreamSynchronize(s);  // the last table copy has finished before ds changes
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    launch_m2d<T>(a, g, s);
    d.wpb = best.wpb;
    d.sweep_grid = best.blocks;
    d.xcd_use = best.xcd;
    d.relay = best.relay;
    d.sweep_nitems = sweep_items(p, d.wpb, d.relay);
    ds = diagonal_starts(p, S, d.wpb);
    (void)hipMemcpyAsync(d.sweep_dstart, ds.data(), ds.size() * sizeof(int), hipMemcpyHostToDevice, s);
    (void)hipStreamSynchronize(s);
    d.dstart_S = S;
    d.dstart_wpb = d.wpb;
    a.sweep_wpb = d.wpb;
    a.sweep_grid = d.sweep_grid;
    a.sweep_xcd = d.xcd_use;
    a.sweep_relay = d.relay;
    a.sweep_nitems = S * d.sweep_nitems;
    d.tuned = true;
}

template <typename T>
// One source iteration: sweep, then moments, residual and - while the
// moments are in registers - the next iteration's directional source.  The
// first iteration of a group forms its source from the moments on entry.
// Without the stage timer the steady iterations are graph replays.  A pending
// autotune runs at the first iteration, between the source and the sweep.
// formed: the group source kernel already wrote the first directional source.
void enqueue_iteration(dsn_problem *p, SolveArgs<T> &a, int g, bool first, bool formed, hipStream_t s)
{
    StageTimer &t = p->dev.timer;
    size_t e;
    int n;
    t.cur_iter = first ? 0 : t.cur_iter + 1;
    if (!first && !t.on) {
        hipGraphExec_t x = iteration_graph<T>(p, a, g);
        if (x && hipGraphLaunch(x, s) == hipSuccess) return;
    }
    if (first) {
        if (!formed) {
            e = t.begin();
            n = launch_m2d<T>(a, g, s);
            t.end(DSN_STAGE_M2D, e, n);
        }
        if (p->dev.tune_pending) tune_sweep<T>(p, a, g, s);
    }
    // the sweep stage times the sweep kernel alone (events recorded around
    // its launch, after the ticket reset and before the parity flip)
    hipEvent_t eb = nullptr, ee = nullptr;
    t.pair(DSN_STAGE_SWEEP, 1, eb, ee);
    sweep_forward_faces<T>(p, a, g, s, eb, ee);
    e = t.begin();
    n = launch_d2m<T>(a, g, true, s);
    t.end(DSN_STAGE_D2M, e, n);
}

// Runs one group's source iteration to convergence (or its fixed count).
// Iterations are enqueued in chunks between host checks of the control
// blocks; the stage timer drops the ones that found their group converged.
// rule: the stop rule of the group's test (see k_resid).
template <typename T>
dsn_status iterate_group(dsn_problem *p, SolveArgs<T> &a, int g, const dsn_solve_opts &o, hipStream_t s,
                         int &chunk_hint, bool formed, int rule)
{
    DeviceState &d = p->dev;
    Ctl *const hctl = d.h_ctl;
    const int G = p->G, S = a.S;
    const int target = o.fixed_iters ? o.fixed_iters[g] : -1;
    launch_ctl_init(a.ctl, G, S, g, target, o.max_iters, o.fixed_iters ? 0.0 : o.tol, o.stagnation_stop, rule, s);
    if (target >= 0) {
        for (int it = 0; it < target; ++it) enqueue_iteration<T>(p, a, g, it == 0, formed, s);
        d.timer.cur_iter = -1;
        DSN_HIP(hipGetLastError());
        return DSN_OK;
    }
    int enq = 0;
    int chunk = std::max(1, chunk_hint);
    for (;;) {
        for (int c = 0; c < chunk; ++c) enqueue_iteration<T>(p, a, g, enq + c == 0, formed, s);
        enq += chunk;
        DSN_HIP(hipGetLastError());
        DSN_HIP(hipMemcpyAsync(hctl, a.ctl, (size_t)S * G * sizeof(Ctl), hipMemcpyDeviceToHost, s));
        DSN_HIP(hipStreamSynchronize(s));
        bool all = true;
        for (int k = 0; k < S; ++k) all = all && hctl[(size_t)k * G + g].done;
        if (all || enq >= o.max_iters) break;
        chunk = 2;
    }
    int most = 0;
    for (int k = 0; k < S; ++k) most = std::max(most, hctl[(size_t)k * G + g].iters);
    d.timer.flush(most);  // stream synchronised above
    d.timer.cur_iter = -1;
    chunk_hint = std::max(1, most - 2);
    return DSN_OK;
}

// Source parameters and spectra of src[0 .. S-1] into ar's per-source
// arrays (the host copies are kept until the stream has them).
template <typename T>
dsn_status upload_sources(dsn_problem *p, const SolveArgs<T> &ar, const dsn_source *src, int S, hipStream_t s)
{
    const int G = p->G;
    std::vector<double> par((size_t)S * kSrcPar), spec((size_t)S * G);
    for (int k = 0; k < S; ++k) {
        const dsn_source &sc = src[k];
        double *pk = &par[(size_t)kSrcPar * k];
        for (int t = 0; t < 3; ++t) {
            pk[t] = sc.position[t];
            pk[3 + t] = sc.axis[t];
        }
        pk[6] = std::cos(std::min(sc.half_angle, M_PI));
        pk[7] = sc.half_angle >= M_PI ? 1.0 : 0.0;
        pk[11] = -1.0;  // cone
        if (sc.fan_half_thickness > 0 && sc.half_angle < M_PI) {
            // fan-plane normal: its part orthogonal to the axis, unit length
            const double a2 = sc.axis[0] * sc.axis[0] + sc.axis[1] * sc.axis[1] + sc.axis[2] * sc.axis[2];
            const double na = (sc.fan_normal[0] * sc.axis[0] + sc.fan_normal[1] * sc.axis[1] +
                               sc.fan_normal[2] * sc.axis[2]) / a2;
            double nrm[3], l2 = 0.0;
            for (int t = 0; t < 3; ++t) {
                nrm[t] = sc.fan_normal[t] - na * sc.axis[t];
                l2 += nrm[t] * nrm[t];
            }
            for (int t = 0; t < 3; ++t) pk[8 + t] = nrm[t] / std::sqrt(l2);
            pk[11] = std::sin(sc.fan_half_thickness);
        }
        std::memcpy(&spec[(size_t)k * G], sc.spectrum, G * sizeof(double));
    }
    DSN_HIP(hipMemcpyAsync((void *)ar.src_par, par.data(), par.size() * sizeof(double), hipMemcpyHostToDevice,
                           s));
    DSN_HIP(hipMemcpyAsync((void *)ar.src_spec, spec.data(), spec.size() * sizeof(double), hipMemcpyHostToDevice,
                           s));
    DSN_HIP(hipStreamSynchronize(s));
    return DSN_OK;
}

template <typename T>
dsn_status solve_sources(dsn_problem *p, const dsn_source *src, int32_t n_src, const dsn_solve_opts &o,
                         double *phi_total, double *phi_unc, dsn_solve_info *info, hipStream_t s, int max_batch = 0)
{
    DeviceState &d = p->dev;
    d.wait_limit = o.wait_limit;
    d.tune_pending = o.autotune == 1 && !d.tuned;
    const Geom &gm = p->geom;
    const int G = p->G;
    dsn_status worst = DSN_OK;
    double updates = 0.0;
    // combine: all n_src sources act together in one solve (their
    // uncollided fluences and first-collision sources add up; one collided
    // solution), e.g. the cone beams of a CT ring
    const bool combine = o.combine_sources != 0;
    const int limit = combine ? n_src : max_batch > 0 ? max_batch : batch_limit(p);
    for (int b0 = 0; b0 < n_src; b0 += limit) {
        const int S = std::min(limit, n_src - b0);  // sources ray traced
        dsn_status st = combine ? ensure_combined(p, S) : ensure_batch(p, S);
        if (st != DSN_OK) return st;
        SolveArgs<T> a = make_args<T>(p, combine ? 1 : S);
        SolveArgs<T> ar = a;  // the ray traces: one per source
        ar.S = S;
        if (combine) {
            ar.phiu = d.c_phiu;
            ar.oms = d.c_oms;
            ar.src_par = d.c_par;
            ar.src_spec = d.c_spec;
        }
        st = upload_sources<T>(p, ar, src + b0, S, s);
        if (st != DSN_OK) return st;
        size_t ev = d.timer.begin();
        launch_raytrace<T>(ar, s);
        if (combine) {
            // one collided solve driven by the summed first-collision source
            launch_sum_uncollided<T>(ar, S, d.c_usum, d.c_pusum, s);
            a.phiu = d.c_pusum;
            a.usum = d.c_usum;
        }
        d.timer.end(DSN_STAGE_SETUP, ev, combine ? 2 : 1);
        const int Sc = a.S;  // sources with a collided solution in this pass
        int chunk_hint = 4;
        double *pt = phi_total + (size_t)b0 * G * gm.V;
        double *pu = phi_unc ? phi_unc + (size_t)b0 * G * gm.V : nullptr;
        for (int g = 0; g < G; ++g) {
            ev = d.timer.begin();
            launch_group_source<T>(a, g, true, s);  // also forms the first directional source
            d.timer.end(DSN_STAGE_SETUP, ev, 1);
            st = iterate_group<T>(p, a, g, o, s, chunk_hint, true, o.stop_rule);
            if (st != DSN_OK) return st;
            ev = d.timer.begin();
            launch_finalize<T>(a, g, pt, pu, s);
            d.timer.end(DSN_STAGE_SETUP, ev, 1);
            if (d.timer.on) {
                DSN_HIP(hipStreamSynchronize(s));
                d.timer.flush();
            }
        }
        DSN_HIP(hipGetLastError());
        DSN_HIP(hipMemcpyAsync(d.h_ctl, d.ctl, (size_t)Sc * G * sizeof(Ctl), hipMemcpyDeviceToHost, s));
        DSN_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < Sc; ++k) {
            const Ctl *c = d.h_ctl + (size_t)k * G;
            for (int g = 0; g < G; ++g) {
                if (info && info->iters) info->iters[(size_t)(b0 + k) * G + g] = c[g].iters;
                if (info && info->residual) info->residual[(size_t)(b0 + k) * G + g] = c[g].r;
                updates += (double)c[g].iters * (double)gm.V * (double)p->Nd;
            }
            st = status_of(c, G);
            if (st == DSN_ERR_NUMERICAL) return st;
            if (st != DSN_OK) worst = st;
        }
        int flags[2] = {0, 0};
        DSN_HIP(hipMemcpyAsync(flags, d.sweep_ctr, sizeof(flags), hipMemcpyDeviceToHost, s));
        DSN_HIP(hipStreamSynchronize(s));
        if (flags[1]) return sweep_failed(p, flags[1]);
    }
    if (info) {
        info->updates = updates;
        info->sweep_bytes = updates * 2.0 * sizeof(T);
    }
    if (worst != DSN_OK) g_err = "max_iters reached before tol";
    return worst;
}

// ---------------------------------------------------------------------------
// Fused batch (dsn_solve_batch, batch_mode 1): every problem of the
// batch iterates the same group in lockstep on one stream, and each source
// iteration is one sweep launch over every (problem, source) pair - the
// problems' argument blocks in a device table, their tickets merged diagonal
// by diagonal - followed by one moments launch and one convergence-test
// launch over every pair (the same tables), the whole iteration replayed as
// one HIP graph.  A problem whose sources' group has
// converged leaves the later launches of that group at once, as in a single
// solve.  Results equal those of the problems solved one by one (the same
// kernels and arithmetic; the launch shape changes no result).
// ---------------------------------------------------------------------------
constexpr int kFacesFused = 9;  // face words written by a fused batch (the next single sweep invalidates them)

// Why a fused batch cannot run these problems ("" if it can).
std::string fused_obstacle(dsn_problem *const *probs, int32_t n_probs, const int32_t *n_src)
{
    const dsn_problem *first = nullptr;
    int n = 0;
    for (int b = 0; b < n_probs; ++b) {
        if (n_src[b] == 0) continue;
        const dsn_problem *p = probs[b];
        if (!first) first = p;
        if (p->fixup != first->fixup || p->has_density != first->has_density)
            return "the problems differ in the fixup or in having a per-voxel density";
        ++n;
    }
    if (n > 0xFFFF) return "too many problems";
    if (first && first->Nd * (double)first->geom.NJ * first->geom.NK > 1e9) return "too many sweep items";
    return "";
}

// One round of a fused batch: n_src[b] sources srcs[b] of problem b (their
// results to phi_total[b], their iteration counts to iters[b] [n_src[b]][G]
// when given).  tune: time the fused launch's shapes at the first group.
template <typename T>
dsn_status fused_round(dsn_problem *const *probs, int32_t n_probs, const dsn_source *const *srcs,
                       const int32_t *n_src, const dsn_solve_opts &o, double *const *phi_total,
                       int32_t *const *iters, bool tune_shape, double &updates, int shape[2], hipStream_t s)
{
    constexpr bool fp64 = sizeof(T) == 8;
    std::vector<int> ids;
    for (int b = 0; b < n_probs; ++b)
        if (n_src[b] > 0) ids.push_back(b);
    const int n = (int)ids.size();
    if (n == 0) return DSN_OK;
    dsn_problem *const p0 = probs[ids[0]];
    const int G = p0->G, D = p0->D, mode = p0->fixup;
    dsn_status st;
    // every problem's device state, source buffers (face words cleared: this
    // batch's sweeps stamp them from a counter block of their own) and ray traces
    std::vector<SolveArgs<T>> tab(n);
    double psi_bytes = 0.0, items = 0.0;
    for (int q = 0; q < n; ++q) {
        dsn_problem *p = probs[ids[q]];
        const int S = n_src[ids[q]];
        if ((st = ensure_device(p)) != DSN_OK || (st = ensure_batch(p, S)) != DSN_OK) return st;
        DeviceState &d = p->dev;
        d.wait_limit = o.wait_limit;
        d.timer.on = false;
        if ((st = invalidate_faces(d, (size_t)d.S_cap_alloc * sizes_of(p).face)) != DSN_OK) return st;
        d.face_tagged = kFacesFused;
        tab[q] = make_args<T>(p, S);
        if ((st = upload_sources<T>(p, tab[q], srcs[ids[q]], S, s)) != DSN_OK) return st;
        launch_raytrace<T>(tab[q], s);
        psi_bytes += (double)S * p->Nd * (double)p->geom.Vp * sizeof(T);
        items += (double)S * sweep_items(p, 1);
    }
    if (items >= (double)(1 << 29)) return fail(DSN_ERR_UNSUPPORTED, "too many sweep items in one fused batch");
    int dev = 0, n_cu = 0;
    DSN_HIP(hipGetDevice(&dev));
    DSN_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    int wl[8];
    const int nw = sweep_multi_choices(fp64, wl);
    std::vector<int> cand_w;
    for (int i = 0; i < nw; ++i)
        if (D % wl[i] == 0 && sweep_grid_multi<T>(wl[i], mode, n_cu) > 0) cand_w.push_back(wl[i]);
    if (cand_w.empty()) return fail(DSN_ERR_UNSUPPORTED, "no fused sweep kernel for this angular order");
    int W = cand_w[0];
    for (int w : cand_w)
        if (w == sweep_wpb(D, fp64)) W = w;
    // per-call device memory: the problems' table, the segments and the counter block
    struct Mem {
        std::vector<void *> v;
        ~Mem()
        {
            for (void *x : v) (void)hipFree(x);
        }
    } mem;
    auto alloc = [&](size_t bytes) -> void * {
        void *x = nullptr;
        if (hipMalloc(&x, bytes) != hipSuccess) return nullptr;
        mem.v.push_back(x);
        return x;
    };
    // the launch's own argument block (multi set), its merged ticket order
    SolveArgs<T> M = tab[0];
    std::vector<int> seg;
    int *seg_dev = nullptr;
    int maxdiag = 0;
    for (int q = 0; q < n; ++q) maxdiag = std::max(maxdiag, tab[q].g.NJ + tab[q].g.NK - 1);
    // the merged ticket order for w directions per block: segment (diagonal
    // dd, problem q) for dd = 0, 1, ... and the problems in order
    auto build_segments = [&](int w) {
        std::vector<int> start, code;
        long t = 0;
        for (int dd = 0; dd < maxdiag; ++dd)
            for (int q = 0; q < n; ++q) {
                const int NJ = tab[q].g.NJ, NK = tab[q].g.NK;
                if (dd > NJ + NK - 2) continue;
                const int lo = std::max(0, dd - (NK - 1)), hi = std::min(dd, NJ - 1);
                start.push_back((int)t);
                code.push_back(q << 16 | dd);
                t += (long)(hi - lo + 1) * 8 * (D / w) * tab[q].S;
            }
        M.nseg = (int)start.size();
        seg = start;
        seg.push_back((int)t);
        seg.insert(seg.end(), code.begin(), code.end());
        M.sweep_nitems = (int)t;
    };
    SolveArgs<T> *tab_dev = (SolveArgs<T> *)alloc(n * sizeof(SolveArgs<T>));
    int *ctr_dev = (int *)alloc(kCtrInts * sizeof(int));
    build_segments(W);
    seg_dev = (int *)alloc(seg.size() * sizeof(int));
    if (!tab_dev || !ctr_dev || !seg_dev) return fail(DSN_ERR_OUT_OF_MEMORY, "hipMalloc failed (fused batch tables)");
    DSN_HIP(hipMemcpyAsync(tab_dev, tab.data(), n * sizeof(SolveArgs<T>), hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemsetAsync(ctr_dev, 0, kCtrInts * sizeof(int), s));
    M.multi = tab_dev;
    M.nmulti = n;
    M.seg = seg_dev;
    M.sweep_ctr = ctr_dev;
    M.sweep_xcd = 0;
    M.sweep_relay = 0;
    M.sweep_mode = mode;
    M.stream_nt = psi_bytes > 256.0 * 1024 * 1024 ? 1 : 0;
    M.sweep_spin_limit = o.wait_limit > 0 ? o.wait_limit : kDefaultWaitLimit;
    auto set_shape = [&](int w, int grid) -> dsn_status {
        build_segments(w);
        M.sweep_wpb = w;
        M.sweep_grid = grid;
        DSN_HIP(hipMemcpyAsync(seg_dev, seg.data(), seg.size() * sizeof(int), hipMemcpyHostToDevice, s));
        DSN_HIP(hipStreamSynchronize(s));  // seg is rewritten by the next call
        return DSN_OK;
    };
    if ((st = set_shape(W, sweep_grid_multi<T>(W, mode, n_cu))) != DSN_OK) return st;
    auto sweep_all = [&](int g, hipStream_t on, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
        launch_sweep_multi<T>(M, tab.data(), n, g, on, e0, e1);
    };
    // one source iteration: the fused sweep, then the moments and the
    // convergence test of every (problem, source) pair, two more launches
    long vp_max = 0;
    int s_max = 0;
    for (int q = 0; q < n; ++q) {
        vp_max = std::max(vp_max, tab[q].g.Vp);
        s_max = std::max(s_max, tab[q].S);
    }
    auto unit = [&](int g, hipStream_t on) {
        sweep_all(g, on);
        launch_d2m_multi<T>(M.multi, tab[0], n, vp_max, s_max, M.stream_nt != 0, g, on);
    };
    // the fused sweep's launch shape: every built waves-per-block value that
    // divides the directions of an octant, full, 3/4 and 1/2 resident grid,
    // one untimed and two timed launches each on the first group's source
    // (formed again from the moments before every launch and at the end)
    auto tune = [&](int g) -> dsn_status {
        struct Events {
            hipEvent_t e[2] = {nullptr, nullptr};
            ~Events()
            {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } evs;
        hipEvent_t *ev = evs.e;
        DSN_HIP(hipEventCreate(&ev[0]));
        DSN_HIP(hipEventCreate(&ev[1]));
        float best = 1e30f;
        int bw = M.sweep_wpb, bg = M.sweep_grid;
        for (int w : cand_w) {
            const int full = sweep_grid_multi<T>(w, mode, n_cu);
            for (int f = 4; f >= 2; --f) {
                if ((st = set_shape(w, std::max(1, full * f / 4))) != DSN_OK) return st;
                float tot = 0.f;
                for (int r = 0; r < 3; ++r) {
                    for (int q = 0; q < n; ++q) launch_m2d<T>(tab[q], g, s);
                    sweep_all(g, s, ev[0], ev[1]);
                    DSN_HIP(hipEventSynchronize(ev[1]));
                    float ms = 0.f;
                    DSN_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
                    if (r) tot += ms;
                }
                if (tot < best) {
                    best = tot;
                    bw = w;
                    bg = M.sweep_grid;
                }
            }
        }
        int flags[2] = {0, 0};
        DSN_HIP(hipMemcpy(flags, M.sweep_ctr, sizeof(flags), hipMemcpyDeviceToHost));
        if (flags[1]) return fail(DSN_ERR_DEVICE, "a sweep wait timed out while timing the fused launch shapes");
        for (int q = 0; q < n; ++q) launch_m2d<T>(tab[q], g, s);
        return set_shape(bw, bg);
    };
    // the steady iteration of group g as one graph (direct launches if
    // capture is not available)
    hipStream_t cap = nullptr;
    std::vector<hipGraphExec_t> graphs;
    struct GraphsGuard {
        std::vector<hipGraphExec_t> &g;
        hipStream_t &c;
        ~GraphsGuard()
        {
            for (hipGraphExec_t x : g) (void)hipGraphExecDestroy(x);
            if (c) (void)hipStreamDestroy(c);
        }
    } graphs_guard{graphs, cap};
    auto graph_of = [&](int g) -> hipGraphExec_t {
        if (!cap && hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) {
            cap = nullptr;
            return nullptr;
        }
        std::shared_lock<std::shared_mutex> lk(g_capture_gate, std::defer_lock);
        if (t_gate_depth == 0) lk.lock();
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
        unit(g, cap);
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = ec == hipSuccess ? hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) : ec;
        if (graph) (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        graphs.push_back(exec);
        return exec;
    };
    int chunk_hint = 4;
    std::vector<Ctl> hc;
    for (int g = 0; g < G; ++g) {
        const int target = o.fixed_iters ? o.fixed_iters[g] : -1;
        for (int q = 0; q < n; ++q) {
            launch_group_source<T>(tab[q], g, true, s);  // also forms the first directional source
            launch_ctl_init(tab[q].ctl, G, tab[q].S, g, target, o.max_iters, o.fixed_iters ? 0.0 : o.tol,
                            o.stagnation_stop, o.stop_rule, s);
        }
        if (g == 0 && tune_shape && (st = tune(g)) != DSN_OK) return st;
        DSN_HIP(hipGetLastError());
        hipGraphExec_t gx = nullptr;
        auto enqueue = [&](int count) {
            for (int c = 0; c < count; ++c) {
                if (!gx) gx = graph_of(g);
                if (!gx || hipGraphLaunch(gx, s) != hipSuccess) unit(g, s);
            }
        };
        if (target >= 0) {
            enqueue(target);
        } else {
            int enq = 0, chunk = std::max(1, chunk_hint), most = 0;
            for (;;) {
                enqueue(chunk);
                enq += chunk;
                DSN_HIP(hipGetLastError());
                bool all = true;
                most = 0;
                for (int q = 0; q < n; ++q) {
                    const SolveArgs<T> &a = tab[q];
                    hc.resize((size_t)a.S * G);
                    DSN_HIP(hipMemcpyAsync(hc.data(), a.ctl, hc.size() * sizeof(Ctl), hipMemcpyDeviceToHost, s));
                    DSN_HIP(hipStreamSynchronize(s));
                    for (int k = 0; k < a.S; ++k) {
                        all = all && hc[(size_t)k * G + g].done;
                        most = std::max(most, hc[(size_t)k * G + g].iters);
                    }
                }
                if (all || enq >= o.max_iters) break;
                chunk = 2;
            }
            chunk_hint = std::max(1, most - 2);
        }
        for (int q = 0; q < n; ++q)
            launch_finalize<T>(tab[q], g, phi_total[ids[q]], nullptr, s);
    }
    DSN_HIP(hipGetLastError());
    DSN_HIP(hipStreamSynchronize(s));
    int flags[2] = {0, 0};
    DSN_HIP(hipMemcpy(flags, M.sweep_ctr, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[1]) {
        for (int q = 0; q < n; ++q) (void)invalidate_faces(probs[ids[q]]->dev, (size_t)probs[ids[q]]->dev.S_cap_alloc *
                                                                                sizes_of(probs[ids[q]]).face);
        return fail(DSN_ERR_DEVICE, "a sweep wait timed out (fused batch); results are invalid");
    }
    // iteration counts
    dsn_status worst = DSN_OK;
    for (int q = 0; q < n; ++q) {
        const SolveArgs<T> &a = tab[q];
        hc.resize((size_t)a.S * G);
        DSN_HIP(hipMemcpy(hc.data(), a.ctl, hc.size() * sizeof(Ctl), hipMemcpyDeviceToHost));
        int32_t *it = iters ? iters[ids[q]] : nullptr;
        for (int k = 0; k < a.S; ++k) {
            const Ctl *c = &hc[(size_t)k * G];
            for (int g = 0; g < G; ++g) {
                if (it) it[(size_t)k * G + g] = c[g].iters;
                updates += (double)c[g].iters * (double)a.g.V * (double)a.Nd;
            }
            const dsn_status sk = status_of(c, G);
            if (sk == DSN_ERR_NUMERICAL) return sk;
            if (sk != DSN_OK) worst = sk;
        }
    }
    shape[0] = M.sweep_wpb;
    shape[1] = M.sweep_grid;
    return worst;
}

// Frees a problem's per-source buffers (they are allocated again, for the
// sources asked for, by the next call that needs them).
void release_sources(dsn_problem *p)
{
    DeviceWide gate;
    DeviceState &d = p->dev;
    if (d.src_allocs.empty()) return;
    (void)hipDeviceSynchronize();
    for (void *q : d.src_allocs) (void)hipFree(q);
    d.src_allocs.clear();
    d.bytes -= d.src_bytes;
    d.src_bytes = 0;
    d.S_cap = 0;
    d.S_cap_alloc = 0;
    d.dstart_S = 0;
    if (d.h_ctl) (void)hipHostFree(d.h_ctl);
    d.h_ctl = nullptr;
}

// Sources per batch of every problem of a dsn_solve_batch call, chosen
// together so that all problems' per-source buffers fit in device memory at
// the same time (at most 64 a problem, as in a single solve).  A problem that
// holds buffers for more sources than it will use gives them back first when
// another one has to grow.
dsn_status joint_batch_limits(dsn_problem *const *probs, int32_t n_probs, const int32_t *n_src, std::vector<int> &m)
{
    for (int b = 0; b < n_probs; ++b)
        if (n_src[b] > 0) {
            dsn_status st = ensure_device(probs[b]);
            if (st != DSN_OK) return st;
        }
    size_t free_b = 0, total_b = 0;
    DSN_HIP(hipMemGetInfo(&free_b, &total_b));
    double held = 0.0, need = 0.0;
    m.assign(n_probs, 0);
    for (int b = 0; b < n_probs; ++b) {
        if (n_src[b] == 0) continue;
        held += (double)probs[b]->dev.src_bytes;
        m[b] = std::min(64, (int)n_src[b]);
        need += (double)m[b] * (double)per_source_bytes(probs[b]);
    }
    const double avail = 0.8 * ((double)free_b + held);
    if (need > avail)
        for (int b = 0; b < n_probs; ++b)
            if (m[b] > 0) m[b] = std::max(1, (int)((double)m[b] * avail / need));
    bool grow = false;
    for (int b = 0; b < n_probs; ++b) grow = grow || m[b] > probs[b]->dev.S_cap;
    if (grow)
        for (int b = 0; b < n_probs; ++b)
            if (m[b] > 0 && probs[b]->dev.S_cap > m[b]) release_sources(probs[b]);
    return DSN_OK;
}

// A fused batch in rounds: each round takes up to m_b of problem b's
// remaining sources, the m_b chosen so that every problem's buffers for
// its round fit in device memory together (at most 64 sources a problem,
// like a single solve's batches).
template <typename T>
dsn_status solve_batch_fused(dsn_problem *const *probs, int32_t n_probs, const dsn_source *const *srcs,
                             const int32_t *n_src, const dsn_solve_opts &o, double *const *phi_total,
                             dsn_solve_info *info, hipStream_t s)
{
    std::vector<int> m;
    dsn_status st0 = joint_batch_limits(probs, n_probs, n_src, m);
    if (st0 != DSN_OK) return st0;
    std::vector<int> done(n_probs, 0), rowstart(n_probs, 0);
    for (int b = 1; b < n_probs; ++b) rowstart[b] = rowstart[b - 1] + n_src[b - 1];
    const int G = probs[0]->G;
    double updates = 0.0;
    int shape[2] = {0, 0};
    dsn_status worst = DSN_OK;
    for (int round = 0;; ++round) {
        std::vector<int32_t> cnt(n_probs, 0);
        std::vector<const dsn_source *> sp(n_probs, nullptr);
        std::vector<double *> out(n_probs, nullptr);
        std::vector<int32_t *> it(n_probs, nullptr);
        bool any = false;
        for (int b = 0; b < n_probs; ++b) {
            cnt[b] = std::min(m[b], (int)n_src[b] - done[b]);
            if (cnt[b] <= 0) {
                cnt[b] = 0;
                continue;
            }
            any = true;
            sp[b] = srcs[b] + done[b];
            out[b] = phi_total[b] + (size_t)done[b] * G * probs[b]->geom.V;
            it[b] = info && info->iters ? info->iters + (size_t)(rowstart[b] + done[b]) * G : nullptr;
        }
        if (!any) break;
        const dsn_status st = fused_round<T>(probs, n_probs, sp.data(), cnt.data(), o, out.data(), it.data(),
                                             round == 0 && o.autotune == 1, updates, shape, s);
        if (st != DSN_OK && st != DSN_ERR_NOT_CONVERGED) return st;
        if (st != DSN_OK) worst = st;
        for (int b = 0; b < n_probs; ++b) done[b] += cnt[b];
    }
    if (info) {
        info->updates = updates;
        info->sweep_bytes = updates * 2.0 * sizeof(T);
        info->sweep_waves_per_block = shape[0];
        info->sweep_blocks = shape[1];
        info->sweep_xcd_queues = 0;
        info->sweep_relay = 0;
    }
    return worst;
}

dsn_status ensure_adjoint(dsn_problem *p)
{
    DeviceState &d = p->dev;
    if (d.adj_ready) return DSN_OK;
    const Sizes s = sizes_of(p);
    dsn_status st;
    if ((st = dev_alloc(d, (void **)&d.phia, s.phic)) != DSN_OK) return st;
    if ((st = dev_alloc(d, &d.psi2, s.psi)) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.ctl_adj, s.ctl)) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.ctl_free, s.ctl)) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.wdir, (size_t)p->Nd * sizeof(double))) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.phit_tmp, (size_t)p->G * p->geom.V * sizeof(double))) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.dot_part, 1024 * sizeof(double))) != DSN_OK) return st;
    if ((st = dev_alloc(d, (void **)&d.dot_out, sizeof(double))) != DSN_OK) return st;
    if (p->fixup) {
        // the adjoint sweeps (tagged words) get face buffers of their own, so
        // they never meet the forward sweeps' sign-parity words
        if ((st = dev_alloc(d, (void **)&d.mask, (size_t)p->Nd * p->geom.Vp)) != DSN_OK) return st;
        if ((st = dev_alloc(d, &d.afaceY, s.face)) != DSN_OK) return st;
        if ((st = dev_alloc(d, &d.afaceZ, s.face)) != DSN_OK) return st;
        DeviceWide gate;
        DSN_HIP(hipMemset(d.afaceY, 0xFF, s.face));
        DSN_HIP(hipMemset(d.afaceZ, 0xFF, s.face));
        DSN_HIP(hipDeviceSynchronize());
    }
    DSN_HIP(hipMemcpy(d.wdir, p->w.data(), (size_t)p->Nd * sizeof(double), hipMemcpyHostToDevice));
    d.adj_ready = true;
    return DSN_OK;
}

__global__ void k_fill_zero(double *x, long n)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

template <typename T>
dsn_status adjoint_impl(dsn_problem *p, const dsn_source &src, const double *W, const dsn_solve_opts &o, double *J,
                        double *grad, double *phi_total_user, dsn_solve_info *info, hipStream_t s)
{
    DeviceState &d = p->dev;
    d.wait_limit = o.wait_limit;
    const int G = p->G;
    const long V = p->geom.V;
    double *phit = phi_total_user ? phi_total_user : d.phit_tmp;
    // forward solve (keeps every group's converged moments on the device)
    dsn_solve_info fi;
    std::vector<int32_t> it_f(G);
    fi.iters = it_f.data();
    fi.residual = nullptr;
    dsn_status st = solve_sources<T>(p, &src, 1, o, phit, nullptr, &fi, s, 1);
    if (st != DSN_OK && st != DSN_ERR_NOT_CONVERGED) return st;
    dsn_status worst = st;
    launch_dot(W, phit, (long)G * V, d.dot_part, 1024, d.dot_out, s);
    DSN_HIP(hipMemcpyAsync(J, d.dot_out, sizeof(double), hipMemcpyDeviceToHost, s));
    // adjoint source iteration, lowest-energy group first, reversed sweeps
    // With the fixup the forward solve is linearised with every cell's set
    // of fixed axes frozen at the converged solution: before a group's
    // adjoint iterations one forward sweep from its converged moments records
    // the sets (kRecord), and the adjoint sweeps use the transposed frozen
    // cell (kTrans) on face buffers of their own.
    const bool fx = p->fixup != 0;
    SolveArgs<T> aa = make_args<T>(p);
    aa.phic = d.phia;
    aa.ctl = d.ctl_adj;
    aa.rev = 1;
    if (fx) {
        aa.sweep_mode = 3;
        aa.mask = d.mask;
        aa.faceY = (unsigned long long *)d.afaceY;
        aa.faceZ = (unsigned long long *)d.afaceZ;
    }
    for (int g = 0; g < G; ++g) launch_ctl_init(d.ctl_free, G, 1, g, -1, 1, 1.0, 0, 0, s);
    SolveArgs<T> fw = make_args<T>(p);  // forward recomputation from the converged moments
    fw.ctl = d.ctl_free;
    if (fx) {
        fw.sweep_mode = 2;
        fw.mask = d.mask;
    }
    int chunk = 4;
    double updates = fi.updates;
    for (int g = G - 1; g >= 0; --g) {
        if (fx) {
            launch_group_source_keep<T>(fw, g, s);
            launch_m2d_always<T>(fw, g, s);
            sweep_forward_faces<T>(p, fw, g, s);
        }
        launch_adj_source<T>(aa, g, W, 1, s);
        // the adjoint iterations stop on the L2 change (rule 0) whatever the forward rule
        if ((st = iterate_group<T>(p, aa, g, o, s, chunk, false, 0)) != DSN_OK) return st;
    }
    DSN_HIP(hipGetLastError());
    DSN_HIP(hipMemcpyAsync(d.h_ctl, d.ctl_adj, G * sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DSN_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> it_a(G);
    for (int g = 0; g < G; ++g) {
        it_a[g] = d.h_ctl[g].iters;
        updates += (double)d.h_ctl[g].iters * (double)V * (double)p->Nd;
    }
    st = status_of(d.h_ctl, G);
    if (st == DSN_ERR_NUMERICAL) return st;
    if (st != DSN_OK) worst = st;
    // gradient: recompute psi^g (forward) and chi^g (adjoint) from the converged
    // moments, one group at a time, then the ray back-projection
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((V + 255) / 256)), dim3(256), 0, s, grad, V);
    SolveArgs<T> ad = aa;
    ad.ctl = d.ctl_free;
    ad.psi = (T *)d.psi2;
    for (int g = 0; g < G; ++g) {
        launch_group_source_keep<T>(fw, g, s);
        launch_m2d_always<T>(fw, g, s);
        sweep_forward_faces<T>(p, fw, g, s);
        launch_adj_source<T>(ad, g, W, 0, s);
        launch_m2d_always<T>(ad, g, s);
        sweep_forward_faces<T>(p, ad, g, s);
        launch_grad_accum<T>(fw, ad, g, grad, s);
    }
    launch_backproject<T>(fw, d.phia, W, src.position, grad, s);
    DSN_HIP(hipGetLastError());
    DSN_HIP(hipStreamSynchronize(s));
    int flags[2] = {0, 0};
    DSN_HIP(hipMemcpy(flags, d.sweep_ctr, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[1]) return sweep_failed(p, flags[1]);
    if (info) {
        if (info->iters)
            for (int g = 0; g < G; ++g) {
                info->iters[g] = it_f[g];
                info->iters[G + g] = it_a[g];
            }
        info->updates = updates + 2.0 * G * (double)V * p->Nd;
    }
    if (worst != DSN_OK) g_err = "max_iters reached before tol";
    return worst;
}

// ---------------------------------------------------------------------------
// Forward solve that allocates nothing (dsn_solve_noalloc), for callers that
// cannot allocate device memory.  Every device array of the solve - the
// problem tables in pencil order, the angular fluence, the moments, the face
// words, the sweep's counters and the residual partials - is carved out of
// one file-scope device array.  Each GPU holds its own copy of the array
// until the process ends; its device address comes from hipGetSymbolAddress
// once per device and is the only way host code refers to it.  Every call on
// a GPU reuses that GPU's array: whatever a call needs to start from a known
// state (sweep counters, face words, face parity) is cleared by a fill kernel
// at the start of the call, and calls that overlap on one GPU race.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxScratchDevices];
int g_scratch_ncu[kMaxScratchDevices];

// The device address of the current device's scratch array and its compute
// unit count (looked up once per device, with that device current).
dsn_status scratch_of(unsigned char **ptr, int *n_cu)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail(DSN_ERR_DEVICE, "no HIP device available");
    int dev = 0;
    DSN_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(DSN_ERR_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        hipDeviceProp_t prop;
        DSN_HIP(hipGetDeviceProperties(&prop, dev));
        if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
            return fail(DSN_ERR_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
        void *q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return fail(DSN_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ncu[dev] = prop.multiProcessorCount;
        g_scratch_ptr[dev] = (unsigned char *)q;
    }
    *ptr = g_scratch_ptr[dev];
    *n_cu = g_scratch_ncu[dev];
    return DSN_OK;
}

__global__ void k_fill_u32(unsigned *x, long n, unsigned v)
{
    const long i = blockIdx.x * 256L + threadIdx.x;
    if (i < n) x[i] = v;
}

void fill_u32(void *x, size_t bytes, unsigned v, hipStream_t s)
{
    const long n = (long)(bytes / 4);
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (unsigned *)x, n, v);
}

// Bump carving of the scratch array, 256-byte aligned pieces.  With base
// null it only counts.
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <typename X>
    X *take(size_t bytes)
    {
        const size_t o = (off + 255) & ~size_t(255);
        off = o + (bytes ? bytes : 16);
        return base ? (X *)(base + o) : nullptr;
    }
};

// The arguments of a one-source solve with every array carved from c.
template <typename T>
SolveArgs<T> carve_args(dsn_problem *p, Carve &c, int wpb, int relay, int grid, uint8_t **mat_nat, double **dens_nat)
{
    const Geom &g = p->geom;
    const Sizes z = sizes_of(p);
    SolveArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.g = g;
    a.G = p->G;
    a.L = p->L;
    a.Nm = p->Nm;
    a.Nd = p->Nd;
    a.D = p->D;
    a.nmat = p->nmat;
    *mat_nat = c.take<uint8_t>((size_t)g.V);
    *dens_nat = p->has_density ? c.take<double>((size_t)g.V * sizeof(double)) : nullptr;
    a.mat_nat = *mat_nat;
    a.dens_nat = *dens_nat;
    a.mat = c.take<uint8_t>(z.mat);
    a.dens = c.take<double>(z.dens);
    a.xs_t = c.take<double>(z.xs_t);
    a.xs_s = c.take<double>(z.xs_s);
    a.M0 = c.take<T>(z.M0);
    a.D0 = c.take<double>(z.D0);
    a.cdir = c.take<T>(z.cdir);
    a.phiu = c.take<double>(z.phiu);
    a.oms = c.take<double>(z.oms);
    a.phic = c.take<double>(z.phic);
    a.F = c.take<T>(z.F);
    a.usum = nullptr;
    a.sig = c.take<T>(z.sig);
    a.psi = c.take<T>(z.psi);
    a.faceY = c.take<unsigned long long>(z.face);
    a.faceZ = c.take<unsigned long long>(z.face);
    a.part = c.take<double>(z.part);
    a.ctl = c.take<Ctl>(z.ctl);
    a.sweep_ctr = c.take<int>(kCtrInts * sizeof(int));
    a.sweep_dstart = c.take<int>(((size_t)g.NJ + g.NK + 1) * sizeof(int));
    a.face_par = c.take<int>(sizeof(int));
    a.src_par = c.take<double>(kSrcPar * sizeof(double));
    a.src_spec = c.take<double>(z.spec);
    a.sweep_nitems = sweep_items(p, wpb, relay);
    a.sweep_grid = grid;
    a.sweep_wpb = wpb;
    a.sweep_xcd = 0;
    a.sweep_relay = relay;
    a.sweep_mode = p->fixup;
    a.mask = nullptr;
    a.sweep_spin_limit = kDefaultWaitLimit;
    a.rev = 0;
    a.sig_from_mat = p->has_density ? 0 : 1;
    a.stream_nt = 0;  // the whole working set is far below the last-level cache
    a.wdir = nullptr;
    a.S = 1;
    return a;
}

template <typename T>
dsn_status solve_noalloc(dsn_problem *p, const dsn_source &src, const dsn_solve_opts &o, double *phi_total,
                         double *phi_unc, dsn_solve_info *info, hipStream_t s)
{
    const bool fp64 = sizeof(T) == 8;
    // the handle's launch shape when it has one on the global queue, else
    // the default shape (the sizes do not depend on the shape)
    const DeviceState &d = p->dev;
    int wpb = sweep_wpb(p->D, fp64), grid = 0, relay = 0;
    if (d.ready && d.tuned && d.xcd_use == 0) {
        wpb = d.wpb;
        grid = d.sweep_grid;
        relay = d.relay;
    }
    uint8_t *mat_nat = nullptr;
    double *dens_nat = nullptr;
    Carve count{nullptr};
    (void)carve_args<T>(p, count, wpb, relay, 1, &mat_nat, &dens_nat);
    if (count.off > kScratchBytes)
        return fail(DSN_ERR_UNSUPPORTED, "dsn_solve_noalloc: the solve needs " + std::to_string(count.off) +
                                             " bytes of device memory, above its fixed maximum of " +
                                             std::to_string(kScratchBytes));
    if ((double)sweep_items(p, wpb, relay) >= (double)(1 << 29))
        return fail(DSN_ERR_UNSUPPORTED, "too many sweep items (directions x pencils)");
    unsigned char *base = nullptr;
    int n_cu = 0;
    dsn_status st = scratch_of(&base, &n_cu);
    if (st != DSN_OK) return st;
    if (grid < 1) grid = sweep_grid<T>(wpb, p->fixup, n_cu);
    if (grid < 1) return fail(DSN_ERR_UNSUPPORTED, "no sweep kernel of this shape fits the device");
    Carve c{base};
    SolveArgs<T> a = carve_args<T>(p, c, wpb, relay, grid, &mat_nat, &dens_nat);
    const Geom &gm = p->geom;
    const Sizes z = sizes_of(p);
    const int G = p->G;
    a.sweep_spin_limit = o.wait_limit > 0 ? o.wait_limit : kDefaultWaitLimit;
    // problem tables and source parameters (host -> device copies only, from
    // host memory the handle owns, so every copy's source outlives it)
    double *par = p->par_host;
    for (int t = 0; t < 3; ++t) {
        par[t] = src.position[t];
        par[3 + t] = src.axis[t];
        par[8 + t] = 0.0;
    }
    par[6] = std::cos(std::min(src.half_angle, M_PI));
    par[7] = src.half_angle >= M_PI ? 1.0 : 0.0;
    par[11] = -1.0;  // cone
    if (src.fan_half_thickness > 0 && src.half_angle < M_PI) {
        const double a2 = src.axis[0] * src.axis[0] + src.axis[1] * src.axis[1] + src.axis[2] * src.axis[2];
        const double na =
            (src.fan_normal[0] * src.axis[0] + src.fan_normal[1] * src.axis[1] + src.fan_normal[2] * src.axis[2]) / a2;
        double nrm[3], l2 = 0.0;
        for (int t = 0; t < 3; ++t) {
            nrm[t] = src.fan_normal[t] - na * src.axis[t];
            l2 += nrm[t] * nrm[t];
        }
        for (int t = 0; t < 3; ++t) par[8 + t] = nrm[t] / std::sqrt(l2);
        par[11] = std::sin(src.fan_half_thickness);
    }
    {
        // the diagonal table of the sweep's tickets (one source)
        const int NJ = gm.NJ, NK = gm.NK, ngrp = p->D / wpb;
        int *ds = p->dstart_host.data();
        ds[0] = 0;
        for (int dd = 0; dd <= NJ + NK - 2; ++dd) {
            const int lo = std::max(0, dd - (NK - 1)), hi = std::min(dd, NJ - 1);
            ds[dd + 1] = ds[dd] + (hi - lo + 1) * 8 * ngrp;
        }
        ds[NJ + NK] = ds[NJ + NK - 1];
    }
    DSN_HIP(hipMemcpyAsync(mat_nat, p->material.data(), (size_t)gm.V, hipMemcpyHostToDevice, s));
    if (dens_nat)
        DSN_HIP(hipMemcpyAsync(dens_nat, p->density.data(), (size_t)gm.V * sizeof(double), hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.xs_t, p->sigma_t.data(), z.xs_t, hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.xs_s, p->sigma_s.data(), z.xs_s, hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.M0, fp64 ? (const void *)p->M0.data() : (const void *)p->M0f.data(), z.M0,
                           hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.D0, p->D0.data(), z.D0, hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.cdir, fp64 ? (const void *)p->cdir.data() : (const void *)p->cdirf.data(), z.cdir,
                           hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.sweep_dstart, p->dstart_host.data(), p->dstart_host.size() * sizeof(int),
                           hipMemcpyHostToDevice, s));
    std::memcpy(p->spec_host.data(), src.spectrum, z.spec);
    DSN_HIP(hipMemcpyAsync((void *)a.src_par, par, kSrcPar * sizeof(double), hipMemcpyHostToDevice, s));
    DSN_HIP(hipMemcpyAsync((void *)a.src_spec, p->spec_host.data(), z.spec, hipMemcpyHostToDevice, s));
    // state the last call on this GPU left behind: tickets, abort flag and
    // epoch start at zero, the face parity at zero, every face word at the
    // all-ones value no sweep accepts
    fill_u32(a.sweep_ctr, kCtrInts * sizeof(int), 0u, s);
    fill_u32(a.face_par, sizeof(int), 0u, s);
    fill_u32(a.faceY, z.face, 0xFFFFFFFFu, s);
    fill_u32(a.faceZ, z.face, 0xFFFFFFFFu, s);
    launch_voxels_to_pencils(gm, mat_nat, dens_nat, (uint8_t *)a.mat, (double *)a.dens, s);
    launch_raytrace<T>(a, s);
    DSN_HIP(hipGetLastError());
    Ctl &hc = p->ctl_host[0];  // the group's control block, read back between chunks
    for (int g = 0; g < G; ++g) {
        launch_group_source<T>(a, g, true, s);  // also forms the first directional source
        const int target = o.fixed_iters ? o.fixed_iters[g] : -1;
        launch_ctl_init(a.ctl, G, 1, g, target, o.max_iters, o.fixed_iters ? 0.0 : o.tol, o.stagnation_stop,
                        o.stop_rule, s);
        if (target >= 0) {
            for (int it = 0; it < target; ++it) {
                launch_sweeps<T>(a, g, s);
                launch_d2m<T>(a, g, true, s);
            }
        } else {
            // iterations in chunks between host reads of the group's control
            // block (an iteration enqueued after convergence returns at once)
            int enq = 0, chunk = 4;
            for (;;) {
                for (int k = 0; k < chunk; ++k) {
                    launch_sweeps<T>(a, g, s);
                    launch_d2m<T>(a, g, true, s);
                }
                enq += chunk;
                DSN_HIP(hipGetLastError());
                DSN_HIP(hipMemcpyAsync(&hc, a.ctl + g, sizeof(Ctl), hipMemcpyDeviceToHost, s));
                DSN_HIP(hipStreamSynchronize(s));
                if (hc.done || enq >= o.max_iters) break;
                chunk = 2;
            }
        }
        launch_finalize<T>(a, g, phi_total, phi_unc, s);
    }
    DSN_HIP(hipGetLastError());
    int *flags = p->flags_host;
    DSN_HIP(hipMemcpyAsync(p->ctl_host.data(), a.ctl, (size_t)G * sizeof(Ctl), hipMemcpyDeviceToHost, s));
    DSN_HIP(hipMemcpyAsync(flags, a.sweep_ctr, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    DSN_HIP(hipStreamSynchronize(s));
    if (flags[1]) return fail(DSN_ERR_DEVICE, "sweep dependency wait timed out (results invalid)");
    double updates = 0.0;
    for (int g = 0; g < G; ++g) {
        const Ctl &cg = p->ctl_host[g];
        if (info && info->iters) info->iters[g] = cg.iters;
        if (info && info->residual) info->residual[g] = cg.r;
        updates += (double)cg.iters * (double)gm.V * (double)p->Nd;
    }
    if (info) {
        info->updates = updates;
        info->sweep_bytes = updates * 2.0 * sizeof(T);
        info->sweep_waves_per_block = wpb;
        info->sweep_blocks = std::min(grid, a.sweep_nitems);
        info->sweep_xcd_queues = 0;
        info->sweep_relay = relay;
    }
    return status_of(p->ctl_host.data(), G);
}

}  // namespace

extern "C" {

const char *dsn_last_error(void) { return g_err.c_str(); }

int32_t dsn_sweep_tuning(const dsn_problem *p, int32_t *waves_per_block, int32_t *blocks, int32_t *xcd_queues,
                         int32_t *relay, float *ms, int32_t cap)
{
    if (!p) return 0;
    const DeviceState &d = p->dev;
    for (int i = 0; i < d.tune_n && i < cap; ++i) {
        if (waves_per_block) waves_per_block[i] = d.tune_log[i].wpb;
        if (blocks) blocks[i] = d.tune_log[i].blocks;
        if (xcd_queues) xcd_queues[i] = d.tune_log[i].xcd;
        if (relay) relay[i] = d.tune_log[i].relay;
        if (ms) ms[i] = d.tune_log[i].ms;
    }
    return d.tune_n;
}

dsn_status dsn_set_sweep_shape(dsn_problem *p, int32_t waves_per_block, int32_t blocks, int32_t xcd_queues,
                               int32_t relay)
{
    try {
        if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        const bool fp64 = p->precision == DSN_FP64;
        const int w = waves_per_block;
        int wl[kMaxWpb];
        const int nw = sweep_wpb_choices(fp64, wl);
        bool built = false;
        for (int i = 0; i < nw; ++i) built = built || wl[i] == w;
        if (!built || w > kMaxWpb || p->D % w != 0)
            return fail(DSN_ERR_INVALID_ARG, "waves_per_block must be a built choice that divides the directions "
                                             "of an octant");
        if (blocks < 1 || blocks > 1 << 20) return fail(DSN_ERR_INVALID_ARG, "blocks must be in 1..2^20");
        if (xcd_queues < 0) return fail(DSN_ERR_INVALID_ARG, "xcd_queues must be >= 0");
        if (relay < 0) return fail(DSN_ERR_INVALID_ARG, "relay must be >= 0");
        if (relay > 0 && xcd_queues > 0)
            return fail(DSN_ERR_INVALID_ARG, "column-relay sweeps use the global ticket queue (xcd_queues 0)");
        if (relay > 0) {
            int cw[kMaxCol], cr[kMaxCol];
            const int nc = sweep_col_choices(fp64, cw, cr);
            bool col_built = false;
            for (int i = 0; i < nc; ++i) col_built = col_built || (cw[i] == w && cr[i] == relay);
            if (!col_built)
                return fail(DSN_ERR_INVALID_ARG, "(waves_per_block, relay) is not a built column-relay shape");
        }
        dsn_status st = ensure_device(p);
        if (st != DSN_OK) return st;
        DeviceState &d = p->dev;
        if (d.grid_of[w] < 1) return fail(DSN_ERR_UNSUPPORTED, "no sweep kernel of that shape fits the device");
        if (relay > 0 && col_grid_of(d, w, relay) < 1)
            return fail(DSN_ERR_UNSUPPORTED, "the column-relay sweep's LDS does not fit for this x extent");
        if (xcd_queues != 0) {
            if (xcd_queues != d.xcd_nq || !sweep_xcd_supported(fp64, p->fixup, w))
                return fail(DSN_ERR_UNSUPPORTED, "per-XCD queues: FP32 with the fixup, waves_per_block <= 4, and "
                                                 "xcd_queues equal to the device's XCD count");
        }
        d.wpb = w;
        d.sweep_grid = blocks;
        d.xcd_use = xcd_queues;
        d.relay = relay;
        d.sweep_nitems = sweep_items(p, w, relay);
        d.dstart_S = 0;  // the diagonal table is rebuilt for the new shape at the next solve
        d.tuned = true;
        return DSN_OK;
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

int32_t dsn_xcd_queues(dsn_problem *p)
{
    try {
        if (!p) {
            (void)fail(DSN_ERR_INVALID_ARG, "problem is NULL");
            return -1;
        }
        if (ensure_device(p) != DSN_OK) return -1;
        return p->dev.xcd_nq;
    } catch (...) {
        (void)fail(DSN_ERR_DEVICE, "unexpected exception");
        return -1;
    }
}

dsn_status dsn_quadrature(int32_t sn_order, double *omega, double *w)
{
    if (!omega || !w) return fail(DSN_ERR_INVALID_ARG, "omega and w must not be NULL");
    std::vector<double> om, ww;
    std::string err;
    if (!lqn_build(sn_order, om, ww, err)) return fail(DSN_ERR_INVALID_ARG, err);
    std::memcpy(omega, om.data(), om.size() * sizeof(double));
    std::memcpy(w, ww.data(), ww.size() * sizeof(double));
    return DSN_OK;
}

dsn_status dsn_create(const dsn_problem_desc *d, dsn_problem **out)
{
    try {
        if (!d || !out) return fail(DSN_ERR_INVALID_ARG, "desc and out must not be NULL");
        *out = nullptr;
        if (d->nx < 1 || d->ny < 1 || d->nz < 1) return fail(DSN_ERR_INVALID_ARG, "mesh sizes must be >= 1");
        if (!(d->dx > 0) || !(d->dy > 0) || !(d->dz > 0) || !std::isfinite(d->dx) || !std::isfinite(d->dy) ||
            !std::isfinite(d->dz))
            return fail(DSN_ERR_INVALID_ARG, "voxel pitch must be finite and > 0");
        if (d->n_materials < 1 || d->n_materials > kMaxMat)
            return fail(d->n_materials < 1 ? DSN_ERR_INVALID_ARG : DSN_ERR_UNSUPPORTED,
                        "n_materials must be in 1..16");
        if (d->n_groups < 1) return fail(DSN_ERR_INVALID_ARG, "n_groups must be >= 1");
        if (!lqn_supported(d->sn_order)) return fail(DSN_ERR_INVALID_ARG, "sn_order must be one of 2,4,6,8,10,12,16");
        if (d->legendre_order < 0 || d->legendre_order > d->sn_order - 1)
            return fail(DSN_ERR_INVALID_ARG, "legendre_order must be in 0..N-1");
        if (d->legendre_order > kMaxL) return fail(DSN_ERR_UNSUPPORTED, "legendre_order above 5 is not built");
        if (d->fixup != 0 && d->fixup != 1) return fail(DSN_ERR_INVALID_ARG, "fixup must be 0 or 1");
        if (d->precision != DSN_FP64 && d->precision != DSN_FP32)
            return fail(DSN_ERR_INVALID_ARG, "precision must be DSN_FP64 or DSN_FP32");
        if (!d->material || !d->sigma_t || !d->sigma_s)
            return fail(DSN_ERR_INVALID_ARG, "material, sigma_t and sigma_s must not be NULL");
        const long V = (long)d->nx * d->ny * d->nz;
        const int G = d->n_groups, L = d->legendre_order, M = d->n_materials;
        for (long v = 0; v < V; ++v)
            if (d->material[v] >= M) return fail(DSN_ERR_INVALID_ARG, "material id >= n_materials");
        if (d->density)
            for (long v = 0; v < V; ++v)
                if (!std::isfinite(d->density[v]) || d->density[v] < 0)
                    return fail(DSN_ERR_INVALID_ARG, "density must be finite and >= 0");
        if (!finite_all(d->sigma_t, (size_t)M * G)) return fail(DSN_ERR_INVALID_ARG, "sigma_t not finite");
        for (long i = 0; i < (long)M * G; ++i)
            if (d->sigma_t[i] < 0) return fail(DSN_ERR_INVALID_ARG, "sigma_t must be >= 0");
        const size_t nss = (size_t)M * (L + 1) * G * G;
        if (!finite_all(d->sigma_s, nss)) return fail(DSN_ERR_INVALID_ARG, "sigma_s not finite");
        for (int m = 0; m < M; ++m)
            for (int l = 0; l <= L; ++l)
                for (int g = 0; g < G; ++g)
                    for (int gp = 0; gp < G; ++gp) {
                        const double x = d->sigma_s[(((size_t)m * (L + 1) + l) * G + g) * G + gp];
                        if (gp > g && x != 0.0) return fail(DSN_ERR_INVALID_ARG, "upscatter (g' > g) is not allowed");
                        if (l == 0 && x < 0) return fail(DSN_ERR_INVALID_ARG, "sigma_s,0 must be >= 0");
                    }
        dsn_problem *p = new dsn_problem();
        Geom &gm = p->geom;
        gm.nx = d->nx; gm.ny = d->ny; gm.nz = d->nz;
        gm.NJ = (d->ny + kCB - 1) / kCB;
        gm.NK = (d->nz + kCB - 1) / kCB;
        gm.Vp = (long)gm.NJ * gm.NK * gm.nx * kLanes;
        gm.V = V;
        gm.dx = d->dx; gm.dy = d->dy; gm.dz = d->dz;
        p->nmat = M; p->G = G; p->L = L; p->Nm = (L + 1) * (L + 1); p->N = d->sn_order;
        p->Nd = d->sn_order * (d->sn_order + 2); p->D = p->Nd / 8;
        p->fixup = d->fixup; p->precision = d->precision;
        p->has_density = d->density != nullptr;
        p->material.assign(d->material, d->material + V);
        if (d->density) p->density.assign(d->density, d->density + V);
        p->sigma_t.assign(d->sigma_t, d->sigma_t + (size_t)M * G);
        p->sigma_s.assign(d->sigma_s, d->sigma_s + nss);
        std::string err;
        if (!lqn_build(p->N, p->omega, p->w, err)) { delete p; return fail(DSN_ERR_INVALID_ARG, err); }
        // moment tables of octant 0 and the parity check that lets the
        // kernels reconstruct the other seven octants by sign flips
        const int D = p->D, Nm = p->Nm;
        p->M0.assign((size_t)D * Nm, 0.0);
        p->D0.assign((size_t)D * Nm, 0.0);
        std::vector<double> R(Nm), R0(Nm);
        for (int pp = 0; pp < D; ++pp) {
            host_harmonics(L, p->omega[3 * pp], p->omega[3 * pp + 1], p->omega[3 * pp + 2], R0.data());
            for (int lm = 0; lm < Nm; ++lm) {
                int l = 0;
                while ((l + 1) * (l + 1) <= lm) ++l;
                p->M0[(size_t)pp * Nm + lm] = (2.0 * l + 1.0) / (4.0 * M_PI) * R0[lm];
                p->D0[(size_t)pp * Nm + lm] = p->w[pp] * R0[lm];
            }
            for (int o = 1; o < 8; ++o) {
                const int n = o * D + pp;
                host_harmonics(L, p->omega[3 * n], p->omega[3 * n + 1], p->omega[3 * n + 2], R.data());
                for (int lm = 0; lm < Nm; ++lm) {
                    const double chi = (__builtin_popcount(host_lm_class(lm) & o) & 1) ? -1.0 : 1.0;
                    if (std::fabs(R[lm] - chi * R0[lm]) > 1e-12 * (1.0 + std::fabs(R0[lm]))) {
                        delete p;
                        return fail(DSN_ERR_UNSUPPORTED, "quadrature lacks octant reflection symmetry");
                    }
                }
            }
        }
        p->cdir.assign((size_t)p->Nd * 3, 0.0);
        const double h[3] = {d->dx, d->dy, d->dz};
        for (int n = 0; n < p->Nd; ++n)
            for (int t = 0; t < 3; ++t) p->cdir[3 * n + t] = 2.0 * std::fabs(p->omega[3 * n + t]) / h[t];
        p->M0f.assign(p->M0.begin(), p->M0.end());
        p->cdirf.assign(p->cdir.begin(), p->cdir.end());
        p->dstart_host.assign((size_t)gm.NJ + gm.NK + 1, 0);
        p->ctl_host.assign((size_t)G, Ctl());
        p->spec_host.assign((size_t)G, 0.0);
        *out = p;
        return DSN_OK;
    } catch (const std::bad_alloc &) {
        return fail(DSN_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(DSN_ERR_INVALID_ARG, "unexpected host exception");
    }
}

void dsn_destroy(dsn_problem *p)
{
    if (!p) return;
    {
        DeviceWide gate;
        if (p->dev.device >= 0) (void)hipDeviceSynchronize();
    }
    dev_release(p->dev);
    delete p;
}

size_t dsn_workspace_bytes(const dsn_problem *p)
{
    if (!p) return 0;
    if (p->dev.ready) return p->dev.bytes;
    return sizes_of(p).total();
}

dsn_status dsn_solve(dsn_problem *p, const dsn_source *src, int32_t n_src, const dsn_solve_opts *opts,
                     double *phi_total, double *phi_uncollided, dsn_solve_info *info)
{
    try {
        const auto t0 = std::chrono::steady_clock::now();
        if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        if (n_src < 0 || (n_src > 0 && !src)) return fail(DSN_ERR_INVALID_ARG, "bad source list");
        if (!phi_total && n_src > 0) return fail(DSN_ERR_INVALID_ARG, "phi_total is NULL");
        dsn_status st = check_opts(p, opts);
        if (st != DSN_OK) return st;
        if (opts->combine_sources && n_src == 0)
            return fail(DSN_ERR_INVALID_ARG, "combine_sources needs at least one source");
        for (int i = 0; i < n_src; ++i)
            if ((st = check_source(p, src[i])) != DSN_OK) return st;
        if (info) {
            info->updates = 0;
            info->seconds = 0;
            info->sweep_bytes = 0;
            info->sweep_waves_per_block = 0;
            info->sweep_blocks = 0;
            info->sweep_xcd_queues = 0;
            for (int k = 0; k < DSN_NUM_STAGES; ++k) { info->stage_ms[k] = 0; info->stage_launches[k] = 0; }
        }
        if (n_src == 0) return DSN_OK;
        if ((st = ensure_device(p)) != DSN_OK) return st;
        hipStream_t s = (hipStream_t)opts->stream;
        StageTimer &tm = p->dev.timer;
        tm.on = opts->profile != 0;
        tm.s = s;
        tm.used = 0;
        tm.stage_of.clear();
        for (int k = 0; k < DSN_NUM_STAGES; ++k) { tm.ms[k] = 0; tm.launches[k] = 0; }
        if (p->precision == DSN_FP32)
            st = solve_sources<float>(p, src, n_src, *opts, phi_total, phi_uncollided, info, s);
        else
            st = solve_sources<double>(p, src, n_src, *opts, phi_total, phi_uncollided, info, s);
        if (tm.on) {
            (void)hipStreamSynchronize(s);
            tm.flush();
            tm.on = false;
        }
        if (info) {
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            for (int k = 0; k < DSN_NUM_STAGES; ++k) {
                info->stage_ms[k] = tm.ms[k];
                info->stage_launches[k] = tm.launches[k];
            }
            info->sweep_waves_per_block = p->dev.wpb;
            info->sweep_blocks = p->dev.sweep_grid;
            info->sweep_xcd_queues = p->dev.xcd_use;
            info->sweep_relay = p->dev.relay;
        }
        return st;
    } catch (const std::bad_alloc &) {
        return fail(DSN_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

dsn_status dsn_solve_noalloc(dsn_problem *p, const dsn_source *src, const dsn_solve_opts *opts, double *phi_total,
                             double *phi_uncollided, dsn_solve_info *info)
{
    try {
        const auto t0 = std::chrono::steady_clock::now();
        if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        if (!src) return fail(DSN_ERR_INVALID_ARG, "source is NULL");
        if (!phi_total) return fail(DSN_ERR_INVALID_ARG, "phi_total is NULL");
        dsn_status st = check_opts(p, opts);
        if (st != DSN_OK) return st;
        if (opts->combine_sources) return fail(DSN_ERR_INVALID_ARG, "dsn_solve_noalloc solves one source");
        if ((st = check_source(p, *src)) != DSN_OK) return st;
        if (info) {
            info->updates = 0;
            info->seconds = 0;
            info->sweep_bytes = 0;
            for (int k = 0; k < DSN_NUM_STAGES; ++k) { info->stage_ms[k] = 0; info->stage_launches[k] = 0; }
        }
        hipStream_t s = (hipStream_t)opts->stream;
        st = p->precision == DSN_FP32 ? solve_noalloc<float>(p, *src, *opts, phi_total, phi_uncollided, info, s)
                                      : solve_noalloc<double>(p, *src, *opts, phi_total, phi_uncollided, info, s);
        if (info)
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return st;
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

dsn_status dsn_solve_adjoint(dsn_problem *p, const dsn_source *src, const double *W, const dsn_solve_opts *opts,
                             double *J, double *dJ_ddensity, double *phi_total, dsn_solve_info *info)
{
    try {
        const auto t0 = std::chrono::steady_clock::now();
        if (!p || !src || !W || !J || !dJ_ddensity)
            return fail(DSN_ERR_INVALID_ARG, "problem, src, W, J and dJ_ddensity must not be NULL");
        dsn_status st = check_opts(p, opts);
        if (st != DSN_OK) return st;
        if ((st = check_source(p, *src)) != DSN_OK) return st;
        if ((st = ensure_device(p)) != DSN_OK) return st;
        if ((st = ensure_adjoint(p)) != DSN_OK) return st;
        hipStream_t s = (hipStream_t)opts->stream;
        p->dev.timer.on = false;
        if (info) {
            info->updates = 0;
            info->sweep_bytes = 0;
            info->sweep_waves_per_block = 0;
            info->sweep_blocks = 0;
            info->sweep_xcd_queues = 0;
            for (int k = 0; k < DSN_NUM_STAGES; ++k) { info->stage_ms[k] = 0; info->stage_launches[k] = 0; }
        }
        dsn_solve_opts oa = *opts;
        oa.combine_sources = 0;  // one source: nothing to combine
        st = p->precision == DSN_FP32 ? adjoint_impl<float>(p, *src, W, oa, J, dJ_ddensity, phi_total, info, s)
                                      : adjoint_impl<double>(p, *src, W, oa, J, dJ_ddensity, phi_total, info, s);
        if (info) {
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            info->sweep_waves_per_block = p->dev.wpb;
            info->sweep_blocks = p->dev.sweep_grid;
            info->sweep_xcd_queues = p->dev.xcd_use;
            info->sweep_relay = p->dev.relay;
        }
        return st;
    } catch (const std::bad_alloc &) {
        return fail(DSN_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

dsn_status dsn_dose(dsn_problem *p, const double *phi, int32_t n, const double *k, double *dose, void *stream)
{
    try {
        if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        if (n < 0) return fail(DSN_ERR_INVALID_ARG, "n must be >= 0");
        if (n == 0) return DSN_OK;
        if (!phi || !k || !dose) return fail(DSN_ERR_INVALID_ARG, "phi, k and dose must be given");
        if (n > 65535) return fail(DSN_ERR_INVALID_ARG, "at most 65535 fluence sets per call");
        const size_t nk = (size_t)p->nmat * p->G;
        for (size_t i = 0; i < nk; ++i)
            if (!std::isfinite(k[i])) return fail(DSN_ERR_INVALID_ARG, "dose factors must be finite");
        dsn_status st = ensure_device(p);
        if (st != DSN_OK) return st;
        DeviceState &d = p->dev;
        if (!d.kdose && (st = dev_alloc(d, (void **)&d.kdose, nk * sizeof(double))) != DSN_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        DSN_HIP(hipMemcpyAsync(d.kdose, k, nk * sizeof(double), hipMemcpyHostToDevice, s));
        launch_dose(d.mat_nat, (long)p->geom.V, p->G, phi, d.kdose, n, dose, s);
        DSN_HIP(hipGetLastError());
        DSN_HIP(hipStreamSynchronize(s));  // the factor table is the caller's host memory
        return DSN_OK;
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

dsn_status dsn_set_density(dsn_problem *p, const double *density)
{
    try {
        if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        dsn_status st = ensure_device(p);
        if (st != DSN_OK) return st;
        DeviceState &d = p->dev;
        const size_t bytes = (size_t)p->geom.V * sizeof(double);
        if (!d.dens_nat) {
            if ((st = dev_alloc(d, (void **)&d.dens_nat, bytes)) != DSN_OK) return st;
        }
        if (density) {
            DSN_HIP(hipMemcpy(d.dens_nat, density, bytes, hipMemcpyDefault));
        } else {
            std::vector<double> ones(p->geom.V, 1.0);
            DSN_HIP(hipMemcpy(d.dens_nat, ones.data(), bytes, hipMemcpyHostToDevice));
        }
        p->has_density = true;
        launch_voxels_to_pencils(p->geom, d.mat_nat, d.dens_nat, d.mat, d.dens, 0);
        DSN_HIP(hipGetLastError());
        DeviceWide gate;
        DSN_HIP(hipDeviceSynchronize());
        return DSN_OK;
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

dsn_status dsn_solve_batch(dsn_problem *const *probs, int32_t n_probs, const dsn_source *const *srcs,
                           const int32_t *n_src, const dsn_solve_opts *opts, double *const *phi_total,
                           dsn_solve_info *info)
{
    try {
        const auto t0 = std::chrono::steady_clock::now();
        if (!probs || n_probs < 1 || !srcs || !n_src || !phi_total)
            return fail(DSN_ERR_INVALID_ARG, "probs, srcs, n_src and phi_total must be given, n_probs >= 1");
        if (opts && opts->combine_sources)
            return fail(DSN_ERR_INVALID_ARG, "combine_sources is not supported by dsn_solve_batch");
        const dsn_problem *p0 = probs[0];
        if (!p0) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
        for (int b = 0; b < n_probs; ++b) {
            const dsn_problem *p = probs[b];
            if (!p) return fail(DSN_ERR_INVALID_ARG, "problem is NULL");
            if (p->G != p0->G || p->N != p0->N || p->L != p0->L || p->precision != p0->precision)
                return fail(DSN_ERR_INVALID_ARG, "batched problems must share G, S_N order, P_L order and precision");
            if (n_src[b] < 0 || (n_src[b] > 0 && (!srcs[b] || !phi_total[b])))
                return fail(DSN_ERR_INVALID_ARG, "bad source list or output of a batched problem");
            for (int c = 0; c < b; ++c)
                if (probs[c] == p) return fail(DSN_ERR_INVALID_ARG, "a problem appears twice in a batch");
            dsn_status st = check_opts(p, opts);
            if (st != DSN_OK) return st;
            for (int i = 0; i < n_src[b]; ++i)
                if ((st = check_source(p, srcs[b][i])) != DSN_OK) return st;
        }
        if (info) {
            info->updates = 0;
            info->sweep_bytes = 0;
            info->sweep_waves_per_block = 0;
            info->sweep_blocks = 0;
            info->sweep_xcd_queues = 0;
            info->sweep_relay = 0;
            for (int k = 0; k < DSN_NUM_STAGES; ++k) { info->stage_ms[k] = 0; info->stage_launches[k] = 0; }
        }
        // fused: one sweep launch per iteration over every (problem, source) pair
        if (opts->batch_mode == 1) {
            const std::string why = fused_obstacle(probs, n_probs, n_src);
            if (!why.empty()) return fail(DSN_ERR_UNSUPPORTED, "fused batch: " + why);
            DeviceWide gate;
            hipStream_t sf = (hipStream_t)opts->stream;
            const dsn_status st = p0->precision == DSN_FP32
                                      ? solve_batch_fused<float>(probs, n_probs, srcs, n_src, *opts, phi_total, info, sf)
                                      : solve_batch_fused<double>(probs, n_probs, srcs, n_src, *opts, phi_total, info, sf);
            if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (st == DSN_ERR_NOT_CONVERGED) g_err = "max_iters reached before tol";
            return st;
        }
        // Every problem runs on a stream of its own (default priority), driven
        // by a host thread of its own, so that phantoms of different sizes
        // overlap on the GPU instead of queueing behind each other.  The
        // problems' streams start after the work already on the caller's
        // stream, and the caller's stream waits for all of them.
        hipStream_t s = (hipStream_t)opts->stream;
        int dev = 0;
        DSN_HIP(hipGetDevice(&dev));
        hipEvent_t start = nullptr;
        DSN_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
        DSN_HIP(hipEventRecord(start, s));
        struct Job {
            dsn_status st = DSN_OK;
            std::string err;
            std::vector<int32_t> it;
            dsn_solve_info ib{};
            hipEvent_t done = nullptr;
        };
        std::vector<int> per_batch;
        {
            const dsn_status st = joint_batch_limits(probs, n_probs, n_src, per_batch);
            if (st != DSN_OK) return st;
        }
        std::vector<Job> jobs(n_probs);
        std::vector<std::thread> workers;
        struct JoinAll {  // joins the started workers on every way out, exceptions included
            std::vector<std::thread> &w;
            ~JoinAll()
            {
                for (std::thread &t : w)
                    if (t.joinable()) t.join();
            }
        } join_all{workers};
        for (int b = 0; b < n_probs; ++b) {
            if (n_src[b] == 0) continue;
            workers.emplace_back([&, b]() {
                Job &j = jobs[b];
                dsn_problem *p = probs[b];
                auto run = [&]() -> dsn_status {
                    DSN_HIP(hipSetDevice(dev));
                    dsn_status st = ensure_device(p);
                    if (st != DSN_OK) return st;
                    DeviceState &d = p->dev;
                    if (!d.batch_stream) DSN_HIP(hipStreamCreateWithFlags(&d.batch_stream, hipStreamNonBlocking));
                    DSN_HIP(hipStreamWaitEvent(d.batch_stream, start, 0));
                    d.timer.on = false;
                    j.it.assign((size_t)n_src[b] * p->G, 0);
                    j.ib.iters = j.it.data();
                    j.ib.residual = nullptr;
                    dsn_solve_opts ob = *opts;
                    ob.autotune = 0;  // problems running together would time each other
                    st = p->precision == DSN_FP32
                             ? solve_sources<float>(p, srcs[b], n_src[b], ob, phi_total[b], nullptr, &j.ib,
                                                    d.batch_stream, per_batch[b])
                             : solve_sources<double>(p, srcs[b], n_src[b], ob, phi_total[b], nullptr, &j.ib,
                                                     d.batch_stream, per_batch[b]);
                    DSN_HIP(hipEventCreateWithFlags(&j.done, hipEventDisableTiming));
                    DSN_HIP(hipEventRecord(j.done, d.batch_stream));
                    return st;
                };
                try {
                    j.st = run();
                } catch (...) {
                    j.st = DSN_ERR_DEVICE;
                    g_err = "unexpected exception in a batched problem";
                }
                j.err = g_err;
            });
        }
        for (std::thread &w : workers) w.join();
        dsn_status worst = DSN_OK;
        size_t row = 0;
        double updates = 0.0, sweep_bytes = 0.0;
        dsn_status hard = DSN_OK;
        std::string hard_err;
        for (int b = 0; b < n_probs; ++b) {
            Job &j = jobs[b];
            if (j.done) {
                (void)hipStreamWaitEvent(s, j.done, 0);
                (void)hipEventDestroy(j.done);
            }
            if (n_src[b] == 0) continue;
            if (j.st != DSN_OK && j.st != DSN_ERR_NOT_CONVERGED && hard == DSN_OK) {
                hard = j.st;
                hard_err = j.err;
            }
            if (j.st == DSN_ERR_NOT_CONVERGED) worst = j.st;
            if (info && info->iters && !j.it.empty())
                std::memcpy(info->iters + row * probs[b]->G, j.it.data(), j.it.size() * sizeof(int32_t));
            row += n_src[b];
            updates += j.ib.updates;
            sweep_bytes += j.ib.sweep_bytes;
        }
        (void)hipEventDestroy(start);
        if (hard != DSN_OK) return fail(hard, hard_err);
        if (info) {
            info->updates = updates;
            info->sweep_bytes = sweep_bytes;
            info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        if (worst != DSN_OK) g_err = "max_iters reached before tol";
        return worst;
    } catch (const std::bad_alloc &) {
        return fail(DSN_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(DSN_ERR_DEVICE, "unexpected exception");
    }
}

}  // extern "C"
