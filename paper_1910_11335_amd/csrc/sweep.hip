// The diamond-difference transport sweep (paper section II.B, eqs. 8-22)
// for gfx950 (CDNA4, wave64): the kernel, its launch shapes and launcher.
// See internal.h for the pencil voxel layout.
#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#include "internal.h"

namespace dsn {

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
// Memory: the skew makes one step touch 15 different 64-voxel rows, so Q/psi
// rows are staged through a per-wave LDS ring and every global access of
// Q/psi moves whole rows; the details are with k_sweep below.
// ---------------------------------------------------------------------------
// Cross-lane moves in the step phase.  There lane L stands for the
// octant-relative column (j_r, k_r) = (L & 7, L >> 3), so the upstream
// neighbours are always lanes L-1 (y) and L-8 (z) whatever the octant.  The y
// move is a whole-wave DPP shift; lanes with j_r = 0 (k_r = 0) take the face
// inflow instead, so the values shifted across column ends are never used.
__device__ __forceinline__ float lane_shr1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_shr1(double v)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(x & 0xffffffffLL), 0x138, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane_from(float v, int src_byte)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_byte, __float_as_int(v)));
}
__device__ __forceinline__ double lane_from(double v, int src_byte)
{
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src_byte, (int)(x & 0xffffffffLL));
    const int hi = __builtin_amdgcn_ds_bpermute(src_byte, (int)(x >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float fmin3(float a, float b, float c) { return fminf(fminf(a, b), c); }
__device__ __forceinline__ double fmin3(double a, double b, double c) { return fmin(fmin(a, b), c); }

// Cell modes of the sweep (the sweep_mode of the argument block):
//   kDD      pure diamond difference
//   kFixup   with the set-to-zero fixup
//   kRecord  with the fixup, and the set of fixed axes of every cell written
//            to mk (bit a: axis a fixed)
//   kTrans   the transpose of the fixup cell with the fixed set mk frozen,
//            for the adjoint sweep along -Omega: psi = (q + sum over free
//            axes of c_a in_a) / (sigma + sum over free axes of c_a), outflow
//            2 psi - in_a on a free axis and psi on a fixed one (reverse-mode
//            differentiation of the frozen cell, adjoint face values scaled
//            by 2 / c_a)
constexpr int kDD = 0, kFixup = 1, kRecord = 2, kTrans = 3;

template <typename T, int MODE>
__device__ __forceinline__ T dd_update(T q, T sg, T cx, T cy, T cz, T csum, T px, T iny, T inz, T &ox_, T &oy_,
                                       T &oz_, unsigned &mk)
{
    if constexpr (MODE == kTrans) {
        const T kx = (mk & 1u) ? T(0) : T(1), ky = (mk & 2u) ? T(0) : T(1), kz = (mk & 4u) ? T(0) : T(1);
        const T p = dd_div<T>(q + kx * cx * px + ky * cy * iny + kz * cz * inz, sg + kx * cx + ky * cy + kz * cz);
        ox_ = (mk & 1u) ? p : T(2) * p - px;
        oy_ = (mk & 2u) ? p : T(2) * p - iny;
        oz_ = (mk & 4u) ? p : T(2) * p - inz;
        return p;
    }
    const T num0 = q + cx * px + cy * iny + cz * inz, den0 = sg + csum;
    T p = dd_div<T>(num0, den0);
    ox_ = T(2) * p - px;
    oy_ = T(2) * p - iny;
    oz_ = T(2) * p - inz;
    if constexpr (MODE == kFixup || MODE == kRecord) {
        // Set-to-zero fixup.  An axis whose outflow is negative is fixed
        // (m_a = 1): its outflow becomes zero, its inflow enters the balance
        // with half weight and its coefficient leaves the denominator; the
        // cell is re-solved, and axes that turn negative are fixed in the
        // next pass (at most three).  A pass in which no axis of a lane turns
        // negative reproduces that lane's values exactly, so the passes run
        // branch-free over the whole wave while any lane still needs one.
        T lo = fmin3(ox_, oy_, oz_);
        if (__any(lo < T(0))) {
            T mx = T(0), my = T(0), mz = T(0);
            const T hx = T(0.5) * cx * px, hy = T(0.5) * cy * iny, hz = T(0.5) * cz * inz;
#pragma unroll
            for (int pass = 0; pass < 3; ++pass) {
                mx = ox_ < T(0) ? T(1) : mx;
                my = oy_ < T(0) ? T(1) : my;
                mz = oz_ < T(0) ? T(1) : mz;
                const T num = num0 - (mx * hx + my * hy + mz * hz);
                const T den = den0 - (mx * cx + my * cy + mz * cz);
                p = dd_div<T>(num, den);
                ox_ = mx != T(0) ? T(0) : T(2) * p - px;
                oy_ = my != T(0) ? T(0) : T(2) * p - iny;
                oz_ = mz != T(0) ? T(0) : T(2) * p - inz;
                if (pass == 2) break;
                lo = fmin3(ox_, oy_, oz_);
                if (!__any(lo < T(0))) break;
            }
            if constexpr (MODE == kRecord)
                mk = (mx != T(0) ? 1u : 0u) | (my != T(0) ? 2u : 0u) | (mz != T(0) ? 4u : 0u);
        }
    }
    return p;
}

// Device-coherent (agent scope) loads and stores: they bypass the per-XCD
// L2, so a block on any XCD sees them.
template <typename T>
__device__ __forceinline__ T coherent_load(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coherent_store(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Buffer resources for the sweep's memory traffic.  Every load and store of
// the chunk loop is issued unconditionally: a row outside the pencil gets an
// offset beyond its buffer's size (a row before the first wraps to an
// unsigned offset of 2^31 or more; every buffer is below 2 GiB), so the
// hardware range check turns its load into zero and drops its store.  With
// no branches around memory instructions the compiler waits only for the
// loads it needs, never for the completion of earlier stores.
typedef __amdgpu_buffer_rsrc_t Rsrc;
typedef __attribute__((ext_vector_type(2))) unsigned U32x2;
constexpr int kDstLds = 256;            // diagonal-start table entries kept in LDS
constexpr int kSigTab = 32;             // per-block sigma table: materials < kMaxMat, the ghost byte 255 -> 31
static_assert(kMaxMat <= 16, "the ghost byte must land on a zero entry of the sigma table");
constexpr int kTicketStop = 1 << 30;     // ticket counter after an abort (above any item count)
constexpr int kRawDword3 = 0x00020000;   // raw (untyped) 32-bit buffer access
constexpr int kSC1 = 16;                 // device-coherent: bypasses the per-XCD L2
constexpr int kVolatileSC1 = (int)0x80000010u;
constexpr int kSC0 = 1;                  // bypasses the CU's L1, coherent in the XCD's L2
constexpr int kVolatileSC0 = (int)0x80000001u;
constexpr int kNT = 2;                   // non-temporal: streamed data, not kept in the caches
constexpr int kQueueCtr = 4;             // first per-XCD ticket counter in the counter block

__device__ __forceinline__ Rsrc make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, kRawDword3);
}
template <int AUX = 0>
__device__ __forceinline__ float buf_load(Rsrc r, unsigned off, float)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX = 0>
__device__ __forceinline__ double buf_load(Rsrc r, unsigned off, double)
{
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
    return __longlong_as_double((long long)(((unsigned long long)v[1] << 32) | v[0]));
}
template <int AUX = 0>
__device__ __forceinline__ void buf_store(Rsrc r, unsigned off, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, off, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void buf_store(Rsrc r, unsigned off, double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    __builtin_amdgcn_raw_buffer_store_b64(U32x2{(unsigned)b, (unsigned)(b >> 32)}, r, off, 0, AUX);
}

// Face words.  An upstream block publishes face values that a downstream
// block polls; each word carries a stamp of the sweep that wrote it, in the
// same naturally aligned word as the data (single-copy atomic), so a reader
// that sees the current stamp has that word's data: no separate flag and no
// wait for store completion.  Stores and polls are device-coherent, except
// in the per-XCD-queue sweeps, where producer and consumer share one XCD and
// its L2 (plain stores, loads that bypass only the CU's L1).
//
// TaggedFace<T>: every 32-bit half of a value in one 64-bit word {half,
// epoch}; the epoch grows with every sweep launch.  Works for any value.
//
// SignFace<T>: for sweeps with the set-to-zero fixup, whose outflows are
// never negative, the value without its sign bit (one 32-bit word in FP32,
// one 64-bit word in FP64) and in the sign bit a per-source parity that
// flips after every sweep in which the source ran.
// A word left from that source's previous sweep has the other parity; words
// older than that never survive, because every sweep of a source rewrites all
// its face words.  All-ones (a NaN) is never accepted, which is how freshly
// allocated or invalidated faces read.
template <typename T>
struct TaggedFace {
    static constexpr int N = sizeof(T) / 4;  // 64-bit words per value
    static constexpr unsigned BYTES = 8 * N;
    typedef U32x2 Word[N];
    template <int AUX>
    static __device__ __forceinline__ void load(Word &w, Rsrc r, unsigned off)
    {
#pragma unroll
        for (int q = 0; q < N; ++q) w[q] = __builtin_amdgcn_raw_buffer_load_b64(r, off + 8 * q, 0, AUX);
    }
    static __device__ __forceinline__ bool ok(const Word &w, unsigned stamp)
    {
        bool good = true;
#pragma unroll
        for (int q = 0; q < N; ++q) good = good && w[q][1] == stamp;
        return good;
    }
    static __device__ __forceinline__ T value(const Word &w)
    {
        if constexpr (N == 1)
            return __uint_as_float(w[0][0]);
        else
            return __longlong_as_double((long long)(((unsigned long long)w[1][0] << 32) | w[0][0]));
    }
    template <int AUX>
    static __device__ __forceinline__ void put(Rsrc r, unsigned off, T v, unsigned stamp)
    {
        if constexpr (N == 1) {
            __builtin_amdgcn_raw_buffer_store_b64(U32x2{__float_as_uint(v), stamp}, r, off, 0, AUX);
        } else {
            const unsigned long long b = (unsigned long long)__double_as_longlong(v);
            __builtin_amdgcn_raw_buffer_store_b64(U32x2{(unsigned)b, stamp}, r, off, 0, AUX);
            __builtin_amdgcn_raw_buffer_store_b64(U32x2{(unsigned)(b >> 32), stamp}, r, off + 8, 0, AUX);
        }
    }
};
template <typename T>
struct SignFace;
template <>
struct SignFace<float> {
    static constexpr unsigned BYTES = 4;
    typedef unsigned Word;
    template <int AUX>
    static __device__ __forceinline__ void load(Word &w, Rsrc r, unsigned off)
    {
        w = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX);
    }
    static __device__ __forceinline__ bool ok(Word w, unsigned parity)
    {
        return (w >> 31) == parity && (w & 0x7FFFFFFFu) <= 0x7F800000u;
    }
    static __device__ __forceinline__ float value(Word w) { return __uint_as_float(w & 0x7FFFFFFFu); }
    template <int AUX>
    static __device__ __forceinline__ void put(Rsrc r, unsigned off, float v, unsigned parity)
    {
        __builtin_amdgcn_raw_buffer_store_b32((__float_as_uint(v) & 0x7FFFFFFFu) | (parity << 31), r, off, 0, AUX);
    }
};
template <>
struct SignFace<double> {
    static constexpr unsigned BYTES = 8;
    typedef U32x2 Word;  // {low half, high half with the parity in bit 31}
    template <int AUX>
    static __device__ __forceinline__ void load(Word &w, Rsrc r, unsigned off)
    {
        w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX);
    }
    static __device__ __forceinline__ bool ok(const Word &w, unsigned parity)
    {
        const unsigned hi = w[1] & 0x7FFFFFFFu;
        return (w[1] >> 31) == parity && (hi < 0x7FF00000u || (hi == 0x7FF00000u && w[0] == 0u));
    }
    static __device__ __forceinline__ double value(const Word &w)
    {
        return __longlong_as_double((long long)(((unsigned long long)(w[1] & 0x7FFFFFFFu) << 32) | w[0]));
    }
    template <int AUX>
    static __device__ __forceinline__ void put(Rsrc r, unsigned off, double v, unsigned parity)
    {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        const unsigned hi = ((unsigned)(b >> 32) & 0x7FFFFFFFu) | (parity << 31);
        __builtin_amdgcn_raw_buffer_store_b64(U32x2{(unsigned)b, hi}, r, off, 0, AUX);
    }
};
// Fixup sweeps (outflows never negative) carry the sign-parity words; pure DD
// and transposed sweeps the tagged ones, and so do the per-XCD-queue sweeps:
// their face words live in an XCD's L2, and only an epoch that is new with
// every launch makes a line left there by an earlier launch unacceptable.
template <typename T, int MODE, bool XCD>
struct FaceCodecSel {
    typedef typename std::conditional<!XCD && (MODE == kFixup || MODE == kRecord), SignFace<T>, TaggedFace<T>>::type
        type;
};

// Material bytes of octant-relative rows 8c .. 8c+7 of a pencil (64 bytes
// per row, one per column): physically 512 contiguous bytes, which lane l
// loads 8 at a time (physical row l / 8 of the block, columns 8 (l mod 8)
// .. 8 (l mod 8) + 7).  Rows outside the pencil lie outside the buffer and
// read as zero; a lane's 8 bytes never straddle two rows.
__device__ __forceinline__ U32x2 load_mat_rows(Rsrc r, int c, int sx, int nx, int lane)
{
    const int row0 = sx > 0 ? 8 * c : nx - 8 - 8 * c;  // physical row at the start of the block
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, (unsigned)(row0 * 64 + 8 * lane), 0, 0);
    return U32x2{v[0], v[1]};
}
// octant-relative row (within the chunk) of the bytes lane l loaded
__device__ __forceinline__ int mat_row(int sx, int lane) { return sx > 0 ? lane >> 3 : 7 - (lane >> 3); }

// sigma in the sweep.  SM = false: the group's sigma_t array (pencil order,
// type T).  SM = true (no per-voxel density, so sigma_t depends on the
// material only): one byte per voxel, the material, looked up in a per-block
// table of the group's cross sections (index 255, the ghost, maps to zero).
template <typename T, bool SM>
struct SigSrc;
template <typename T>
struct SigSrc<T, false> {
    typedef T Reg;
    static constexpr int ROW = 64 * sizeof(T);  // bytes per pencil row
    static __device__ __forceinline__ Reg load(Rsrc r, unsigned off) { return buf_load(r, off, T()); }
    static __device__ __forceinline__ T value(Reg x, const T *) { return x; }
};
template <typename T>
struct SigSrc<T, true> {
    typedef unsigned Reg;
    static constexpr int ROW = 64;
    static __device__ __forceinline__ Reg load(Rsrc r, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b8(r, off, 0, 0);
    }
    static __device__ __forceinline__ T value(Reg x, const T *table) { return table[x]; }
};

// Persistent, pipelined sweep of all directions.
//
// Work item = (octant o, group of WPB directions dg, pencil (J_r, K_r),
// source), one block; wave w of the block sweeps direction dg * WPB + w.
// Blocks take tickets from a global counter; tickets are numbered by pencil
// diagonal J_r + K_r first, so an item's upstream pencils (J_r - 1, K_r) and
// (J_r, K_r - 1) always hold smaller tickets, i.e. they were taken by blocks
// that are already running: no block waits on work that has not started, and
// every wait ends.
//
// Pipelining: outgoing face rows are published as soon as each 8-step chunk
// completes them; a downstream wave reads the face rows of its next chunk
// ahead of time and, when it commits them, re-reads any word whose stamp is
// not yet the current sweep's.  Downstream pencils therefore run a couple of
// chunks behind their upstream neighbours instead of waiting for whole
// pencils (KBA-style pipelining inside one GPU).  Every wait is bounded; on
// timeout the wave raises a global abort flag, the block leaves at its next
// ticket, and the host reports an error.
//
// Per wave and chunk c (steps t = 8c .. 8c+7; lane (j_r, k_r) updates row
// i_r = t - j_r - k_r at step t):
//   - psi (holding the source Q on entry) rows 8c .. 8c+7 are loaded a chunk
//     ahead as whole rows and committed to an LDS ring (row r in slot
//     r mod 24); steps read and overwrite them in place; rows 8c-16 .. 8c-9
//     are complete and go back to memory as whole rows;
//   - with sigma from the material (SM), the material bytes of rows 8c ..
//     8c+7 ride with the psi rows: whole rows, loaded a chunk ahead, into a
//     byte ring in LDS with the same slots; each step reads the byte of the
//     lane's own cell and looks sigma up in the block's table.  With
//     sigma in memory (per-voxel density), each lane reads sigma of its own
//     column for the next chunk's rows straight from memory, one load per
//     step right after that step has used the current value;
//   - face rows are stored skewed: a face value of row r needed (or made)
//     by a lane with skew s at step r + s sits in ring slot (r + s) mod 16,
//     so every step reads and writes one slot common to all lanes.
// Waves of a block share nothing but the ticket, so there is no barrier
// inside an item.  In FP32 the register budget is held to four waves per
// SIMD (16 per CU, e.g. four blocks of four directions) where the LDS allows
// that many.
//
// XCD (sweep_xcd = nq > 0): octant o is swept only by blocks running on XCD
// o mod nq, which take tickets from that XCD's own counter; all pencils of a
// direction then run on one XCD, so the face words between them need only
// be coherent in that XCD's L2 (plain stores, loads that bypass only the
// CU's L1).  Each block takes its queue from the XCD it runs on
// (hardware register XCC_ID), so a queue's blocks always share one L2.  The
// runtime enables it only after seeing consecutive workgroups go to
// consecutive XCDs (round robin; the first XCD depends on the hardware
// queue) and launches a whole number of blocks per XCD; a check after the
// launch reports any queue that no block served.
//
// NT: the psi rows are loaded and stored non-temporally (the runtime sets it
// when the launch's angular fluence exceeds the last-level cache, so that
// the streamed rows do not displace the face words and material bytes).
//
// MULTI: several problems (meshes) in one launch (k_sweep_multi): a0.multi
// holds their argument blocks and a0.seg the merged ticket order; an item's
// geometry, arrays and cross sections are its own problem's.
template <typename T, int MODE, int WPB, bool SM, bool XCD, bool NT, bool MULTI>
__device__ __forceinline__ void sweep_body(const SolveArgs<T> &a0, int g)
{
    constexpr int kLoadAux = XCD ? kSC0 : kSC1, kPollAux = XCD ? kVolatileSC0 : kVolatileSC1;
    constexpr int kStoreAux = XCD ? 0 : kSC1;
    constexpr int kPsiAux = NT ? kNT : 0;
    typedef SigSrc<T, SM> Sig;
    typedef typename FaceCodecSel<T, MODE, XCD>::type Face;
    constexpr bool kSignFace = std::is_same<Face, SignFace<T>>::value;
    constexpr int RQ = 24, RF = 16, CH = 8;
    constexpr int RB = 64 * sizeof(T);          // bytes per pencil row
    constexpr int FB = 8 * (int)Face::BYTES;    // bytes per face row
    __shared__ T sQ[WPB][RQ][64];
    __shared__ T sFYi[WPB][RF][8], sFZi[WPB][RF][8], sFYo[WPB][RF][8], sFZo[WPB][RF][8];
    __shared__ int sTicket;
    __shared__ int sDst[kDstLds];  // first ticket of every pencil diagonal, when it fits
    __shared__ T sSigT[SM ? kSigTab : 1];
    __shared__ __align__(16) unsigned char sMt[SM ? WPB : 1][SM ? RQ : 1][64];  // SM: material byte ring (slots as sQ)
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int D = a0.D, ngrp = D / WPB;
    constexpr bool multi = MULTI;
    // [0] next ticket (an abort lifts it to kTicketStop, so every later ticket
    // is past the end), [1] abort flag for the host, [2] epoch, [kQueueCtr +
    // q] next ticket of XCD q's queue
    int *const ctr = a0.sweep_ctr;
    const unsigned epoch = (unsigned)ctr[2];  // written by k_sweep_reset before this launch
    const int nq = XCD ? a0.sweep_xcd : 1;
    const int xq = XCD ? (int)__builtin_amdgcn_readfirstlane(__builtin_amdgcn_s_getreg((3 << 11) | 20)) % nq : 0;
    int *const tctr = XCD ? &ctr[kQueueCtr + xq] : &ctr[0];  // this block's ticket counter
    const int nitems = XCD ? a0.sweep_nitems / nq : a0.sweep_nitems;

    // An iteration enqueued after every source's group converged does
    // nothing: leave before touching the ticket queue.
    bool live = false;
    if constexpr (MULTI) {
        for (int q = 0; q < a0.nmulti; ++q) {
            const SolveArgs<T> &aq = a0.multi[q];
            for (int s = 0; s < aq.S; ++s) live = live || !aq.ctl[(long)s * aq.G + g].done;
        }
    } else {
        for (int s = 0; s < a0.S; ++s) live = live || !a0.ctl[(long)s * a0.G + g].done;
    }
    if (!live) return;
    int sig_of = -1;  // problem whose cross sections sSigT holds
    if (SM && !multi) {
        for (int i = threadIdx.x; i < kSigTab; i += 64 * WPB)
            sSigT[i] = i < a0.nmat ? (T)a0.xs_t[i * a0.G + g] : T(0);
        sig_of = 0;
    }
    // first ticket of every pencil diagonal (of every segment when multi)
    const int ndiag = multi ? a0.nseg : a0.g.NJ + a0.g.NK - 1;
    const int *const dstart = multi ? a0.seg : a0.sweep_dstart;
    const bool dst_lds = ndiag <= kDstLds;
    if (dst_lds)
        for (int i = threadIdx.x; i < ndiag; i += 64 * WPB) sDst[i] = dstart[i];
    // The next item's ticket is taken three chunks before an item ends, so
    // the atomic's latency hides behind those chunks while a ticket held in
    // advance (possibly the upstream of another block's item) waits at most
    // three chunks.  A block holds at most two tickets, the one it works on
    // and the next; the smallest unfinished ticket is therefore always being
    // worked on, and its upstream items (smaller tickets) are finished: the
    // queue always makes progress.
    int tnext = 0;
    bool have_next = false;  // thread 0 only
    for (;;) {
        if (threadIdx.x == 0) {
            sTicket = have_next ? tnext : atomicAdd(tctr, 1);
            have_next = false;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(sTicket);
        __syncthreads();
        if (t >= nitems) break;
        const int tq = t * nq;  // an XCD queue's diagonal starts are the global ones / nq
        // ticket -> (diagonal, position, direction group, octant, source); the
        // diagonal starts increase, so d = #{starts of diagonals 1.. <= t}
        int d = 0;
        if (dst_lds) {
            for (int base = 1; base < ndiag; base += 64) {
                const int i = base + lane;
                d += __popcll(__ballot(i < ndiag && sDst[i] <= tq));
            }
            d = __builtin_amdgcn_readfirstlane(d);
        } else {
            // the largest d with dstart[d] <= tq (starts strictly increase)
            int hi = ndiag - 1;
            while (d < hi) {
                const int mid = (d + hi + 1) >> 1;
                if (dstart[mid] <= tq) d = mid;
                else hi = mid - 1;
            }
        }
        int u = t - (dst_lds ? __builtin_amdgcn_readfirstlane(sDst[d]) : dstart[d]) / nq;
        // the item's problem and its pencil diagonal
        int pi = 0;
        if constexpr (MULTI) {
            const int code = a0.seg[ndiag + 1 + d];
            pi = code >> 16;
            d = code & 0xFFFF;
        }
        const SolveArgs<T> &A = MULTI ? a0.multi[pi] : a0;
        if (SM && pi != sig_of) {  // uniform over the block; no wave is inside an item
            for (int i = threadIdx.x; i < kSigTab; i += 64 * WPB)
                sSigT[i] = i < A.nmat ? (T)A.xs_t[i * A.G + g] : T(0);
            __syncthreads();
            sig_of = pi;
        }
        const int NJ = A.g.NJ, NK = A.g.NK, nx = A.g.nx;
        const long Vp = A.g.Vp;
        const int Jlo = d - (NK - 1) > 0 ? d - (NK - 1) : 0;
        const int Jhi = d < NJ - 1 ? d : NJ - 1;
        const int P = Jhi - Jlo + 1;
        const int qd = u % P;
        u /= P;
        const int dg = u % ngrp;
        u /= ngrp;
        int o, src;
        if constexpr (XCD) {
            const int opq = 8 / nq;  // octants per queue
            o = (u % opq) * nq + xq;
            src = u / opq;
        } else {
            o = u & 7;
            src = u >> 3;
        }
        const SolveArgs<T> a = at_source(A, src);
        if (a.ctl[g].done) continue;  // this source's group has converged
        const int n = o * D + dg * WPB + w;
        const unsigned stamp = kSignFace ? (unsigned)a.face_par[0] : epoch;
        // sweep geometry: the direction's octant, or the opposite one for the
        // adjoint (the transpose of the DD sweep along W is the sweep along -W)
        const int og = a.rev ? (o ^ 7) : o;
        const int sx = (og & 1) ? -1 : 1, sy = (og & 2) ? -1 : 1, sz = (og & 4) ? -1 : 1;
        const int Jr = Jlo + qd, Kr = d - Jr;
        const int J = sy > 0 ? Jr : NJ - 1 - Jr, K = sz > 0 ? Kr : NK - 1 - Kr;
        // step phase: lane = (j_r, k_r); its physical column (jp, kp)
        const int jr = lane & 7, kr = lane >> 3;
        const int jp = sy > 0 ? jr : 7 - jr, kp = sz > 0 ? kr : 7 - kr;
        const int pl = jp + 8 * kp;
        const int skew = jr + kr;
        const int srcZ = ((lane - 8) & 63) << 2;
        const bool yb = jr == 0, zb = kr == 0, yo = jr == 7, zo = kr == 7;
        const T cx = a.cdir[3 * n], cy = a.cdir[3 * n + 1], cz = a.cdir[3 * n + 2];
        const T csum = cx + cy + cz;
        const long pen = (long)K * NJ + J;
        const Rsrc rPsi = make_rsrc(a.psi + psi_run(pen, a.Nd, n, nx), (unsigned)(nx * RB));
        const Rsrc rSig = SM ? make_rsrc(a.mat + pen * nx * 64, (unsigned)(nx * 64))
                             : make_rsrc(a.sig + pen * nx * 64, (unsigned)(nx * RB));
        // fixed-axis sets, one byte per cell and direction ([Nd][Vp], pencil
        // order): written by kRecord sweeps, read by kTrans sweeps
        constexpr bool kMask = MODE == kRecord || MODE == kTrans;
        const Rsrc rMask = make_rsrc(kMask ? a.mask + (long)n * Vp + pen * nx * 64 : a.mat,
                                     kMask ? (unsigned)(nx * 64) : 0u);
        const int mbase = sx > 0 ? 0 : (nx - 1) * 64, mstep = sx * 64;
        // face words: [direction][pencil][row][8] of Face::BYTES each (the
        // buffers are sized for the widest codec)
        constexpr int FU = Face::BYTES / 4;  // 32-bit units per face value
        unsigned *const fY = (unsigned *)a.faceY, *const fZ = (unsigned *)a.faceZ;
        const long fdir = (long)n * NJ * NK * nx * 8 * FU;
        const long fown = fdir + pen * nx * 8 * FU;
        const bool hasY = Jr > 0, hasZ = Kr > 0;
        const unsigned fbytes = (unsigned)(nx * FB);
        // the last pencil along y (z) has no downstream neighbour there: its
        // outgoing y (z) words would never be read, so they are not stored
        const Rsrc rFYo = make_rsrc(fY + fown, Jr < NJ - 1 ? fbytes : 0u);
        const Rsrc rFZo = make_rsrc(fZ + fown, Kr < NK - 1 ? fbytes : 0u);
        const Rsrc rFYi = make_rsrc(fY + (hasY ? fdir + ((long)K * NJ + (J - sy)) * nx * 8 * FU : 0), hasY ? fbytes : 0);
        const Rsrc rFZi = make_rsrc(fZ + (hasZ ? fdir + ((long)(K - sz) * NJ + J) * nx * 8 * FU : 0), hasZ ? fbytes : 0);
        // Octant-relative row r is physical row sx > 0 ? r : nx-1-r, at byte
        // pbase + r * pstep of the pencil.  For every r outside [0, nx) that
        // offset (plus a lane offset below one row) is negative or past the
        // end, i.e. out of the buffer: loads there read zero and stores are
        // dropped, with no test.
        const int pstep = sx * RB, pbase = sx > 0 ? 0 : (nx - 1) * RB;
        const int fstep = sx * FB, fbase = sx > 0 ? 0 : (nx - 1) * FB;
        const int lofs = lane * (int)sizeof(T);  // load phase: lane = physical column
        // load phase for faces: lane = (row in chunk ro, entry e); Y entries
        // are indexed by kp and used by the lane j_r = 0 with skew k_r, Z
        // entries by jp and used by the lane k_r = 0 with skew j_r
        const int e = lane & 7, ro = lane >> 3;
        const int skY = sz > 0 ? e : 7 - e, skZ = sy > 0 ? e : 7 - e;
        const int eoff = e * (int)Face::BYTES;

        // sigma (SM: material byte) of octant-relative row r at byte sbase + r * sstep
        constexpr int SR = Sig::ROW;
        const int sbase = sx > 0 ? 0 : (nx - 1) * SR, sstep = sx * SR;
        const int slofs = pl * (SR / 64);  // the lane's own column (step phase)
        auto sig_off = [&](int ir0) { return sbase + ir0 * sstep + slofs; };

        T pq[CH];  // psi rows of the next chunk (load phase)
        U32x2 pmt;                 // SM: material bytes of the next chunk (load phase)
        typename Sig::Reg ps[CH];  // !SM: sigma of the lane's column at the current chunk's steps
        unsigned pm[CH];           // kTrans: fixed-axis sets of the lane's cells at the current chunk's steps
        typename Face::Word pfy, pfz;
        auto load_rows = [&](int c) {
            int off = pbase + CH * c * pstep + lofs;
#pragma unroll
            for (int b = 0; b < CH; ++b, off += pstep) pq[b] = buf_load<kPsiAux>(rPsi, (unsigned)off, T());
            const unsigned fo = (unsigned)(fbase + (CH * c + ro) * fstep + eoff);
            Face::template load<kLoadAux>(pfy, rFYi, fo);
            Face::template load<kLoadAux>(pfz, rFZi, fo);
            if constexpr (SM) pmt = load_mat_rows(rSig, c, sx, nx, lane);
        };
        // commit chunk c (rows past the end hold zeros and are never used);
        // face words whose stamp is not yet this sweep's are read again
        auto commit = [&](int c) -> bool {
            const int q0 = (CH * c) % RQ;  // 0, 8 or 16: no wrap inside the chunk
#pragma unroll
            for (int b = 0; b < CH; ++b) sQ[w][q0 + b][lane] = pq[b];
            if constexpr (SM) *(U32x2 *)&sMt[w][q0 + mat_row(sx, lane)][8 * (lane & 7)] = pmt;
            const int r = CH * c + ro;
            const bool valid = r < nx;
            bool okY = !valid || !hasY || Face::ok(pfy, stamp);
            bool okZ = !valid || !hasZ || Face::ok(pfz, stamp);
            int spins = 0;
            bool good = true;
            if (__any(!(okY && okZ))) {
                const unsigned fo = (unsigned)(fbase + r * fstep + eoff);
                do {
                    __builtin_amdgcn_s_sleep(2);
                    if (!okY) {
                        Face::template load<kPollAux>(pfy, rFYi, fo);
                        okY = Face::ok(pfy, stamp);
                    }
                    if (!okZ) {
                        Face::template load<kPollAux>(pfz, rFZi, fo);
                        okZ = Face::ok(pfz, stamp);
                    }
                    if (++spins > a0.sweep_spin_limit || ((spins & 255) == 0 && coherent_load(&ctr[1]))) {
                        atomicMax(&ctr[0], kTicketStop);
                        if constexpr (XCD)
                            for (int q = 0; q < nq; ++q) atomicMax(&ctr[kQueueCtr + q], kTicketStop);
                        coherent_store(&ctr[1], 1);
                        good = false;
                        break;
                    }
                } while (__any(!(okY && okZ)));
            }
            sFYi[w][(r + skY) & (RF - 1)][e] = Face::value(pfy);
            sFZi[w][(r + skZ) & (RF - 1)][e] = Face::value(pfz);
            return good;
        };
        T px = T(0), oy = T(0), oz = T(0);
        // One chunk of CH steps.  The chunk's LDS inputs are read first, the
        // steps run from registers, psi and the face outflows go back to LDS
        // at the end.  Lanes outside 0 <= i_r < nx step too, with no test:
        // before its first row a lane sees zero source, sigma and inflow
        // (zeroed ring slots, out-of-range loads), so it carries zero x
        // inflow into row 0; past the last row its results land only in ring
        // slots and face slots of rows that are never stored.
        auto steps = [&](int c) {
            const int t0 = CH * c, ir0 = t0 - skew;
            int s0 = ir0 % RQ;
            s0 = s0 < 0 ? s0 + RQ : s0;
            const int ft = t0 & (RF - 1);  // 0 or 8
            int sq[CH];
            T q[CH], fy[CH], fz[CH], po[CH], yo_[CH], zo_[CH], sg[CH];
#pragma unroll
            for (int b = 0; b < CH; ++b) {
                sq[b] = s0 + b < RQ ? s0 + b : s0 + b - RQ;
                q[b] = sQ[w][sq[b]][pl];
                fy[b] = sFYi[w][ft + b][kp];
                fz[b] = sFZi[w][ft + b][jp];
                if constexpr (SM) sg[b] = sSigT[sMt[w][sq[b]][pl] & (kSigTab - 1)];
            }
            int so = sig_off(ir0 + CH);
            int mo = mbase + ir0 * mstep + pl;  // kRecord / kTrans: the lane's cell at step b
#pragma unroll
            for (int b = 0; b < CH; ++b, so += sstep, mo += mstep) {
                T iny = lane_shr1(oy);
                T inz = lane_from(oz, srcZ);
                iny = yb ? fy[b] : iny;
                inz = zb ? fz[b] : inz;
                T ox_, oy_, oz_;
                unsigned mk = 0;
                if constexpr (MODE == kTrans) mk = pm[b];
                if constexpr (!SM) sg[b] = Sig::value(ps[b], sSigT);
                po[b] = dd_update<T, MODE>(q[b], sg[b], cx, cy, cz, csum, px, iny, inz, ox_, oy_, oz_, mk);
                if constexpr (MODE == kRecord)
                    __builtin_amdgcn_raw_buffer_store_b8((unsigned char)mk, rMask, mo, 0, 0);
                if constexpr (MODE == kTrans)
                    pm[b] = __builtin_amdgcn_raw_buffer_load_b8(rMask, mo + CH * mstep, 0, 0);  // next chunk
                yo_[b] = oy_;
                zo_[b] = oz_;
                px = ox_;
                oy = oy_;
                oz = oz_;
                if constexpr (!SM) ps[b] = Sig::load(rSig, (unsigned)so);  // the next chunk's sigma
            }
#pragma unroll
            for (int b = 0; b < CH; ++b) sQ[w][sq[b]][pl] = po[b];
            if (yo) {
#pragma unroll
                for (int b = 0; b < CH; ++b) sFYo[w][ft + b][kp] = yo_[b];
            }
            if (zo) {
#pragma unroll
                for (int b = 0; b < CH; ++b) sFZo[w][ft + b][jp] = zo_[b];
            }
        };
        // psi rows 8c-16 .. 8c-9 (slots ((8c-16) mod 24) + b) and face rows
        // 8c-14 .. 8c-7 are complete after chunk c
        auto writeback = [&](int c) {
            const int qw = (CH * c + CH) % RQ;  // (8c - 16) mod 24
            T v[CH];
#pragma unroll
            for (int b = 0; b < CH; ++b) v[b] = sQ[w][qw + b][lane];
            int off = pbase + (CH * c - 16) * pstep + lofs;
#pragma unroll
            for (int b = 0; b < CH; ++b, off += pstep) buf_store<kPsiAux>(rPsi, (unsigned)off, v[b]);
            // Y entry e of row r was made by the lane with skew 7 + skY at
            // step r + 7 + skY (Z likewise)
            const int r = CH * c - 14 + ro;
            const unsigned fo = (unsigned)(fbase + r * fstep + eoff);
            Face::template put<kStoreAux>(rFYo, fo, sFYo[w][(r + 7 + skY) & (RF - 1)][e], stamp);
            Face::template put<kStoreAux>(rFZo, fo, sFZo[w][(r + 7 + skZ) & (RF - 1)][e], stamp);
        };

        const int nchunks = (nx + 15) / CH + 1;
        const int cnext = nchunks > 3 ? nchunks - 3 : 0;  // chunk that takes the next ticket
        // Same issue order as inside the loop (rows, faces, then sigma), so
        // the wait at the loop head can leave the newest loads in flight.
        // rows -14 .. -1 (ring slots 10 .. 23) and the face inflow rings start
        // at zero
#pragma unroll
        for (int s = RQ - 14; s < RQ; ++s) sQ[w][s][lane] = T(0);
        if constexpr (SM) {
#pragma unroll
            for (int s = RQ - 14; s < RQ; ++s) sMt[w][s][lane] = 255;  // the ghost: zero sigma
        }
        sFYi[w][lane >> 2][(lane & 3) * 2] = T(0);
        sFYi[w][lane >> 2][(lane & 3) * 2 + 1] = T(0);
        sFZi[w][lane >> 2][(lane & 3) * 2] = T(0);
        sFZi[w][lane >> 2][(lane & 3) * 2 + 1] = T(0);
        load_rows(0);
        __builtin_amdgcn_sched_barrier(0);
        {
            int so = sig_off(-skew);
            if constexpr (!SM) {
#pragma unroll
                for (int b = 0; b < CH; ++b, so += sstep) ps[b] = Sig::load(rSig, (unsigned)so);
            }
            if constexpr (MODE == kTrans) {
                int mo = mbase - skew * mstep + pl;
#pragma unroll
                for (int b = 0; b < CH; ++b, mo += mstep) pm[b] = __builtin_amdgcn_raw_buffer_load_b8(rMask, mo, 0, 0);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        writeback(-1);  // all out of range: only mirrors the loop's issue pattern
        __builtin_amdgcn_sched_barrier(0);
        for (int c = 0; c < nchunks; ++c) {
            if (!commit(c)) break;  // abort: the block leaves at the next ticket
            if (c == cnext && threadIdx.x == 0) {
                tnext = atomicAdd(tctr, 1);
                have_next = true;
            }
            load_rows(c + 1);
            steps(c);
            writeback(c);
        }
    }
}

template <typename T, int MODE, int WPB, bool SM, bool XCD, bool NT>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && WPB >= 2 ? (WPB >= 10 ? 3 : 4) : 1))) void k_sweep(SolveArgs<T> a0, int g)
{
    sweep_body<T, MODE, WPB, SM, XCD, NT, false>(a0, g);
}

// The sweep of every (problem, source) pair of a fused batch in one launch.
template <typename T, int MODE, int WPB, bool SM, bool NT>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && WPB >= 2 ? (WPB >= 10 ? 3 : 4) : 1))) void k_sweep_multi(SolveArgs<T> a0, int g)
{
    sweep_body<T, MODE, WPB, SM, false, NT, true>(a0, g);
}

// Column-relay sweep: the same cell updates as k_sweep with the y faces
// kept on chip.
//
// Work item = (octant o, group of W directions dg, pencil row K_r,
// source): every pencil (J_r, K_r), J_r = 0 .. NJ-1, of W directions.  The
// block has W x R waves; wave (slot, role) sweeps direction dg * W + slot
// over the pencils J_r = role, role + R, role + 2R, ... in turn, each with
// the per-wave pipeline of k_sweep (LDS row ring, skewed face rings, chunks
// of 8 steps).  The y outflow of pencil J_r is the y inflow of pencil
// J_r + 1, which the wave of the next role sweeps: it is handed over in LDS
// (a buffer of one pencil's face rows per wave, with counters of the rows
// published and consumed), so y faces never reach memory.  Only the z faces
// between rows K_r - 1 and K_r go through the stamped face words of k_sweep.
// The handover waits are bounded like the face-word polls.
//
// Tickets are numbered row by row (all items of K_r = 0 first), so an
// item's upstream item (K_r - 1) holds a smaller ticket and is already
// running: every wait ends.  Inside a block the waits point to smaller J_r
// only (the inflow of J_r comes from J_r - 1; a wave re-fills its handover
// buffer with pencil J_r + R only after J_r + 1 has read those rows).
template <typename T, int MODE, int W, int R, bool SM, bool NT>
__global__ __launch_bounds__(64 * W * R) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void k_sweep_col(SolveArgs<T> a0, int g)
{
    static_assert(MODE == kDD || MODE == kFixup, "forward cell modes only");
    constexpr int kLoadAux = kSC1, kPollAux = kVolatileSC1, kStoreAux = kSC1;
    constexpr int kPsiAux = NT ? kNT : 0;
    typedef SigSrc<T, SM> Sig;
    typedef typename FaceCodecSel<T, MODE, false>::type Face;
    constexpr bool kSignFace = std::is_same<Face, SignFace<T>>::value;
    constexpr int NW = W * R;
    constexpr int RQ = 24, RF = 16, CH = 8;
    constexpr int RB = 64 * sizeof(T);
    constexpr int FB = 8 * (int)Face::BYTES;
    __shared__ T sQ[NW][RQ][64];
    __shared__ T sFYi[NW][RF][8], sFZi[NW][RF][8], sFYo[NW][RF][8], sFZo[NW][RF][8];
    __shared__ int sTicket, sNext, sAbort;
    __shared__ int sProd[NW], sCons[NW];  // handover rows published / consumed (counted over the wave's pencils)
    __shared__ T sSigT[SM ? kSigTab : 1];
    __shared__ __align__(16) unsigned char sMt[SM ? NW : 1][SM ? RQ : 1][64];  // SM: material byte ring (slots as sQ)
    extern __shared__ unsigned char sDyn[];  // handover buffers [NW][nx][8] of T
    T *const sRelay = (T *)sDyn;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int slot = w / R, role = w % R;
    const int D = a0.D, ngrp = D / W;
    const int NJ = a0.g.NJ, NK = a0.g.NK, nx = a0.g.nx;
    int *const ctr = a0.sweep_ctr;
    const unsigned epoch = (unsigned)ctr[2];
    const int nitems = a0.sweep_nitems;
    const int per_row = a0.S * 8 * ngrp;  // items of one pencil row K_r

    bool live = false;
    for (int s = 0; s < a0.S; ++s) live = live || !a0.ctl[(long)s * a0.G + g].done;
    if (!live) return;
    if (SM)
        for (int i = threadIdx.x; i < kSigTab; i += 64 * NW)
            sSigT[i] = i < a0.nmat ? (T)a0.xs_t[i * a0.G + g] : T(0);
    if (threadIdx.x == 0) sNext = -1;
    // A wave of the last role takes the next ticket three chunks before its
    // last pencil ends (the block's last work), so the atomic hides behind
    // those chunks; a block holds at most two tickets, and the smallest
    // unfinished ticket is always being worked on.
    for (;;) {
        __syncthreads();  // every wave is done with the previous item (and sNext is written)
        if (threadIdx.x == 0) {
            sTicket = sNext >= 0 ? sNext : atomicAdd(&ctr[0], 1);
            sNext = -1;
            sAbort = 0;
        }
        if (threadIdx.x < NW) {
            sProd[threadIdx.x] = 0;
            sCons[threadIdx.x] = 0;
        }
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(sTicket);
        if (t >= nitems) break;
        const int Kr = t / per_row;
        int u = t - Kr * per_row;
        const int dg = u % ngrp;
        u /= ngrp;
        const int o = u & 7, src = u >> 3;
        const SolveArgs<T> a = at_source(a0, src);
        if (a.ctl[g].done) continue;  // this source's group has converged
        const int n = o * D + dg * W + slot;
        const unsigned stamp = kSignFace ? (unsigned)a.face_par[0] : epoch;
        const int sx = (o & 1) ? -1 : 1, sy = (o & 2) ? -1 : 1, sz = (o & 4) ? -1 : 1;
        const int K = sz > 0 ? Kr : NK - 1 - Kr;
        const int jr = lane & 7, kr = lane >> 3;
        const int jp = sy > 0 ? jr : 7 - jr, kp = sz > 0 ? kr : 7 - kr;
        const int pl = jp + 8 * kp;
        const int skew = jr + kr;
        const int srcZ = ((lane - 8) & 63) << 2;
        const bool yb = jr == 0, zb = kr == 0, yo = jr == 7, zo = kr == 7;
        const T cx = a.cdir[3 * n], cy = a.cdir[3 * n + 1], cz = a.cdir[3 * n + 2];
        const T csum = cx + cy + cz;
        constexpr int FU = Face::BYTES / 4;
        unsigned *const fZ = (unsigned *)a.faceZ;
        const long fdir = (long)n * NJ * NK * nx * 8 * FU;
        const bool hasZ = Kr > 0;
        const unsigned fbytes = (unsigned)(nx * FB);
        const int pstep = sx * RB, pbase = sx > 0 ? 0 : (nx - 1) * RB;
        const int fstep = sx * FB, fbase = sx > 0 ? 0 : (nx - 1) * FB;
        const int lofs = lane * (int)sizeof(T);
        const int e = lane & 7, ro = lane >> 3;
        const int skY = sz > 0 ? e : 7 - e, skZ = sy > 0 ? e : 7 - e;
        const int eoff = e * (int)Face::BYTES;
        constexpr int SR = Sig::ROW;
        const int sbase = sx > 0 ? 0 : (nx - 1) * SR, sstep = sx * SR;
        const int slofs = pl * (SR / 64);
        const int nchunks = (nx + 15) / CH + 1;
        // handover buffers: this wave's outflow, and the inflow from the
        // wave of the previous role (the last role's for role 0, one pencil
        // behind)
        const int win = slot * R + (role + R - 1) % R;
        T *const relOut = sRelay + (long)w * nx * 8;
        const T *const relIn = sRelay + (long)win * nx * 8;
        const int npen = role < NJ ? (NJ - 1 - role) / R + 1 : 0;
        bool good = true;
        for (int k = 0; k < npen && good; ++k) {
            const int Jr = role + R * k;
            const int J = sy > 0 ? Jr : NJ - 1 - Jr;
            const bool hasY = Jr > 0, needY = Jr < NJ - 1;
            const int seq_in = role == 0 ? k - 1 : k;  // the inflow's pencil in its producer's order
            const long pen = (long)K * NJ + J;
            const Rsrc rPsi = make_rsrc(a.psi + psi_run(pen, a.Nd, n, nx), (unsigned)(nx * RB));
            const Rsrc rSig = SM ? make_rsrc(a.mat + pen * nx * 64, (unsigned)(nx * 64))
                                 : make_rsrc(a.sig + pen * nx * 64, (unsigned)(nx * RB));
            const long fown = fdir + pen * nx * 8 * FU;
            const Rsrc rFZo = make_rsrc(fZ + fown, Kr < NK - 1 ? fbytes : 0u);  // the last row's are never read
            const Rsrc rFZi = make_rsrc(fZ + (hasZ ? fdir + ((long)(K - sz) * NJ + J) * nx * 8 * FU : 0),
                                        hasZ ? fbytes : 0);
            T pq[CH];
            U32x2 pmt;                 // SM: material bytes of the next chunk (load phase)
            typename Sig::Reg ps[CH];  // !SM: sigma of the lane's column at the current chunk's steps
            typename Face::Word pfz;
            auto load_rows = [&](int c) {
                int off = pbase + CH * c * pstep + lofs;
#pragma unroll
                for (int b = 0; b < CH; ++b, off += pstep) pq[b] = buf_load<kPsiAux>(rPsi, (unsigned)off, T());
                const unsigned fo = (unsigned)(fbase + (CH * c + ro) * fstep + eoff);
                Face::template load<kLoadAux>(pfz, rFZi, fo);
                if constexpr (SM) pmt = load_mat_rows(rSig, c, sx, nx, lane);
            };
            // a bounded wait on a handover counter of this block
            auto wait_lds = [&](const int *cnt, int need) -> bool {
                int spins = 0;
                while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < need) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > a0.sweep_spin_limit ||
                        ((spins & 255) == 0 && (__hip_atomic_load(&sAbort, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_WORKGROUP) ||
                                                coherent_load(&ctr[1]))))
                        return false;
                }
                return true;
            };
            auto abort_all = [&]() {
                atomicMax(&ctr[0], kTicketStop);
                coherent_store(&ctr[1], 1);
                __hip_atomic_store(&sAbort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            };
            auto commit = [&](int c) -> bool {
                const int q0 = (CH * c) % RQ;
#pragma unroll
                for (int b = 0; b < CH; ++b) sQ[w][q0 + b][lane] = pq[b];
                if constexpr (SM) *(U32x2 *)&sMt[w][q0 + mat_row(sx, lane)][8 * (lane & 7)] = pmt;
                const int r = CH * c + ro;
                const bool valid = r < nx;
                bool okZ = !valid || !hasZ || Face::ok(pfz, stamp);
                int spins = 0;
                if (__any(!okZ)) {
                    const unsigned fo = (unsigned)(fbase + r * fstep + eoff);
                    do {
                        __builtin_amdgcn_s_sleep(2);
                        if (!okZ) {
                            Face::template load<kPollAux>(pfz, rFZi, fo);
                            okZ = Face::ok(pfz, stamp);
                        }
                        if (++spins > a0.sweep_spin_limit || ((spins & 255) == 0 && coherent_load(&ctr[1]))) {
                            abort_all();
                            return false;
                        }
                    } while (__any(!okZ));
                }
                sFZi[w][(r + skZ) & (RF - 1)][e] = Face::value(pfz);
                T fy = T(0);
                if (hasY) {
                    const int upto = CH * c + CH < nx ? CH * c + CH : nx;
                    if (!wait_lds(&sProd[win], seq_in * nx + upto)) {
                        abort_all();
                        return false;
                    }
                    if (valid) fy = relIn[r * 8 + e];
                }
                sFYi[w][(r + skY) & (RF - 1)][e] = fy;
                if (hasY && lane == 0)  // the rows of this chunk are read: the producer may reuse them
                    __hip_atomic_store(&sCons[win], seq_in * nx + (CH * c + CH < nx ? CH * c + CH : nx),
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                return true;
            };
            auto sig_off = [&](int ir0) { return sbase + ir0 * sstep + slofs; };
            T px = T(0), oy = T(0), oz = T(0);
            auto steps = [&](int c) {
                const int t0 = CH * c, ir0 = t0 - skew;
                int s0 = ir0 % RQ;
                s0 = s0 < 0 ? s0 + RQ : s0;
                const int ft = t0 & (RF - 1);
                int sq[CH];
                T q[CH], fy[CH], fz[CH], po[CH], yo_[CH], zo_[CH], sg[CH];
#pragma unroll
                for (int b = 0; b < CH; ++b) {
                    sq[b] = s0 + b < RQ ? s0 + b : s0 + b - RQ;
                    q[b] = sQ[w][sq[b]][pl];
                    fy[b] = sFYi[w][ft + b][kp];
                    fz[b] = sFZi[w][ft + b][jp];
                    if constexpr (SM) sg[b] = sSigT[sMt[w][sq[b]][pl] & (kSigTab - 1)];
                }
                int so = sig_off(ir0 + CH);
#pragma unroll
                for (int b = 0; b < CH; ++b, so += sstep) {
                    T iny = lane_shr1(oy);
                    T inz = lane_from(oz, srcZ);
                    iny = yb ? fy[b] : iny;
                    inz = zb ? fz[b] : inz;
                    T ox_, oy_, oz_;
                    unsigned mk = 0;
                    if constexpr (!SM) sg[b] = Sig::value(ps[b], sSigT);
                    po[b] = dd_update<T, MODE>(q[b], sg[b], cx, cy, cz, csum, px, iny, inz, ox_, oy_, oz_, mk);
                    yo_[b] = oy_;
                    zo_[b] = oz_;
                    px = ox_;
                    oy = oy_;
                    oz = oz_;
                    if constexpr (!SM) ps[b] = Sig::load(rSig, (unsigned)so);
                }
#pragma unroll
                for (int b = 0; b < CH; ++b) sQ[w][sq[b]][pl] = po[b];
                if (yo) {
#pragma unroll
                    for (int b = 0; b < CH; ++b) sFYo[w][ft + b][kp] = yo_[b];
                }
                if (zo) {
#pragma unroll
                    for (int b = 0; b < CH; ++b) sFZo[w][ft + b][jp] = zo_[b];
                }
            };
            auto writeback = [&](int c) -> bool {
                const int qw = (CH * c + CH) % RQ;
                T v[CH];
#pragma unroll
                for (int b = 0; b < CH; ++b) v[b] = sQ[w][qw + b][lane];
                int off = pbase + (CH * c - 16) * pstep + lofs;
#pragma unroll
                for (int b = 0; b < CH; ++b, off += pstep) buf_store<kPsiAux>(rPsi, (unsigned)off, v[b]);
                const int r = CH * c - 14 + ro;
                const unsigned fo = (unsigned)(fbase + r * fstep + eoff);
                Face::template put<kStoreAux>(rFZo, fo, sFZo[w][(r + 7 + skZ) & (RF - 1)][e], stamp);
                if (needY) {
                    // rows CH c - 14 .. CH c - 7 are complete; before they
                    // overwrite the previous pencil's, its reader must be done
                    // with them
                    const int hi = CH * c - 6 < nx ? CH * c - 6 : nx;
                    if (hi > 0) {
                        if (k > 0 && !wait_lds(&sCons[w], (k - 1) * nx + hi)) {
                            abort_all();
                            return false;
                        }
                        if (r >= 0 && r < nx) relOut[r * 8 + e] = sFYo[w][(r + 7 + skY) & (RF - 1)][e];
                        if (lane == 0)
                            __hip_atomic_store(&sProd[w], k * nx + hi, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
                return true;
            };
            const int cnext = nchunks > 3 ? nchunks - 3 : 0;
#pragma unroll
            for (int s = RQ - 14; s < RQ; ++s) sQ[w][s][lane] = T(0);
            if constexpr (SM) {
#pragma unroll
                for (int s = RQ - 14; s < RQ; ++s) sMt[w][s][lane] = 255;  // the ghost: zero sigma
            }
            sFYi[w][lane >> 2][(lane & 3) * 2] = T(0);
            sFYi[w][lane >> 2][(lane & 3) * 2 + 1] = T(0);
            sFZi[w][lane >> 2][(lane & 3) * 2] = T(0);
            sFZi[w][lane >> 2][(lane & 3) * 2 + 1] = T(0);
            load_rows(0);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (!SM) {
                int so = sig_off(-skew);
#pragma unroll
                for (int b = 0; b < CH; ++b, so += sstep) ps[b] = Sig::load(rSig, (unsigned)so);
            }
            __builtin_amdgcn_sched_barrier(0);
            for (int c = 0; c < nchunks; ++c) {
                if (!commit(c)) {
                    good = false;
                    break;
                }
                if (c == cnext && k == npen - 1 && role == R - 1 && slot == 0 && lane == 0)
                    sNext = atomicAdd(&ctr[0], 1);
                load_rows(c + 1);
                steps(c);
                if (!writeback(c)) {
                    good = false;
                    break;
                }
            }
        }
    }
}

// Before every sweep: ticket counter back to zero and the next epoch for the
// tagged face words, kept in [1, 2^31 - 1] (invalidated words hold all ones).
// Both live in device memory, so a captured graph replays correctly.
__global__ void k_sweep_reset(int *ctr)
{
    if (blockIdx.x == 0 && threadIdx.x < 8) ctr[kQueueCtr + threadIdx.x] = 0;  // per-XCD queues
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[0] = 0;
        ctr[2] = (int)((unsigned)ctr[2] % 0x7FFFFFFEu + 1u);
    }
}

// The XCD each workgroup runs on (hardware register XCC_ID), for the
// runtime's check of the workgroup-to-XCD mapping before it uses per-XCD
// queues.
__global__ void k_xcc_probe(int *out, int n)
{
    if (threadIdx.x == 0 && (int)blockIdx.x < n) out[blockIdx.x] = (int)__builtin_amdgcn_s_getreg((3 << 11) | 20);
}

// Order-independent checksum of n 32-bit words (wrapping sum of the words
// and of their rotations), for comparing two sweeps' angular fluence bit for
// bit.
__global__ void k_checksum(const unsigned *x, long n, unsigned long long *out)
{
    unsigned long long acc = 0;
    for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256)
        acc += (unsigned long long)x[i] * 0x9E3779B1ull + ((unsigned long long)((unsigned)i * 0x85EBCA6Bu) ^ x[i]);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

// After a sweep with per-XCD queues: if some source was live and a queue's
// counter never reached its item count (no block ran on that XCD), the abort
// flag is raised with value 2 and the host reports the launch as failed.
__global__ void k_xcd_drained(const Ctl *ctl, int G, int g, int S, int *ctr, int nq, int nitems_q)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bool live = false;
    for (int s = 0; s < S; ++s) live = live || !ctl[(long)s * G + g].done;
    bool drained = true;
    for (int q = 0; q < nq; ++q) drained = drained && ctr[kQueueCtr + q] >= nitems_q;
    if (live && !drained) ctr[1] = 2;
}

// After a sweep with sign-parity faces: flip the parity of every source that
// ran (its group had not converged), so its next sweep rejects these words.
__global__ void k_face_parity_flip(const Ctl *ctl, int G, int g, int S, int *par)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S && !ctl[(long)s * G + g].done) par[s] ^= 1;
}


// Default waves per block (directions of one octant that share a pencil
// item); the runtime may pick another divisor of D by timing.
int sweep_wpb(int D, bool fp64)
{
    if (D % 4 == 0 && !fp64) return 4;
    if (D % 2 == 0) return 2;
    return 1;
}

// Waves per block the sweep is built for (FP64 rows take twice the LDS, so
// its list stops at 6).
#define DSN_WPB_F32(X) X(1) X(2) X(3) X(4) X(5) X(6) X(9) X(10) X(12)
#define DSN_WPB_F64(X) X(1) X(2) X(3) X(4) X(5) X(6)

int sweep_wpb_choices(bool fp64, int *out)
{
    int n = 0;
#define DSN_PUT(W) out[n++] = W;
    if (fp64) {
        DSN_WPB_F64(DSN_PUT)
    } else {
        DSN_WPB_F32(DSN_PUT)
    }
#undef DSN_PUT
    return n;
}

// NT (non-temporal angular fluence) variants for the forward cell modes
template <typename T, int MODE, int WPB>
static const void *sweep_kernel(bool sm, bool nt)
{
    if constexpr (MODE == kDD || MODE == kFixup) {
        if (nt)
            return sm ? (const void *)&k_sweep<T, MODE, WPB, true, false, true>
                      : (const void *)&k_sweep<T, MODE, WPB, false, false, true>;
    }
    return sm ? (const void *)&k_sweep<T, MODE, WPB, true, false, false>
              : (const void *)&k_sweep<T, MODE, WPB, false, false, false>;
}

// Per-XCD-queue variants: FP32 with the fixup, up to four waves per block.
template <typename T>
static const void *sweep_kernel_xcd(int wpb, int mode, bool sm, bool nt)
{
    if constexpr (sizeof(T) == 4) {
        if (mode != kFixup) return nullptr;
#define DSN_XPICK(W)                                                                                  \
    if (wpb == W)                                                                                     \
        return nt ? (sm ? (const void *)&k_sweep<float, kFixup, W, true, true, true>                  \
                        : (const void *)&k_sweep<float, kFixup, W, false, true, true>)                \
                  : (sm ? (const void *)&k_sweep<float, kFixup, W, true, true, false>                 \
                        : (const void *)&k_sweep<float, kFixup, W, false, true, false>);
        DSN_XPICK(1) DSN_XPICK(2) DSN_XPICK(3) DSN_XPICK(4)
#undef DSN_XPICK
    }
    return nullptr;
}

bool sweep_xcd_supported(bool fp64, int mode, int wpb) { return !fp64 && mode == kFixup && wpb >= 1 && wpb <= 4; }

// Column-relay variants (forward cell modes): (directions, roles) per block
// of W x R waves.
#define DSN_COL_F32(X) X(1, 2) X(1, 4) X(2, 2) X(2, 4)
#define DSN_COL_F64(X) X(1, 2) X(1, 4)

int sweep_col_choices(bool fp64, int *w_out, int *r_out)
{
    int n = 0;
#define DSN_PUT2(W, R) w_out[n] = W, r_out[n++] = R;
    if (fp64) {
        DSN_COL_F64(DSN_PUT2)
    } else {
        DSN_COL_F32(DSN_PUT2)
    }
#undef DSN_PUT2
    return n;
}

template <typename T, int MODE, int W, int R>
static const void *sweep_kernel_col_nt(bool sm, bool nt)
{
    if (nt)
        return sm ? (const void *)&k_sweep_col<T, MODE, W, R, true, true>
                  : (const void *)&k_sweep_col<T, MODE, W, R, false, true>;
    return sm ? (const void *)&k_sweep_col<T, MODE, W, R, true, false>
              : (const void *)&k_sweep_col<T, MODE, W, R, false, false>;
}

template <typename T>
static const void *sweep_kernel_col(int w, int r, int mode, bool sm, bool nt)
{
    if (mode != kDD && mode != kFixup) return nullptr;
#define DSN_CPICK(W, R)                                                                                  if (w == W && r == R)                                                                                   return mode == kDD ? sweep_kernel_col_nt<T, kDD, W, R>(sm, nt) : sweep_kernel_col_nt<T, kFixup, W, R>(sm, nt);
    if constexpr (sizeof(T) == 8) {
        DSN_COL_F64(DSN_CPICK)
    } else {
        DSN_COL_F32(DSN_CPICK)
    }
#undef DSN_CPICK
    return nullptr;
}

// Dynamic LDS of a column-relay block: one pencil of y-face rows per wave.
static size_t col_lds_bytes(int w, int r, int nx, size_t tsize) { return (size_t)w * r * nx * 8 * tsize; }

bool sweep_tagged_faces(bool fp64, int mode, int wpb, int xcd)
{
    return mode == kDD || mode == kTrans || (xcd > 0 && sweep_xcd_supported(fp64, mode, wpb));
}

template <typename T>
static const void *sweep_kernel_of(int wpb, int mode, bool sm, bool nt)
{
#define DSN_PICK(W)                                           \
    if (wpb == W) {                                           \
        switch (mode) {                                       \
        case kDD: return sweep_kernel<T, kDD, W>(sm, nt);         \
        case kFixup: return sweep_kernel<T, kFixup, W>(sm, nt);   \
        case kRecord: return sweep_kernel<T, kRecord, W>(sm, nt); \
        case kTrans: return sweep_kernel<T, kTrans, W>(sm, nt);   \
        default: return nullptr;                              \
        }                                                     \
    }
    if constexpr (sizeof(T) == 8) {
        DSN_WPB_F64(DSN_PICK)
    } else {
        DSN_WPB_F32(DSN_PICK)
    }
#undef DSN_PICK
    return nullptr;
}

// Fused-batch (several problems per launch) variants: the forward cell
// modes, global queue, up to five waves per block in FP32 and three in FP64
// (every S_N order up to S16 has a divisor of N(N+2)/8 among them).
#define DSN_WPB_MULTI_F32(X) X(1) X(2) X(3) X(4) X(5)
#define DSN_WPB_MULTI_F64(X) X(1) X(2) X(3)

int sweep_multi_choices(bool fp64, int *out)
{
    int n = 0;
#define DSN_PUT(W) out[n++] = W;
    if (fp64) {
        DSN_WPB_MULTI_F64(DSN_PUT)
    } else {
        DSN_WPB_MULTI_F32(DSN_PUT)
    }
#undef DSN_PUT
    return n;
}

template <typename T, int MODE, int WPB>
static const void *sweep_kernel_multi_nt(bool sm, bool nt)
{
    if (nt)
        return sm ? (const void *)&k_sweep_multi<T, MODE, WPB, true, true>
                  : (const void *)&k_sweep_multi<T, MODE, WPB, false, true>;
    return sm ? (const void *)&k_sweep_multi<T, MODE, WPB, true, false>
              : (const void *)&k_sweep_multi<T, MODE, WPB, false, false>;
}

template <typename T>
static const void *sweep_kernel_multi(int wpb, int mode, bool sm, bool nt)
{
    if (mode != kDD && mode != kFixup) return nullptr;
#define DSN_MPICK(W)                                                                                   \
    if (wpb == W)                                                                                      \
        return mode == kDD ? sweep_kernel_multi_nt<T, kDD, W>(sm, nt) : sweep_kernel_multi_nt<T, kFixup, W>(sm, nt);
    if constexpr (sizeof(T) == 8) {
        DSN_WPB_MULTI_F64(DSN_MPICK)
    } else {
        DSN_WPB_MULTI_F32(DSN_MPICK)
    }
#undef DSN_MPICK
    return nullptr;
}

// Resident blocks of the fused-batch sweep (grid size), 0 if not built.
template <typename T>
int sweep_grid_multi(int wpb, int mode, int n_cu)
{
    int per_cu = 1 << 30;
    for (int sm = 0; sm < 2; ++sm) {
        const void *f = sweep_kernel_multi<T>(wpb, mode, sm != 0, false);
        if (!f) return 0;
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * wpb, 0) != hipSuccess || n < 1) n = 1;
        per_cu = n < per_cu ? n : per_cu;
    }
    return per_cu * n_cu;
}

// One sweep over every (problem, source) pair of a fused batch: a.multi (device
// copy of host_tab) and a.seg set, a.sweep_ctr the batch's own counter block;
// then each problem's face parity flips for its sources that ran.
template <typename T>
int launch_sweep_multi(const SolveArgs<T> &a, const SolveArgs<T> *host_tab, int n, int g, hipStream_t s,
                       hipEvent_t ev_before, hipEvent_t ev_after)
{
    const void *f = sweep_kernel_multi<T>(a.sweep_wpb, a.sweep_mode, a.sig_from_mat != 0, a.stream_nt != 0);
    if (!f) return 0;
    hipLaunchKernelGGL(k_sweep_reset, dim3(1), dim3(64), 0, s, a.sweep_ctr);
    SolveArgs<T> arg = a;
    int gi = g;
    void *params[2] = {&arg, &gi};
    const unsigned grid = (unsigned)(a.sweep_grid < a.sweep_nitems ? a.sweep_grid : a.sweep_nitems);
    if (ev_before) (void)hipEventRecord(ev_before, s);
    (void)hipLaunchKernel(f, dim3(grid), dim3(64 * a.sweep_wpb), params, 0, s);
    if (ev_after) (void)hipEventRecord(ev_after, s);
    if (a.sweep_mode == kFixup)
        for (int q = 0; q < n; ++q) {
            const SolveArgs<T> &b = host_tab[q];
            hipLaunchKernelGGL(k_face_parity_flip, dim3((b.S + 63) / 64), dim3(64), 0, s, b.ctl, b.G, g, b.S,
                               b.face_par);
        }
    return 1;
}

// Resident blocks of the column-relay sweep with w directions and r roles per
// block for an x extent of nx (grid size), 0 if there is no such kernel or
// its LDS does not fit.
template <typename T>
int sweep_grid_col(int w, int r, int mode, int nx, int n_cu)
{
    int per_cu = 1 << 30;
    for (int sm = 0; sm < 2; ++sm) {
        const void *f = sweep_kernel_col<T>(w, r, mode, sm != 0, false);
        if (!f) return 0;
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * w * r, col_lds_bytes(w, r, nx, sizeof(T))) !=
                hipSuccess ||
            n < 1) {
            (void)hipGetLastError();
            return 0;
        }
        per_cu = n < per_cu ? n : per_cu;
    }
    return per_cu * n_cu;
}

// Resident blocks of the sweep kernel with wpb waves per block in cell mode
// `mode` (grid size), 0 if there is no such kernel.
template <typename T>
int sweep_grid(int wpb, int mode, int n_cu)
{
    int per_cu = 1 << 30;
    for (int sm = 0; sm < 2; ++sm) {  // both sigma variants: the smaller residency
        const void *f = sweep_kernel_of<T>(wpb, mode, sm != 0, false);
        if (!f) return 0;
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, 64 * wpb, 0) != hipSuccess || n < 1) n = 1;
        per_cu = n < per_cu ? n : per_cu;
    }
    return per_cu * n_cu;
}

// Launches the sweep in cell mode a.sweep_mode with a.sweep_wpb waves per
// block (one of the built choices; the runtime never passes another) between
// the ticket reset and, for sign-parity faces, the parity flip.
template <typename T>
int launch_sweeps(const SolveArgs<T> &a, int g, hipStream_t s, hipEvent_t ev_before, hipEvent_t ev_after)
{
    // per-XCD queues where such a kernel is built (FP32 fixup sweeps), else
    // the global queue
    const bool col = sweep_uses_col(a);
    const bool xcd = !col && a.sweep_xcd > 0 && sweep_xcd_supported(sizeof(T) == 8, a.sweep_mode, a.sweep_wpb);
    const bool nt = a.stream_nt != 0;
    const void *f = col ? sweep_kernel_col<T>(a.sweep_wpb, a.sweep_relay, a.sweep_mode, a.sig_from_mat != 0, nt)
                    : xcd ? sweep_kernel_xcd<T>(a.sweep_wpb, a.sweep_mode, a.sig_from_mat != 0, nt)
                          : sweep_kernel_of<T>(a.sweep_wpb, a.sweep_mode, a.sig_from_mat != 0, nt);
    if (!f) return 0;
    hipLaunchKernelGGL(k_sweep_reset, dim3(1), dim3(64), 0, s, a.sweep_ctr);
    unsigned grid = (unsigned)(a.sweep_grid < a.sweep_nitems ? a.sweep_grid : a.sweep_nitems);
    if (xcd)  // a whole number of blocks per XCD, at least one each
        grid = (grid + a.sweep_xcd - 1) / a.sweep_xcd * a.sweep_xcd;
    SolveArgs<T> arg = a;
    if (!xcd) arg.sweep_xcd = 0;
    if (a.sweep_relay > 0 && !col) {
        // a handle tuned to column-relay items sweeps the other cell modes
        // (the adjoint's) with pencil items of as many directions per block
        arg.sweep_relay = 0;
        arg.sweep_nitems = a.sweep_nitems * a.g.NJ;
        grid = (unsigned)(arg.sweep_grid < arg.sweep_nitems ? arg.sweep_grid : arg.sweep_nitems);
    }
    void *params[2] = {&arg, &g};
    const int waves = col ? a.sweep_wpb * a.sweep_relay : a.sweep_wpb;
    const size_t lds = col ? col_lds_bytes(a.sweep_wpb, a.sweep_relay, a.g.nx, sizeof(T)) : 0;
    if (ev_before) (void)hipEventRecord(ev_before, s);
    (void)hipLaunchKernel(f, dim3(grid), dim3(64 * waves), params, lds, s);
    if (ev_after) (void)hipEventRecord(ev_after, s);
    if (xcd)
        hipLaunchKernelGGL(k_xcd_drained, dim3(1), dim3(64), 0, s, a.ctl, a.G, g, a.S, a.sweep_ctr, a.sweep_xcd,
                           a.sweep_nitems / a.sweep_xcd);
    else if (a.sweep_mode == kFixup || a.sweep_mode == kRecord)
        hipLaunchKernelGGL(k_face_parity_flip, dim3((a.S + 63) / 64), dim3(64), 0, s, a.ctl, a.G, g, a.S, a.face_par);
    return 1;
}

void launch_xcc_probe(int *out, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_xcc_probe, dim3(n), dim3(64), 0, s, out, n);
}

void launch_checksum(const void *x, long n_words, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_checksum, dim3(1024), dim3(256), 0, s, (const unsigned *)x, n_words, out);
}

template int sweep_grid<float>(int, int, int);
template int sweep_grid<double>(int, int, int);
template int sweep_grid_col<float>(int, int, int, int, int);
template int sweep_grid_col<double>(int, int, int, int, int);
template int launch_sweeps<float>(const SolveArgs<float> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template int launch_sweeps<double>(const SolveArgs<double> &, int, hipStream_t, hipEvent_t, hipEvent_t);
template int sweep_grid_multi<float>(int, int, int);
template int sweep_grid_multi<double>(int, int, int);
template int launch_sweep_multi<float>(const SolveArgs<float> &, const SolveArgs<float> *, int, int, hipStream_t,
                                       hipEvent_t, hipEvent_t);
template int launch_sweep_multi<double>(const SolveArgs<double> &, const SolveArgs<double> *, int, int, hipStream_t,
                                        hipEvent_t, hipEvent_t);

}  // namespace dsn
