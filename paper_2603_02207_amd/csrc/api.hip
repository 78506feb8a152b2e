// C-ABI entry points: argument checks, workspace layout and the host-side
// orchestration of the Léja + Hutch++ estimator (Alg. 3) on one GPU.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "ld_internal.h"

namespace ld {
namespace {

#define LD_CHECK_HIP(expr)                                                               \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(LD_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

#define LD_CHECK(expr)            \
    do {                          \
        int rc_ = (expr);         \
        if (rc_ != LD_OK) return rc_; \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// leading dimension of an internal block: a multiple of the 16-byte vector
inline int padded_ld(int cols, int elem) {
    const int v = 16 / elem;
    return (cols + v - 1) / v * v;
}

ld_options resolve(const ld_options* o) {
    ld_options r;
    ld_default_options(&r);
    if (o) r = *o;
    return r;
}

int check_csr_args(const ld_csr* A) {
    if (!A) return fail(LD_EINVAL, "A is null");
    if (A->n <= 0) return fail(LD_EINVAL, "n must be positive");
    if (A->n >= (1ll << 31) || A->nnz < 0 || A->nnz >= (1ll << 31))
        return fail(LD_EINVAL, "n and nnz must fit int32");
    if (A->dtype != LD_F32 && A->dtype != LD_F64) return fail(LD_EINVAL, "dtype must be LD_F32 or LD_F64");
    if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return fail(LD_EINVAL, "null CSR array");
    return LD_OK;
}

CsrDev dev_of(const ld_csr* A) {
    return CsrDev{(int)A->n, (int)A->nnz, A->row_ptr, A->col_idx, A->val};
}

// Workspace of the list of rows with more than kLongRow entries.
size_t long_rows_bytes(const ld_csr* A) {
    return align_up((size_t)A->n * 4) + align_up(((size_t)A->n / 256 + 4) * 4) + align_up(16);
}

// Workspace of the row probe and the diagonal storage (taken whether or not
// the matrix turns out to have it).
size_t dia_bytes(const ld_csr* A, const ld_options& o) {
    if (o.csr_only) return align_up(256);
    return align_up((size_t)A->n * kMaxDiag * (A->dtype == LD_F64 ? 8 : 4)) + align_up((size_t)A->n * 2) +
           align_up(256);
}


// Bump allocator over the caller's (or our own) workspace.
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
    void* take(size_t bytes) {
        void* p = base ? base + used : nullptr;
        used += align_up(bytes);
        return p;
    }
};

// Owns an internally allocated workspace when the caller passed none.
struct OwnedWs {
    void* p = nullptr;
    ~OwnedWs() {
        if (p) (void)hipFree(p);
    }
};

int get_workspace(void* ws, size_t ws_bytes, size_t need, OwnedWs& own, Arena& ar) {
    if (ws) {
        // the carved buffers keep the workspace's alignment, and the step
        // kernels' vector width (hence their grids) assumes 256-byte buffers
        if ((uintptr_t)ws % kAlign != 0) return fail(LD_EINVAL, "workspace must be 256-byte aligned");
        if (ws_bytes < need)
            return fail(LD_EWORKSPACE, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                           std::to_string(need));
        ar.base = (char*)ws;
        ar.size = ws_bytes;
        return LD_OK;
    }
    if (hipMalloc(&own.p, need) != hipSuccess) return fail(LD_ENOMEM, "hipMalloc of workspace failed");
    ar.base = (char*)own.p;
    ar.size = need;
    return LD_OK;
}

int validate_csr(const ld_csr* A, int* dflag, hipStream_t st) {
    LD_CHECK_HIP(hipMemsetAsync(dflag, 0, sizeof(int), st));
    LD_CHECK_HIP(launch_validate_csr(dev_of(A), dflag, st));
    int h = 0;
    LD_CHECK_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    if (h) return fail(LD_ECSR, "row_ptr/col_idx is not a CSR structure with sorted in-range columns");
    return LD_OK;
}

// ---------------------------------------------------------------------------
// Column blocking.  Each n x b block of probe columns runs its own recurrence
// (columns never interact inside it), so a matrix of many columns can be
// processed as several narrower blocks.  When the in/out blocks plus the
// matrix fit the 256 MB Infinity Cache the steps stream from there instead of
// HBM; measured on gfx950, a 5-point step at n = 2^20 runs at ~5.5 TB/s with
// <= 24 FP32 columns and ~3.4 TB/s with 32 or more.  Blocks are stored one
// after another (Blk), so every step reads contiguous memory.
// ---------------------------------------------------------------------------
constexpr double kMallBudget = 240e6;
constexpr int kSmallSlots = 12;   // k x k (<= 64 x 64) FP64 scratch matrices
constexpr int kSlotR1 = 10, kSlotR2 = 11;   // CholQR factors, Y = Q_b R2 R1
constexpr int kMaxDotBlock = 64;  // widest column block of the quadratic-form launches

double matrix_bytes(const ld_csr* A, size_t elem) {
    return (double)A->nnz * (double)(elem + 4) + 4.0 * (double)(A->n + 1);
}

// Bytes a launch reads of the matrix as stored: CSR, or the diagonal storage
// (n x nd values; with constant diagonals 2 bytes of presence bits per row).
double stored_bytes(const ld_csr* A, size_t elem, int dia_nd, bool dia_const) {
    return dia_nd > 0 ? (dia_const ? 2.0 * (double)A->n : (double)A->n * dia_nd * elem) : matrix_bytes(A, elem);
}

// Column blocks of the sketch and of [Q_b | U]: as wide as the two blocks a
// step reads and writes (2 n elem bytes per column) allow within
// kBlockPairBudget and, with the matrix as stored, within the Infinity Cache,
// so that the steps run from the cache rather than HBM.  Every block re-reads
// the matrix, so blocks under 8 columns are taken only while those extra
// reads stay below a tenth of the blocks' own bytes.  Measured on gfx950
// (estimates/s at a forced width): 128^3 grid FP32 one 64-column block 24.7,
// 16 columns 25.2, 12: 28.9, 8: 32.1, 4: 26.5; FP64 one block 11.5, 8: 12.8,
// 4: 16.4; 2048^2 GMRF FP32 one 24-column block 47.9, 8: 41.1, 4: 54.6; FP64
// one block 25.9, 4: 23.9, 2: 32.0; 1024^2 grid FP32 20 columns (a 168 MB
// pair) 168-175, narrower 125-127.
constexpr double kBlockPairBudget = 170e6;

int choose_block_width(const ld_csr* A, size_t elem, int cols, int user, double stored) {
    const int v = 16 / (int)elem;
    if (user > 0) return std::min(cols, (user + v - 1) / v * v);
    const double per_col = 2.0 * (double)A->n * (double)elem;   // block in + block out
    const double room = std::min(kBlockPairBudget, kMallBudget - stored);
    int fit = room > 0 ? (int)(room / per_col) : 0;
    fit = fit / v * v;
    if (fit >= cols || fit < v) return cols;   // one block, or no block fits the cache
    const int nb = (cols + fit - 1) / fit;
    if (fit < 8 && (double)(nb - 1) * stored > 0.1 * per_col * cols) return cols;
    const int bw = (cols + nb - 1) / nb;
    return (bw + v - 1) / v * v;
}

// A column-blocked matrix carved from the workspace.
struct BlkMat {
    void* base = nullptr;
    int cols = 0, bw = 1, ld = 1;
    size_t elem = 4;
    Blk desc() const { return Blk{ld, bw, (long long)ld * n_, 0}; }
    int nblocks() const { return cols == 0 ? 0 : (cols + bw - 1) / bw; }
    int bcols(int i) const { return std::min(bw, cols - i * bw); }
    void* block(int i) const { return (char*)base + (size_t)i * ld * n_ * elem; }
    size_t bytes() const { return (size_t)nblocks() * ld * n_ * elem; }
    long long n_ = 0;
};

BlkMat make_blk(long long n, int cols, int bw, size_t elem) {
    BlkMat b;
    b.n_ = n;
    b.cols = cols;
    b.bw = std::max(1, std::min(bw, std::max(cols, 1)));
    b.ld = padded_ld(b.bw, (int)elem);
    b.elem = elem;
    return b;
}

struct EstLayout {
    int k, kg, nc, nslots, nwg_dot;
    size_t elem;
    BlkMat Y, Q1, X;          // sketch, first CholQR factor, [Q_b | U]
    size_t yb, q1b, xb;       // their regions (see layout_envelope)
    size_t mask, planes, W, part, small, nu, flag;
    // gradient extras: F [Q_b|U], the materialised residual probes, a k-column
    // temporary, the FP64 gradient accumulator of an FP32 matrix, then one of
    // two regions: the squared-basis path's stored vectors (sqb bytes) or the
    // Newton-form path's n x ldg blocks for L, R, lambdas, checkpoints and a
    // segment (fwdb bytes at stride `stride`); the region is the larger one.
    BlkMat FX, Gm, T1;
    size_t grad64 = 0;
    size_t ghalf = 0;          // the squared sweep's half accumulator (diagonal storage)
    int H = 0, sq_stride = 0;        // squared path: forward steps ceil(m/2), checkpoint stride
    size_t sqb = 0;
    int gcols = 0, ldg = 0, nckpt = 0, stride = 0;   // Newton-form path
    size_t gblk = 0, fwdb = 0;
    size_t longb = 0;          // long-row list
};

// Vectors each gradient path keeps (checkpoints every `s` steps plus the
// buffers a segment is recomputed into) and their bytes.
//  Squared path: the sketch's Horner vectors r_t (t = 1..m; checkpoints at
//  multiples of s and at m) and the forward vectors u_a of [Q_b | U] (a =
//  1..H; the same rule), max(2, s-1) scratch blocks each when s > 1, two mu
//  blocks of the reverse sweep and two rbar blocks of the sketch's adjoint.
int sq_ckpts(int last, int s) { return last / s + (last % s != 0); }
size_t sq_region(const EstLayout& L, int m, int s) {
    const size_t yb = align_up(L.Y.bytes()), xb = align_up(L.X.bytes());
    const size_t scratch = s > 1 ? (size_t)std::max(2, s - 1) : 0;
    return yb * (sq_ckpts(m, s) + scratch + 2) + xb * (sq_ckpts(L.H, s) + scratch + 2);
}
//  Newton-form path: L, R, two lambdas, ceil(m/s)-1 checkpoints and a
//  segment of s-1 vectors, all n x ldg.
size_t fwd_region(const EstLayout& L, int m, int s) {
    return align_up(L.gblk) * (size_t)(4 + ((m + s - 1) / s - 1) + (s - 1));
}

// Checkpoint stride: the smallest whose stored vectors fit kCkptBudget, i.e.
// every vector when memory allows (no recomputation); else the sqrt(m)
// stride, which minimises memory.
constexpr double kCkptBudget = 64.0 * (1ull << 30);

template <typename F>
int auto_ckpt_stride(int degree, F region) {
    for (int s = 1; s <= degree; ++s) {
        if ((double)region(s) <= kCkptBudget) return s;
        if (s * s >= degree) break;   // past sqrt(m) memory only grows again
    }
    return std::max(1, (int)std::ceil(std::sqrt((double)degree)));
}

int dot_slots(int degree, int mode) {
    return mode == LD_DOT_SQUARED ? 2 * ((degree + 1) / 2) + 1 : degree + 1;
}

EstLayout layout_estimate(const ld_csr* A, int degree, int n_matvec, bool grad,
                          const ld_options& o, double stored) {
    EstLayout L{};
    const long long n = A->n;
    L.elem = A->dtype == LD_F64 ? 8 : 4;
    L.k = n_matvec / 3;
    L.kg = n_matvec - 2 * L.k;
    L.nc = L.k + L.kg;
    // the gradient keeps the sketch and [Q_b | U] as single blocks (its sweeps
    // take every column of a vector in one row group)
    const int bw1 = grad ? L.k : choose_block_width(A, L.elem, L.k, o.block_cols, stored);
    int bw23 = grad ? L.nc : choose_block_width(A, L.elem, L.nc, o.block_cols, stored);
    if (bw23 > kMaxDotBlock) {   // the column-sum kernels take at most 64 columns per launch
        const int v = 16 / (int)L.elem, nb = (bw23 + kMaxDotBlock - 1) / kMaxDotBlock;
        bw23 = ((L.nc + nb - 1) / nb + v - 1) / v * v;
        while (bw23 > kMaxDotBlock) bw23 -= v;
    }
    L.Y = make_blk(n, L.k, bw1, L.elem);
    L.Q1 = make_blk(n, L.k, bw1, L.elem);
    L.X = make_blk(n, L.nc, bw23, L.elem);
    L.yb = L.Y.bytes();
    L.q1b = L.Q1.bytes();
    L.xb = L.X.bytes();
    const int ldmax = std::max(L.Y.ld, L.X.ld);
    L.nslots = std::max(dot_slots(degree, LD_DOT_SQUARED), dot_slots(degree, LD_DOT_FORWARD));
    L.nwg_dot = step_num_wg_bound((int)n, L.X.bw, (int)L.elem);
    L.mask = (size_t)n * 8;
    L.planes = (size_t)n * 8;   // the sketch's sign words as byte planes
    L.W = (size_t)n * ldmax * L.elem;
    const int kmax = std::max(L.k, L.kg);
    const size_t cross = (size_t)cross_num_wg((int)n) * kmax * kmax * 8;
    const size_t dotp = (size_t)L.X.nblocks() * L.nslots * L.nwg_dot * L.X.bw * 8;
    L.part = std::max(cross, dotp);
    L.small = (size_t)kSmallSlots * 64 * 64 * 8;
    L.nu = (size_t)L.nslots * L.nc * 8;
    L.flag = 256;
    L.longb = long_rows_bytes(A) + dia_bytes(A, o);
    if (grad) {
        L.FX = make_blk(n, L.nc, L.nc, L.elem);             // F [Q_b | U], one row-major block
        L.Gm = make_blk(n, L.kg, L.kg, L.elem);
        L.T1 = make_blk(n, L.k, L.k, L.elem);
        L.grad64 = L.elem == 8 ? 0 : (size_t)A->nnz * 8;
        // upper-entry pair sums of the squared sweep on the diagonal storage:
        // at most (kMaxDiag + 1) / 2 slots per row
        L.ghalf = o.csr_only ? 0 : (size_t)n * ((kMaxDiag + 1) / 2) * 8;
        L.H = (degree + 1) / 2;
        L.sq_stride = o.ckpt_stride > 0 ? std::min(o.ckpt_stride, degree)
                                        : auto_ckpt_stride(degree, [&](int s) { return sq_region(L, degree, s); });
        L.sqb = sq_region(L, degree, L.sq_stride);
        L.gcols = L.nc + L.k;                               // R = [Q_b, U, S] / L = [Q_b, cU, 2Z]
        const int v = 16 / (int)L.elem;
        int lanes = 1;                                      // the adjoint's row group: power of two
        while (lanes * v < L.gcols) lanes <<= 1;
        L.ldg = lanes * v;
        L.gblk = (size_t)n * L.ldg * L.elem;
        // the Newton-form path runs when the squared coefficients are
        // ill-conditioned; it takes the smallest stride whose vectors fit the
        // region (at least its sqrt(m) minimum)
        const int smin = std::max(1, (int)std::ceil(std::sqrt((double)degree)));
        L.stride = o.ckpt_stride > 0 ? std::min(o.ckpt_stride, degree) : smin;
        const size_t region = std::max(L.sqb, fwd_region(L, degree, L.stride));
        if (o.ckpt_stride <= 0)
            for (int st = 1; st < L.stride; ++st)
                if (fwd_region(L, degree, st) <= region) {
                    L.stride = st;
                    break;
                }
        L.nckpt = (degree + L.stride - 1) / L.stride;     // segments of the reverse sweep
        L.fwdb = fwd_region(L, degree, L.stride);
    }
    return L;
}

size_t layout_bytes(const EstLayout& L, bool grad) {
    size_t b = 0;
    for (size_t s : {L.mask, L.planes, L.yb, L.q1b, L.xb, L.W, L.W, L.part, L.small, L.nu, L.flag})
        b += align_up(s);
    b += L.longb;
    if (grad) {
        for (size_t s : {L.FX.bytes(), L.Gm.bytes(), L.T1.bytes(), L.mask, L.grad64, L.ghalf}) b += align_up(s);
        b += std::max(L.sqb, L.fwdb);
    }
    return b;
}

// The workspace is laid out before the call learns how the matrix is stored
// (the diagonal probe runs on the device), while the column blocks depend on
// the stored bytes: the envelope is the CSR layout with each block region as
// large as any storage the call may pick needs, and fit_blocks sets the
// blocks once the storage is known.  The gradient's blocks are fixed (one
// block each), as are blocks the caller sets.
EstLayout layout_envelope(const ld_csr* A, int degree, int n_matvec, bool grad, const ld_options& o) {
    const size_t elem = A->dtype == LD_F64 ? 8 : 4;
    EstLayout L = layout_estimate(A, degree, n_matvec, grad, o, matrix_bytes(A, elem));
    if (grad || o.csr_only || o.block_cols > 0) return L;
    for (int nd = 1; nd <= kMaxDiag; ++nd)
        for (bool cst : {false, true}) {
            const EstLayout M = layout_estimate(A, degree, n_matvec, false, o, stored_bytes(A, elem, nd, cst));
            L.yb = std::max(L.yb, M.yb);
            L.q1b = std::max(L.q1b, M.q1b);
            L.xb = std::max(L.xb, M.xb);
            L.W = std::max(L.W, M.W);
            L.part = std::max(L.part, M.part);
        }
    return L;
}

struct Timer {
    hipEvent_t ev[8];
    int count = 0;
    hipStream_t st;
    bool on;   // false: no events are created (the entry point that allocates nothing)
    Timer(hipStream_t s, bool enabled) : st(s), on(enabled) {
        for (auto& e : ev) e = nullptr;
    }
    void mark() {
        if (on && count < 8 && hipEventCreate(&ev[count]) == hipSuccess) {
            (void)hipEventRecord(ev[count], st);
            ++count;
        }
    }
    double ms(int a, int b) const {
        float t = 0.f;
        if (a < count && b < count && hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess) return t;
        return 0.0;
    }
    ~Timer() {
        for (int i = 0; i < count; ++i) (void)hipEventDestroy(ev[i]);
    }
};

// bytes the recurrence kernels must move (FP values, int32 indices; the
// matrix once per launch, blocks as listed per step kind)
double alg_bytes_step(const ld_csr* A, int cols, int kind, size_t elem, int dia_nd = 0, bool dia_const = false,
                      int sign_bytes = 8) {
    double per = 0;
    switch (kind) {
        case STEP_HORNER_SIGNS: per = 2.0 * elem * cols + sign_bytes; break;   // + sign word or byte planes
        case STEP_HORNER_VEC: per = 3.0 * elem * cols; break;
        case STEP_DOT_FWD: per = 3.0 * elem * cols; break;
        case STEP_DOT_SQ: per = 2.0 * elem * cols; break;
        default: per = 2.0 * elem * cols; break;
    }
    return stored_bytes(A, elem, dia_nd, dia_const) + per * (double)A->n;
}

// Launch one Newton step over all columns of a row-major block, in column
// chunks of col_block (user option of ld_apply_log).
struct LongRows {
    const int* list = nullptr;    // null: the matrix has no row above kLongRow entries
    const int* count = nullptr;
    // diagonal storage of A, when every stored entry lies on one of at most
    // kMaxDiag diagonals (stencils, banded matrices); dia_nd = 0: CSR only
    const void* dia = nullptr;
    int dia_nd = 0;
    int dia_off[kMaxDiag] = {};
    // presence bits per row (bit q = the row stores diagonal q) whenever the
    // diagonal storage is used
    const uint16_t* pres_bits = nullptr;
    // every diagonal one constant: per-row presence bits and the constants
    const uint16_t* dia_pres = nullptr;
    double dia_cval[kMaxDiag] = {};
    int tile_order = LD_TILES_AUTO;   // ld_options.tile_order
    bool skewed = false;              // entries far from even over the eight row bands
};

// Chunked XCD bands for stencils (diagonal storage) whose widest diagonal
// offset D is large: chunks of D/8 rows go to the XCDs in turn, so each XCD's
// consecutive chunks lie D rows apart and the neighbour rows r - D and r + D
// of its active rows were gathered by the same XCD one chunk earlier or come
// one chunk later.  Taken when the launch streams from HBM (its bytes exceed
// the Infinity Cache) or when the three planes r - D, r, r + D of a
// contiguous band would overflow half an XCD's 4 MB L2 (a 3-D grid).
// Measured on gfx950: 128^3 grid 23.4 -> 24.5 estimates/s, 2048^2 GMRF
// 47.1 -> 47.9, 5000^2 GMRF 10.1 -> 10.8; on the cache-resident 1024^2 grid
// chunks cost a quarter of the rate, so contiguous bands stay there.
constexpr double kL2Budget = 2.0 * (1 << 20);

int xcd_chunk_rows(const LongRows& lr, int ld, size_t elem, bool streams) {
    if (lr.dia_nd <= 0) return 0;
    int D = 0;
    for (int q = 0; q < lr.dia_nd; ++q) D = std::max(D, std::abs(lr.dia_off[q]));
    if (D / kXcds < 64) return 0;
    if (!streams && 3.0 * D * (double)ld * (double)elem <= kL2Budget) return 0;
    return D / kXcds;
}

int run_step(bool f64, const ld_csr* A, StepArgs s, int ncols, int col_block, hipStream_t st,
             int* nwg_used, const LongRows& lr) {
    const CsrDev d = dev_of(A);
    s.long_rows = lr.list;
    s.long_count = lr.count;
    s.dia = lr.dia;
    s.dia_nd = lr.dia_nd;
    for (int q = 0; q < kMaxDiag; ++q) s.dia_off[q] = lr.dia_off[q];
    s.dia_pres = lr.dia_pres;
    for (int q = 0; q < kMaxDiag; ++q) s.dia_cval[q] = lr.dia_cval[q];
    // XCD bands keep a stencil's neighbour rows in the XCD's L2 (measured on
    // gfx950: 1.45x faster steps while the blocks stream from the Infinity
    // Cache, within 3% of interleaved from HBM), but give one XCD most of
    // the work when the entries crowd into a few bands (a power-law graph
    // with its hubs first: 1.5x slower); then the tiles are interleaved.
    s.interleave = lr.tile_order == LD_TILES_INTERLEAVED || (lr.tile_order == LD_TILES_AUTO && lr.skewed);
    // Once a launch streams from HBM (working set beyond the Infinity Cache),
    // the output goes out with streaming stores: L2 then keeps more of the
    // input rows that neighbouring tiles gather (measured on gfx950: -7% on a
    // 7-point stencil step over 32 columns at 128^3).  Below that size the
    // next step reads the output back from the cache, and plain stores stay.
    s.nt_out = alg_bytes_step(A, ncols, s.kind, A->dtype == LD_F64 ? 8 : 4, lr.dia_nd, lr.dia_pres != nullptr) >
               kMallBudget;
    s.chunk_rows = s.interleave ? 0 : xcd_chunk_rows(lr, s.ld, f64 ? 8 : 4, s.nt_out);
    int nwg = 0;
    const int gshift = s.gshift;
    // one row group spans at most a wave: 64 lanes of the launch's vector width
    s.c0 = 0;
    col_block = std::min(col_block, step_max_cols(f64, s));
    for (int c0 = 0; c0 < ncols; c0 += col_block) {
        s.c0 = c0;
        s.bcols = std::min(col_block, ncols - c0);
        s.gshift = gshift;
        int used = 0;
        LD_CHECK_HIP(launch_step(f64, d, s, st, &used));
        nwg = std::max(nwg, used);
    }
    if (nwg_used) *nwg_used = nwg;
    return LD_OK;
}


// Per-call matrix preparation, with one host sync for all results: the list
// of rows with more than kLongRow entries, the balance of the entries over
// the eight row bands (tile order), and diagonal storage when every stored
// entry lies on one of at most kMaxDiag diagonals (stencils, banded
// matrices).  The diagonal build takes its candidate offsets from a sample of
// rows and flags any entry off them, in which case the call keeps the CSR
// path.
int prepare_rows(const ld_csr* A, const ld_options& o, Arena& ar, hipStream_t st, LongRows& lr) {
    if (o.tile_order < LD_TILES_AUTO || o.tile_order > LD_TILES_INTERLEAVED)
        return fail(LD_EINVAL, "tile_order must be LD_TILES_AUTO, LD_TILES_XCD_BANDS or LD_TILES_INTERLEAVED");
    int* list = (int*)ar.take((size_t)A->n * 4);
    int* tmp = (int*)ar.take(((size_t)A->n / 256 + 4) * 4);
    int* count = (int*)ar.take(16);
    void* buf = o.csr_only ? nullptr : ar.take((size_t)A->n * kMaxDiag * (A->dtype == LD_F64 ? 8 : 4));
    uint16_t* pres = o.csr_only ? nullptr : (uint16_t*)ar.take((size_t)A->n * 2);
    int* info = (int*)ar.take(256);
    const bool probe = A->n >= 3 && A->nnz > 0;
    const bool want_dia = buf && probe;
    int hcount = 0;
    int h[64] = {};   // the 256-byte info block
    LD_CHECK_HIP(launch_long_rows(dev_of(A), tmp, list, count, st));
    if (probe) {
        LD_CHECK_HIP(hipMemcpyAsync(info, h, sizeof(h), hipMemcpyHostToDevice, st));
        LD_CHECK_HIP(launch_rows_probe(A->dtype == LD_F64, dev_of(A), info, st));
        if (want_dia) LD_CHECK_HIP(launch_dia_build(A->dtype == LD_F64, dev_of(A), buf, pres, info, st));
        LD_CHECK_HIP(hipMemcpyAsync(h, info, sizeof(h), hipMemcpyDeviceToHost, st));
    }
    LD_CHECK_HIP(hipMemcpyAsync(&hcount, count, sizeof(int), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));   // also orders the upload of h before its reuse
    lr = LongRows{};
    lr.tile_order = o.tile_order;
    if (probe) {   // skewed: some band holds more than 1.25x its share of the entries
        long long most = 0;
        for (int i = 0; i < kXcds; ++i) most = std::max(most, (long long)h[kBandInfo + i + 1] - h[kBandInfo + i]);
        lr.skewed = (double)most * kXcds > 1.25 * (double)A->nnz;
    }
    if (hcount > 0) {
        lr.list = list;
        lr.count = count;
    }
    const int nd = h[0];
    if (want_dia && nd >= 1 && nd <= kMaxDiag && !h[12]) {
        lr.dia = buf;
        lr.dia_nd = nd;
        lr.pres_bits = pres;
        for (int q = 0; q < kMaxDiag; ++q) lr.dia_off[q] = q < nd ? h[1 + q] : 0;
        if (!h[kConstFlag] && !o.csr_only) {   // every diagonal holds one value
            lr.dia_pres = pres;
            std::memcpy(lr.dia_cval, h + kConstInfo, sizeof(double) * nd);
        }
    }
    return LD_OK;
}

// Gram / cross product X^T Z reduced to a kx x kz FP64 matrix on the device.
int cross_product(bool f64, int n, const void* X, Blk bx, int kx, const void* Z, Blk bz, int kz,
                  const uint64_t* zmask, double* part, double* out, hipStream_t st) {
    LD_CHECK_HIP(launch_cross(f64, n, X, bx, kx, Z, bz, kz, zmask, part, st));
    LD_CHECK_HIP(launch_reduce(part, cross_num_wg(n), kx * kz, kx * kz, 1, 0, out, kx * kz, st));
    return LD_OK;
}

// One CholQR pass: R from the Gram of Y (factored on the device, breakdown
// code in *dflag, read with the results), then Q = Y R^{-1} (into Q, global
// columns [0, k)).
int cholqr_pass(bool f64, int n, const BlkMat& Y, int k, const BlkMat& Q, double* part, double* dG,
                double* dR, double* dRinv, int* dflag, hipStream_t st) {
    LD_CHECK(cross_product(f64, n, Y.base, Y.desc(), k, Y.base, Y.desc(), k, nullptr, part, dG, st));
    LD_CHECK_HIP(launch_chol_factor(dG, k, dR, dRinv, dflag, st));
    LD_CHECK_HIP(launch_rowmat(f64, n, Y.base, Y.desc(), k, dRinv, k, 1.0, nullptr, nullptr,
                               Blk::plain(1), Q.base, Q.desc(), st));
    return LD_OK;
}

struct EstimateState {
    Plan plan;
    EstLayout L;
    int mode;                       // LD_DOT_FORWARD / LD_DOT_SQUARED
    int probe = LD_PROBE_RADEMACHER;   // distribution of the entries of S and G
    uint64_t key0 = 0;                 // stream key of S
    std::vector<double> coef;       // d (forward) or c (squared)
    void *mask, *W0, *W1;
    double *part, *small, *nu;
    int* flag;
    int spmm_launches = 0;
    double bytes_alg = 0;
    int launches1 = 0, launches23 = 0;
    int ranges23 = 1;               // row-range launches per quadratic-form step
    uint8_t* planes = nullptr;      // S's sign words as byte planes (the sketch's flat steps)
    double bytes1 = 0, bytes23 = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // step-phase brackets
    bool timed = true;              // false: no HIP events (ld_logdet_estimate_noalloc)
    LongRows longrows;
    ~EstimateState() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Breakdown codes the two CholQR factorisations left in flag[1], flag[2].
int cholqr_status(const int* h) {
    for (int i = 0; i < 2; ++i) {
        if (h[i] == 1) return fail(LD_EBREAKDOWN, "non-finite Gram entry in CholQR");
        if (h[i] != 0)
            return fail(LD_EBREAKDOWN, "CholQR Gram matrix is not positive definite (rank-deficient sketch)");
    }
    return LD_OK;
}

int record(EstimateState& S, int i, hipStream_t st) {
    if (!S.timed) return LD_OK;
    if (!S.ev[i]) LD_CHECK_HIP(hipEventCreate(&S.ev[i]));
    LD_CHECK_HIP(hipEventRecord(S.ev[i], st));
    return LD_OK;
}

double elapsed(const EstimateState& S, int a, int b) {
    float t = 0.f;
    if (S.ev[a] && S.ev[b] && hipEventElapsedTime(&t, S.ev[a], S.ev[b]) == hipSuccess) return t;
    return 0.0;
}

int choose_dot_mode(const Plan& p, int requested, std::vector<double>& coef) {
    if (requested == LD_DOT_FORWARD) {
        coef = p.d;
        return LD_DOT_FORWARD;
    }
    std::vector<double> c;
    squared_basis(p.xi, p.d, c);
    if (requested == LD_DOT_AUTO) {
        double sd = 0, sc = 0;
        for (double x : p.d) sd += std::fabs(x);
        for (double x : c) sc += std::fabs(x);
        if (!(sc <= 4.0 * sd)) {
            coef = p.d;
            return LD_DOT_FORWARD;
        }
    }
    coef = c;
    return LD_DOT_SQUARED;
}

// Where a recurrence keeps its vectors: vector t (1 <= t <= last) in a
// checkpoint buffer when t is a multiple of the stride s or t = last, else
// in one of two temporaries (alternating with t) or, while a segment is
// recomputed, in a scratch buffer.
struct VecStore {
    std::vector<void*> ck;        // checkpoints: slot t/s - 1 for multiples of s, then `last`
    std::vector<void*> scratch;   // max(2, s-1) buffers when s > 1
    int s = 1, last = 0;
    void* slot(int t) const {
        if (t % s == 0) return ck[t / s - 1];
        if (t == last) return ck.back();
        return nullptr;
    }
    void* tmp(int t) const { return scratch[t % 2]; }
    void* at(int t) const { return slot(t) ? slot(t) : tmp(t); }
};

int carve_store(Arena& ar, VecStore& v, int last, int s, size_t bytes) {
    v.s = s;
    v.last = last;
    for (int i = 0; i < sq_ckpts(last, s); ++i) v.ck.push_back(ar.take(bytes));
    if (s > 1)
        for (int i = 0; i < std::max(2, s - 1); ++i) v.scratch.push_back(ar.take(bytes));
    return LD_OK;
}

// Horner evaluation of Y = P_m(Q~) S, block by block; S from the sign words
// (Rademacher) or stored (Gaussian).  With `keep` (one block) the Horner
// vectors r_t = sum_{j >= t} d_j prod_{l=t}^{j-1} (T - xi_l) S, t = 1..m, go
// to its buffers (the squared gradient's adjoint of the sketch reads them).
int sketch_phase(const ld_csr* A, EstimateState& S, hipStream_t st, const VecStore* keep = nullptr) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const Plan& p = S.plan;
    const BlkMat& Y = S.L.Y;
    const int m = p.degree;
    // Gaussian S is stored (in Q1's block, free until CholQR) and read by
    // every step; Rademacher S is regenerated from its sign words
    const bool gauss = S.probe == LD_PROBE_GAUSSIAN;
    const int kind = gauss ? STEP_HORNER_VEC : STEP_HORNER_SIGNS;
    for (int b = 0; b < Y.nblocks(); ++b) {
        const int cols = Y.bcols(b), gcol = b * Y.bw;
        // a block whose columns lie in one byte of the sign words reads that byte
        // plane on the diagonal storage (the flat kernel: one contiguous byte per
        // row and wave), else the words.  Measured on gfx950, sketch step: 2048^2
        // GMRF at 4 columns 27.9 -> 25.4 us, 128^3 grid at 8: 31.1 -> 29.5 us;
        // blocks over several planes got slower (a wave then reads several short
        // runs): 1024^2 grid at 20 columns 29.0 -> 33.2 us, 5000^2 GMRF at 10:
        // 569 -> 628 us.
        const bool one_plane = (gcol >> 3) == ((gcol + cols - 1) >> 3);
        const int sign_bytes = one_plane && S.planes && S.longrows.dia_nd > 0 ? 1 : 8;
        // step j (= m-1 .. 0) writes (j even ? block : W0); r_m sits in the other one
        void* bufs[2] = {Y.block(b), S.W0};
        void* const rm = keep ? keep->at(m) : bufs[(m - 1) % 2 == 0 ? 1 : 0];
        void* const sblk = S.L.Q1.block(b);
        if (gauss) {
            LD_CHECK_HIP(launch_gauss_fill(f64, n, cols, S.key0, gcol, 1.0, sblk, Blk::plain(S.L.Q1.ld), st));
            LD_CHECK_HIP(launch_scale_copy(f64, n, cols, sblk, S.L.Q1.ld, p.d[m], rm, Y.ld, st));
        } else {
            LD_CHECK_HIP(launch_fill_signs(f64, n, cols, Y.ld, gcol, (const uint64_t*)S.mask, p.d[m], rm, st));
        }
        for (int j = m - 1; j >= 0; --j) {
            StepArgs s{};
            s.kind = kind;
            s.win = keep ? keep->at(j + 1) : bufs[j % 2 == 0 ? 1 : 0];
            s.wout = keep ? (j == 0 ? Y.block(b) : keep->at(j)) : bufs[j % 2 == 0 ? 0 : 1];
            s.ld = Y.ld;
            s.gshift = gcol;
            s.alpha = p.alpha;
            s.beta = p.beta[j];
            s.dj = p.d[j];
            s.mask = (const uint64_t*)S.mask;
            s.planes = one_plane ? S.planes : nullptr;
            s.vsrc = gauss ? sblk : nullptr;
            s.ldv = S.L.Q1.ld;
            LD_CHECK(run_step(f64, A, s, cols, cols, st, nullptr, S.longrows));
            S.launches1 += 1;
            S.bytes1 += alg_bytes_step(A, cols, kind, S.L.elem, S.longrows.dia_nd, S.longrows.dia_pres != nullptr,
                                       sign_bytes);
        }
    }
    return LD_OK;
}

int orthonormalize_and_deflate(const ld_csr* A, uint64_t seed, EstimateState& S, hipStream_t st);

// Phases 1 (sketch), CholQR2 and deflation; leaves X = [Q_b | U].
int estimate_front(const ld_csr* A, uint64_t seed, EstimateState& S, hipStream_t st, Timer& tm,
                   const VecStore* keep = nullptr) {
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const uint64_t key0 = probe_stream_key(seed, 0);
    const bool gauss = S.probe == LD_PROBE_GAUSSIAN;
    S.key0 = key0;

    if (!gauss) LD_CHECK_HIP(launch_sign_mask(n, L.k, key0, (uint64_t*)S.mask, st, S.planes));
    LD_CHECK(record(S, 0, st));
    LD_CHECK(sketch_phase(A, S, st, keep));
    LD_CHECK(record(S, 1, st));
    S.spmm_launches += S.launches1;
    S.bytes_alg += S.bytes1;
    tm.mark();
    LD_CHECK(orthonormalize_and_deflate(A, seed, S, st));
    tm.mark();
    return LD_OK;
}

// Alg. 3 steps 4 and 6: CholQR2 of the sketch Y (Q1 = Y R1^{-1}, Q_b = Q1
// R2^{-1}, into X[:, :k]) and the deflated residual probes U = G - Q_b Q_b^T G
// (into X[:, k:]); G is probe stream 1.  S's sign words are no longer needed:
// their buffer takes G's.
int orthonormalize_and_deflate(const ld_csr* A, uint64_t seed, EstimateState& S, hipStream_t st) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const uint64_t key1 = probe_stream_key(seed, 1);
    const bool gauss = S.probe == LD_PROBE_GAUSSIAN;
    // ---- CholQR2: Q1 = Y R1^{-1}, Q_b = Q1 R2^{-1} (into X[:, :k])
    double* dG = S.small;
    double* dRinv = S.small + 64 * 64;
    double* dC = S.small + 2 * 64 * 64;
    double* dR1 = S.small + (size_t)kSlotR1 * 64 * 64;
    double* dR2 = S.small + (size_t)kSlotR2 * 64 * 64;
    LD_CHECK(cholqr_pass(f64, n, L.Y, L.k, L.Q1, S.part, dG, dR1, dRinv, S.flag + 1, st));
    LD_CHECK(cholqr_pass(f64, n, L.Q1, L.k, L.X, S.part, dG, dR2, dRinv, S.flag + 2, st));
    // ---- deflation: C = Q_b^T G, U = G - Q_b C (G = probe stream 1) into X[:, k:].
    if (gauss) {   // G stored where U goes, then U = G - Q_b C in place
        const Blk ud = L.X.desc().shifted(L.k);
        LD_CHECK_HIP(launch_gauss_fill(f64, n, L.kg, key1, 0, 1.0, L.X.base, ud, st));
        LD_CHECK(cross_product(f64, n, L.X.base, L.X.desc(), L.k, L.X.base, ud, L.kg, nullptr, S.part, dC, st));
        LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, L.X.desc(), L.k, dC, L.kg, -1.0, nullptr, L.X.base, ud,
                                   L.X.base, ud, st));
    } else {   // the sketch is done with S's sign words: the buffer now takes G's
        const uint64_t* gmask = (const uint64_t*)S.mask;
        LD_CHECK_HIP(launch_sign_mask(n, L.kg, key1, (uint64_t*)S.mask, st));
        LD_CHECK(cross_product(f64, n, L.X.base, L.X.desc(), L.k, nullptr, Blk::plain(1), L.kg, gmask, S.part,
                               dC, st));
        LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, L.X.desc(), L.k, dC, L.kg, -1.0, gmask, nullptr,
                                   Blk::plain(1), L.X.base, L.X.desc().shifted(L.k), st));
    }
    return LD_OK;
}

// Quadratic forms x^T P_m(Q~) x for every column of X; nu_host[slot][col].
// With `keep` (squared basis, one block) the forward vectors u_a = pi_a(T) X,
// a = 1..H, go to its buffers (the squared gradient's reverse sweep reads them).
int estimate_dots(const ld_csr* A, EstimateState& S, hipStream_t st, std::vector<double>& nu_host,
                  const VecStore* keep = nullptr) {
    const bool f64 = A->dtype == LD_F64;
    const Plan& p = S.plan;
    const EstLayout& L = S.L;
    const BlkMat& X = L.X;
    const int m = p.degree;
    const int nslots = S.mode == LD_DOT_SQUARED ? 2 * ((m + 1) / 2) + 1 : m + 1;
    // partial sums of block b: its own region [slot][workgroup][column of the block]
    const size_t slot_stride = (size_t)L.nwg_dot * X.bw;
    LD_CHECK(record(S, 2, st));
    for (int b = 0; b < X.nblocks(); ++b) {
        const int cols = X.bcols(b), gcol = b * X.bw;
        double* const part = S.part + (size_t)b * nslots * slot_stride;
        int nwg = 0;
        if (S.mode == LD_DOT_SQUARED) {
            const int h = (m + 1) / 2;
            // X itself is read once and kept (the gradient needs it); W0/W1 ping-pong
            const void* cur = X.block(b);
            for (int a = 0; a < h; ++a) {
                void* nxt = keep ? keep->at(a + 1) : (a % 2 == 0) ? S.W0 : S.W1;
                StepArgs s{};
                s.kind = STEP_DOT_SQ;
                s.first = a == 0;
                s.win = cur;
                s.wout = nxt;
                s.ld = X.ld;
                s.alpha = p.alpha;
                s.beta = p.beta[a];
                s.ps0 = part;
                s.ps1 = part + (size_t)(2 * a + 1) * slot_stride;
                s.ps2 = part + (size_t)(2 * a + 2) * slot_stride;
                s.part_ld = X.bw;
                s.ranges_out = &S.ranges23;
                int used = 0;
                LD_CHECK(run_step(f64, A, s, cols, cols, st, &used, S.longrows));
                if (a > 0 && used != nwg) return fail(LD_EINVAL, "internal: partial rows differ between steps");
                nwg = used;
                S.launches23 += 1;
                S.bytes23 += alg_bytes_step(A, cols, STEP_DOT_SQ, L.elem, S.longrows.dia_nd, S.longrows.dia_pres != nullptr);
                cur = nxt;
            }
        } else {
            const void* cur = X.block(b);
            void* pp[2] = {S.W0, S.W1};
            for (int j = 0; j < m; ++j) {
                StepArgs s{};
                s.kind = STEP_DOT_FWD;
                s.first = j == 0;
                s.win = cur;
                s.wout = pp[j % 2];
                s.ld = X.ld;
                s.alpha = p.alpha;
                s.beta = p.beta[j];
                s.vsrc = X.block(b);
                s.ldv = X.ld;
                s.ps0 = part;
                s.ps1 = part + (size_t)(j + 1) * slot_stride;
                s.part_ld = X.bw;
                s.ranges_out = &S.ranges23;
                int used = 0;
                LD_CHECK(run_step(f64, A, s, cols, cols, st, &used, S.longrows));
                if (j > 0 && used != nwg) return fail(LD_EINVAL, "internal: partial rows differ between steps");
                nwg = used;
                S.launches23 += 1;
                S.bytes23 += alg_bytes_step(A, cols, STEP_DOT_FWD, L.elem, S.longrows.dia_nd, S.longrows.dia_pres != nullptr);
                cur = pp[j % 2];
            }
        }
        if (nwg > L.nwg_dot) return fail(LD_EINVAL, "internal: dot partials overflow");
        LD_CHECK_HIP(launch_reduce(part, nwg, cols, X.bw, nslots, (long long)slot_stride, S.nu + gcol,
                                   L.nc, st));
    }
    LD_CHECK(record(S, 3, st));
    S.spmm_launches += S.launches23;
    S.bytes_alg += S.bytes23;
    nu_host.assign((size_t)nslots * L.nc, 0.0);
    int hflag[2] = {0, 0};
    LD_CHECK_HIP(hipMemcpyAsync(nu_host.data(), S.nu, sizeof(double) * nu_host.size(),
                                hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipMemcpyAsync(hflag, S.flag + 1, sizeof(hflag), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    return cholqr_status(hflag);
}

int carve(Arena& ar, EstLayout& L, EstimateState& S) {
    S.mask = ar.take(L.mask);
    S.planes = (uint8_t*)ar.take(L.planes);
    L.Y.base = ar.take(L.yb);
    L.Q1.base = ar.take(L.q1b);
    L.X.base = ar.take(L.xb);
    S.W0 = ar.take(L.W);
    S.W1 = ar.take(L.W);
    S.part = (double*)ar.take(L.part);
    S.small = (double*)ar.take(L.small);
    S.nu = (double*)ar.take(L.nu);
    S.flag = (int*)ar.take(L.flag);
    return LD_OK;
}

// The column blocks for the storage prepare_rows picked, inside the regions
// of the envelope the workspace was carved with.
int fit_blocks(const ld_csr* A, int degree, int n_matvec, const ld_options& o, const LongRows& lr, EstLayout& L) {
    if (o.csr_only || o.block_cols > 0 || lr.dia_nd <= 0) return LD_OK;   // the envelope's own blocks
    const EstLayout M =
        layout_estimate(A, degree, n_matvec, false, o, stored_bytes(A, L.elem, lr.dia_nd, lr.dia_pres != nullptr));
    if (M.yb > L.yb || M.q1b > L.q1b || M.xb > L.xb || M.W > L.W || M.part > L.part)
        return fail(LD_EINVAL, "internal: column blocks outgrow the workspace");
    const auto refit = [](BlkMat& dst, const BlkMat& src) {
        void* const base = dst.base;
        dst = src;
        dst.base = base;
    };
    refit(L.Y, M.Y);
    refit(L.Q1, M.Q1);
    refit(L.X, M.X);
    L.nwg_dot = M.nwg_dot;
    return LD_OK;
}

int check_estimate_args(const ld_csr* A, double lmin, double lmax, int degree, int n_matvec) {
    LD_CHECK(check_csr_args(A));
    if (!(lmin > 0.0) || !(lmax > lmin) || !std::isfinite(lmax))
        return fail(LD_EINVAL, "need 0 < lmin < lmax");
    if (degree < 1) return fail(LD_EINVAL, "degree must be >= 1");
    if (n_matvec < 3) return fail(LD_EINVAL, "n_matvec must be >= 3");
    const int k = n_matvec / 3, kg = n_matvec - 2 * k;
    if (k > 64 || kg > 64) return fail(LD_EINVAL, "n_matvec must be <= 192 (k, k_G <= 64)");
    if (k > A->n) return fail(LD_EINVAL, "sketch width k = n_matvec/3 exceeds n");
    return LD_OK;
}


// ---------------------------------------------------------------------------
// Estimate and gradient.  With F = P_m(Q~), c = 1/k_G, Y = F S = Q_b R,
// U = (I - Q_b Q_b^T) G, the derivative of
//     est = n log sigma + tr(Q_b^T F Q_b) + c tr(U^T F U)
// at fixed probes and interval is
//     d est = tr(Q_b^T dF Q_b) + c tr(U^T dF U) + 2 tr(Z^T dF S),
//     Z = (I - Q_b Q_b^T) X Q_b R^{-T},  X = F - c (F U G^T + G U^T F),
// (the basis term comes from differentiating the QR factor of the sketch).
// The derivative w.r.t. a stored entry (r, c) is computed (FP64 accumulator)
// by one of two paths:
//
// Squared basis (the estimate's own quadratic forms, LD_DOT_SQUARED): the
// quadratic forms are x^T F x = sum_a c_2a <u_a, u_a> + c_2a+1 <u_a, u_a+1>,
// u_a = pi_a(T) x, a <= H = ceil(m/2).  Their derivative (for a symmetric
// perturbation; the per-entry derivative of a quadratic form is symmetric in
// (r, c), so the mean of the two mirrored entries is exact) comes from one
// reverse sweep over [Q_b | U]:
//     mu~_H = 2 c_2H u_H,
//     mu~_i = 2 c_2i u_i + 2 c_2i+1 u_i+1 + (T - xi_i) mu~_i+1,
//     grad[(r,c)] += alpha wgt sum_cols (mu~_i+1[r] + c_2i+1 u_i[r]) u_i[c],
// whose end mu~_0 = 2 F [Q_b | U] gives Z.  The basis term is the adjoint of
// the sketch's Horner evaluation r_t = (T - xi_t) r_t+1 + d_t S (Y = r_0):
//     rbar_0 = 2Z, rbar_j+1 = (T - xi_j) rbar_j,
//     grad[(r,c)] += alpha sum_cols rbar_j[r] r_j+1[c]   (per entry, as is).
// Sweeps of H + m steps, against m forward plus m reverse steps over
// [Q_b, U, S] in the Newton form.
//
// Newton form (when the squared coefficients are ill-conditioned): one reverse
// sweep on L = [Q_b, c U, 2Z] and R = [Q_b, U, S]:
// grad[(r,c)] = alpha * sum_i <lam_{i+1}[r], w_i[c]>, with w_i the forward
// Newton vectors of R and lam the Horner adjoint started at lam_m = d_m L.
// One forward pass over R produces the w_i (stored every `stride` steps, all
// of them when memory allows) and, accumulated on the way (Alg. 2's sum),
// F [Q_b | U]: that gives both the two traces of the estimate and the
// k-column algebra of Z, so no separate quadratic-form pass is needed.
// ---------------------------------------------------------------------------
struct GradBufs {
    void* mask2 = nullptr;
    double* grad64 = nullptr;          // FP64 accumulator (the output itself for an FP64 matrix)
    double* ghalf = nullptr;           // squared sweep's upper-entry pair sums (diagonal storage)
    // Newton-form path
    void *Lg = nullptr, *Rg = nullptr, *lam0 = nullptr, *lam1 = nullptr;
    std::vector<void*> ckpt, seg;
    // squared path
    VecStore rs, us;                   // sketch Horner vectors r_t, forward vectors u_a
    void *mu[2] = {nullptr, nullptr}, *rb[2] = {nullptr, nullptr};
};

int upload(const std::vector<double>& h, double* d, hipStream_t st) {
    LD_CHECK_HIP(hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));   // h may die at return
    return LD_OK;
}

int download(const double* d, std::vector<double>& h, hipStream_t st) {
    LD_CHECK_HIP(hipMemcpyAsync(h.data(), d, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    return LD_OK;
}

std::vector<double> diag_matrix(int q, double v) {
    std::vector<double> M((size_t)q * q, 0.0);
    for (int i = 0; i < q; ++i) M[(size_t)i * q + i] = v;
    return M;
}

// The basis term's left factor: writes 2Z (k columns) into `dst`/`dd`, from
// fx = s F [Q_b | U] (layout of L.FX; s = 1 or 2, zscale = 2/s: the algebra
// is linear in fx).  Slot 2 holds C = Q_b^T G from the deflation.
int basis_term(const ld_csr* A, uint64_t seed, EstimateState& S, GradBufs& B, const void* fx, double zscale,
               void* dst, Blk dd, hipStream_t st) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const int k = L.k, kg = L.kg;
    const double c = 1.0 / kg;
    const uint64_t key1 = probe_stream_key(seed, 1);
    double* slot[kSmallSlots];
    for (int i = 0; i < kSmallSlots; ++i) slot[i] = S.small + (size_t)i * 64 * 64;
    const Blk X = L.X.desc(), FXd = L.FX.desc(), Gd = L.Gm.desc(), Td = L.T1.desc();
    // the CholQR factors: Y = Q_b R2 R1
    std::vector<double> R1((size_t)k * k), R2((size_t)k * k);
    LD_CHECK(download(slot[kSlotR1], R1, st));
    LD_CHECK(download(slot[kSlotR2], R2, st));
    // small matrices C = Q_b^T G (slot 2, from the deflation), M1 = U^T F Q_b
    if (S.probe == LD_PROBE_GAUSSIAN) {
        LD_CHECK_HIP(launch_gauss_fill(f64, n, kg, key1, 0, 1.0, L.Gm.base, Gd, st));
    } else {
        LD_CHECK_HIP(launch_sign_mask(n, kg, key1, (uint64_t*)B.mask2, st));
        LD_CHECK_HIP(launch_fill_signs(f64, n, kg, L.Gm.ld, 0, (const uint64_t*)B.mask2, 1.0, L.Gm.base, st));
    }
    std::vector<double> C((size_t)k * kg), Ct((size_t)kg * k);
    LD_CHECK(download(slot[2], C, st));
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < kg; ++j) Ct[(size_t)j * k + i] = C[(size_t)i * kg + j];
    LD_CHECK(upload(Ct, slot[3], st));
    LD_CHECK(cross_product(f64, n, L.X.base, X.shifted(k), kg, fx, FXd, k, nullptr, S.part, slot[4], st));
    // T1 = F Q_b - c F U C^T ; then T1 -= c G M1  (= X Q_b of the derivation)
    LD_CHECK_HIP(launch_rowmat(f64, n, fx, FXd.shifted(k), kg, slot[3], k, -c, nullptr, fx, FXd, L.T1.base, Td,
                               st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.Gm.base, Gd, kg, slot[4], k, -c, nullptr, L.T1.base, Td,
                               L.T1.base, Td, st));
    // P = T1 - Q_b (Q_b^T T1)
    LD_CHECK(cross_product(f64, n, L.X.base, X, k, L.T1.base, Td, k, nullptr, S.part, slot[5], st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, X, k, slot[5], k, -1.0, nullptr, L.T1.base, Td,
                               L.T1.base, Td, st));
    // Z = P R^{-T}, R = R2 R1 (upper triangular)
    std::vector<double> R((size_t)k * k, 0.0), Rinv((size_t)k * k, 0.0), RinvT((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double v = 0.0;
            for (int t = 0; t < k; ++t) v += R2[(size_t)i * k + t] * R1[(size_t)t * k + j];
            R[(size_t)i * k + j] = v;
        }
    for (int j = k - 1; j >= 0; --j) {   // inverse of the upper-triangular R by back substitution
        Rinv[(size_t)j * k + j] = 1.0 / R[(size_t)j * k + j];
        for (int i = j + 1; i < k; ++i) {
            double v = 0.0;
            for (int t = j + 1; t <= i; ++t) v += R[(size_t)j * k + t] * Rinv[(size_t)t * k + i];
            Rinv[(size_t)j * k + i] = -v / R[(size_t)j * k + j];
        }
    }
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) RinvT[(size_t)i * k + j] = Rinv[(size_t)j * k + i];
    LD_CHECK(upload(RinvT, slot[6], st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.T1.base, Td, k, slot[6], k, zscale, nullptr, nullptr, Blk::plain(1), dst,
                               dd, st));
    return LD_OK;
}

// The estimate's two traces from F [Q_b | U]: diag(Q_b^T F Q_b), diag(U^T F U).
int traces_from_fx(const ld_csr* A, EstimateState& S, hipStream_t st, double* t_low, double* t_res) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const int k = L.k, kg = L.kg;
    double* slot0 = S.small;
    double* slot1 = S.small + 64 * 64;
    const Blk X = L.X.desc(), FXd = L.FX.desc();
    LD_CHECK(cross_product(f64, n, L.X.base, X, k, L.FX.base, FXd, k, nullptr, S.part, slot0, st));
    LD_CHECK(cross_product(f64, n, L.X.base, X.shifted(k), kg, L.FX.base, FXd.shifted(k), kg, nullptr, S.part,
                           slot1, st));
    std::vector<double> ql((size_t)k * k), qr((size_t)kg * kg);
    LD_CHECK(download(slot0, ql, st));
    LD_CHECK(download(slot1, qr, st));
    KahanSum tl, tr;
    for (int i = 0; i < k; ++i) tl.add(ql[(size_t)i * k + i]);
    for (int i = 0; i < kg; ++i) tr.add(qr[(size_t)i * kg + i]);
    *t_low = tl.value();
    *t_res = tr.value() / kg;
    return LD_OK;
}

bool streams_from_hbm(const ld_csr* A, const EstLayout& L, int ld) {
    return matrix_bytes(A, L.elem) + 4.0 * (double)A->n * ld * L.elem > kMallBudget;
}

// Newton-form path (see above); the traces come from F [Q_b | U].
int gradient_newton_form(const ld_csr* A, uint64_t seed, EstimateState& S, GradBufs& B, hipStream_t st,
                         double* t_low, double* t_res) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const Plan& p = S.plan;
    const int m = p.degree, k = L.k, kg = L.kg, nc = L.nc;
    const double c = 1.0 / kg;
    const uint64_t key0 = probe_stream_key(seed, 0);
    double* slot[kSmallSlots];
    for (int i = 0; i < kSmallSlots; ++i) slot[i] = S.small + (size_t)i * 64 * 64;
    const Blk X = L.X.desc();
    const Blk Gb = Blk::plain(L.ldg);
    const int gcols = L.gcols, ldg = L.ldg, stride = L.stride;
    {
        int hflag[2] = {0, 0};
        LD_CHECK_HIP(hipMemcpyAsync(hflag, S.flag + 1, sizeof(hflag), hipMemcpyDeviceToHost, st));
        LD_CHECK_HIP(hipStreamSynchronize(st));
        LD_CHECK(cholqr_status(hflag));
    }

    // ---- R = [Q_b, U, S]
    LD_CHECK(upload(diag_matrix(k, 1.0), slot[7], st));
    LD_CHECK(upload(diag_matrix(kg, c), slot[8], st));
    LD_CHECK(upload(diag_matrix(kg, 1.0), slot[9], st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, X, k, slot[7], k, 1.0, nullptr, nullptr, Blk::plain(1),
                               B.Rg, Gb, st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, X.shifted(k), kg, slot[9], kg, 1.0, nullptr, nullptr,
                               Blk::plain(1), B.Rg, Gb.shifted(k), st));
    if (S.probe == LD_PROBE_GAUSSIAN) {
        LD_CHECK_HIP(launch_gauss_fill(f64, n, k, key0, 0, 1.0, (char*)B.Rg + (size_t)nc * L.elem, Blk::plain(ldg),
                                       st));
    } else {
        LD_CHECK_HIP(launch_sign_mask(n, k, key0, (uint64_t*)S.mask, st));
        LD_CHECK_HIP(launch_fill_signs(f64, n, k, ldg, 0, (const uint64_t*)S.mask, 1.0,
                                       (char*)B.Rg + (size_t)nc * L.elem, st));
    }

    // ---- forward Newton vectors of R; FX = sum_j d_j w_j[:, :nc] on the way
    LD_CHECK_HIP(launch_scale_copy(f64, n, nc, B.Rg, ldg, p.d[0], L.FX.base, L.FX.ld, st));
    auto step = [&](const void* in, void* out, int j, bool acc) -> int {
        StepArgs s{};
        s.kind = acc ? STEP_PLAIN_ACC : STEP_PLAIN;
        s.win = in;
        s.wout = out;
        s.ld = ldg;
        s.alpha = p.alpha;
        s.beta = p.beta[j];
        if (acc) {
            s.dj = p.d[j + 1];
            s.acc = L.FX.base;
            s.ldacc = L.FX.ld;
            s.acc_cols = nc;
        }
        return run_step(f64, A, s, gcols, gcols, st, nullptr, S.longrows);
    };
    {
        const void* cur = B.Rg;
        void* tmp[2] = {B.lam0, B.lam1};
        for (int i = 0; i < m; ++i) {
            const int nx = i + 1;   // w_nx is written; w_m only feeds the sum
            const bool keep = nx < m && nx % stride == 0;
            void* dst = keep ? B.ckpt[nx / stride - 1] : (cur == tmp[0] ? tmp[1] : tmp[0]);
            LD_CHECK(step(cur, dst, i, true));
            cur = dst;
        }
    }
    LD_CHECK(traces_from_fx(A, S, st, t_low, t_res));
    // ---- L = [Q_b, c U, 2 Z]
    LD_CHECK(basis_term(A, seed, S, B, L.FX.base, 2.0, B.Lg, Gb.shifted(nc), st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, X, k, slot[7], k, 1.0, nullptr, nullptr, Blk::plain(1),
                               B.Lg, Gb, st));
    LD_CHECK_HIP(launch_rowmat(f64, n, L.X.base, X.shifted(k), kg, slot[8], kg, 1.0, nullptr, nullptr,
                               Blk::plain(1), B.Lg, Gb.shifted(k), st));

    // ---- reverse sweep, segment by segment (recomputing a segment's vectors
    //      from its checkpoint when not all of them are stored)
    LD_CHECK_HIP(launch_scale_copy(f64, n, gcols, B.Lg, ldg, p.d[m], B.lam0, ldg, st));
    void* lam_in = B.lam0;
    void* lam_out = B.lam1;
    const CsrDev d = dev_of(A);
    for (int sg = L.nckpt - 1; sg >= 0; --sg) {
        const int s0 = sg * stride, s1 = std::min(s0 + stride, m);
        std::vector<const void*> w(s1 - s0);
        w[0] = sg == 0 ? B.Rg : B.ckpt[sg - 1];
        for (int t = 1; t < s1 - s0; ++t) {
            LD_CHECK(step(w[t - 1], B.seg[t - 1], s0 + t - 1, false));
            w[t] = B.seg[t - 1];
        }
        for (int i = s1 - 1; i >= s0; --i) {
            AdjArgs a{};
            a.mode = ADJ_HORNER;
            a.lam_in = lam_in;
            a.lam_out = lam_out;
            a.w = w[i - s0];
            a.L = B.Lg;
            a.grad = B.grad64;
            a.ld = ldg;
            a.ncols = gcols;
            a.alpha = p.alpha;
            a.beta = p.beta[i];
            a.dj = p.d[i];
            a.first = i == m - 1;
            a.last = i == 0;
            // as the Newton steps: streaming stores once the sweep works beyond the Infinity Cache
            a.nt_out = streams_from_hbm(A, L, ldg);
            LD_CHECK_HIP(launch_adjoint(f64, d, a, st));
            std::swap(lam_in, lam_out);
        }
    }
    return LD_OK;
}

// Squared-basis path (see above).  The sketch has kept its Horner vectors and
// the quadratic-form pass its forward vectors; the traces came from that pass.
int gradient_squared(const ld_csr* A, uint64_t seed, EstimateState& S, GradBufs& B, hipStream_t st) {
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    const EstLayout& L = S.L;
    const Plan& p = S.plan;
    const int m = p.degree, k = L.k, nc = L.nc, H = L.H;
    const std::vector<double>& cf = S.coef;   // squared-basis coefficients c_0..c_m
    auto coef = [&](int i) { return i >= 0 && i <= m ? cf[i] : 0.0; };
    const CsrDev d = dev_of(A);
    const int ldX = L.X.ld, ldY = L.Y.ld;
    auto plain_step = [&](const void* in, void* out, int j, int ld, int cols) -> int {
        StepArgs s{};
        s.kind = STEP_PLAIN;
        s.win = in;
        s.wout = out;
        s.ld = ld;
        s.alpha = p.alpha;
        s.beta = p.beta[j];
        return run_step(f64, A, s, cols, cols, st, nullptr, S.longrows);
    };
    // u_a for a = 0..H: u_0 is X, the others stored or recomputed per segment
    const VecStore& us = B.us;
    const VecStore& rs = B.rs;
    // on the diagonal storage the sweeps read the diagonals (and take two of
    // the sketch's adjoint steps per gradient update), else the CSR arrays
    const LongRows& lr = S.longrows;
    AdjDia dg{};
    const bool on_dia = lr.dia_nd > 0 && lr.pres_bits;
    if (on_dia) {
        dg.nd = lr.dia_nd;
        for (int q = 0; q < kMaxDiag; ++q) {
            dg.off[q] = lr.dia_off[q];
            dg.cval[q] = lr.dia_cval[q];
        }
        dg.pres = lr.pres_bits;
        dg.dia = lr.dia;
        dg.constant = lr.dia_pres != nullptr;
    }
    // offsets symmetric about the main diagonal (a symmetric pattern): the
    // squared sweep adds each mirrored pair into one slot of the upper entry
    // (half the accumulator traffic), expanded to every entry afterwards
    bool sym = on_dia && B.ghalf;
    if (sym) {
        int q0 = -1;
        for (int q = 0; q < dg.nd; ++q)
            if (dg.off[q] == 0) q0 = q;
        sym = q0 >= 0 && 2 * q0 + 1 == dg.nd;
        for (int h = 1; sym && h <= q0; ++h) sym = dg.off[q0 + h] == -dg.off[q0 - h];
        if (sym) {
            dg.qh0 = q0;
            dg.nh = dg.nd - q0;
        }
    }
    auto sweep = [&](const AdjArgs& a) -> int {
        LD_CHECK_HIP(on_dia ? launch_adjoint_dia(f64, d, a, dg, st) : launch_adjoint(f64, d, a, st));
        return LD_OK;
    };

    // ---- reverse sweep over [Q_b | U] (weights 1 and 1/k_G), segment by segment;
    //      the first step reads mu~_H = 2 c_2H u_H as u_H scaled in the kernel
    int cur = 0;
    const int s = us.s;
    for (int q = (H - 1) / s; q >= 0; --q) {
        const int b0 = q * s, b1 = std::min(b0 + s, H);   // reverse steps i = b1-1 .. b0 need u_b0 .. u_b1-1
        std::vector<const void*> u(b1 - b0);
        u[0] = b0 == 0 ? L.X.base : us.slot(b0);
        for (int t = 1; t < b1 - b0; ++t) {
            void* dst = us.slot(b0 + t) ? us.slot(b0 + t) : us.scratch[t - 1];
            if (!us.slot(b0 + t)) LD_CHECK(plain_step(u[t - 1], dst, b0 + t - 1, ldX, nc));
            u[t] = dst;
        }
        for (int i = b1 - 1; i >= b0; --i) {
            AdjArgs a{};
            a.mode = sym ? ADJ_SQUARED_SYM : ADJ_SQUARED;
            a.lam_in = i == H - 1 ? us.at(H) : B.mu[cur];
            a.lam_scale = i == H - 1 ? 2.0 * coef(2 * H) : 1.0;
            a.lam_out = B.mu[1 - cur];
            a.w = u[i - b0];
            a.grad = sym ? B.ghalf : B.grad64;
            a.ld = ldX;
            a.ncols = nc;
            a.alpha = p.alpha;
            a.beta = p.beta[i];
            a.q0 = 2.0 * coef(2 * i);
            a.q1 = 2.0 * coef(2 * i + 1);
            a.p1 = coef(2 * i + 1);
            a.wsplit = k;
            a.whi = 1.0 / L.kg;
            a.first = i == H - 1;
            a.last = false;   // mu~_0 = 2 F [Q_b | U] is needed
            a.nt_out = streams_from_hbm(A, L, ldX);
            dg.chunk_rows = xcd_chunk_rows(lr, ldX, L.elem, a.nt_out);
            LD_CHECK(sweep(a));
            cur = 1 - cur;
        }
    }
    // the quadratic forms' per-entry derivative is symmetric: mirrored means
    // (from the pair sums of the half accumulator, or in place)
    LD_CHECK_HIP(hipMemsetAsync(S.flag + 3, 0, sizeof(int), st));
    if (sym)
        LD_CHECK_HIP(launch_expand_half(d, dg, B.ghalf, B.grad64, S.flag + 3, st));
    else
        LD_CHECK_HIP(launch_symmetrize(d, B.grad64, S.flag + 3, st));
    // ---- basis term: the adjoint of the sketch's Horner evaluation, from 2Z
    //      (computed from mu~_0 = 2 F [Q_b | U] directly)
    LD_CHECK(basis_term(A, seed, S, B, B.mu[cur], 1.0, B.rb[0], Blk::plain(ldY), st));
    if (rs.s > 1) {   // segments are recomputed from S: its sign words (or its Gaussian block) again
        const uint64_t key0 = probe_stream_key(seed, 0);
        if (S.probe == LD_PROBE_GAUSSIAN)
            LD_CHECK_HIP(launch_gauss_fill(f64, n, k, key0, 0, 1.0, L.Q1.base, Blk::plain(L.Q1.ld), st));
        else
            LD_CHECK_HIP(launch_sign_mask(n, k, key0, (uint64_t*)S.mask, st));
    }
    int rc = 0;
    const int seg = rs.s > 1 ? rs.s : m;   // every vector stored: one segment
    for (int q = 0; q * seg < m; ++q) {
        // steps j = j0 .. j1-1 read r_j+1 for j+1 in (j0, j1], recomputed
        // downwards from the checkpoint r_j1 when not stored
        const int j0 = q * seg, j1 = std::min(j0 + seg, m);
        std::vector<const void*> r(j1 - j0);   // r[t] = r_{j0+1+t}
        r[j1 - j0 - 1] = rs.slot(j1);
        for (int t = j1 - 1; t > j0; --t) {
            void* dst = rs.slot(t) ? rs.slot(t) : rs.scratch[t - j0 - 1];
            if (!rs.slot(t)) {
                StepArgs st2{};
                st2.kind = S.probe == LD_PROBE_GAUSSIAN ? STEP_HORNER_VEC : STEP_HORNER_SIGNS;
                st2.win = r[t - j0];
                st2.wout = dst;
                st2.ld = ldY;
                st2.alpha = p.alpha;
                st2.beta = p.beta[t];
                st2.dj = p.d[t];
                st2.mask = (const uint64_t*)S.mask;
                st2.vsrc = S.probe == LD_PROBE_GAUSSIAN ? L.Q1.base : nullptr;
                st2.ldv = L.Q1.ld;
                LD_CHECK(run_step(f64, A, st2, k, k, st, nullptr, S.longrows));
            }
            r[t - j0 - 1] = dst;
        }
        for (int j = j0; j < j1;) {
            AdjArgs a{};
            a.lam_in = B.rb[rc];
            a.lam_out = B.rb[1 - rc];
            a.w = r[j - j0];
            a.grad = B.grad64;
            a.ld = ldY;
            a.ncols = k;
            a.alpha = p.alpha;
            a.beta = p.beta[j];
            a.first = false;
            a.nt_out = streams_from_hbm(A, L, ldY);
            dg.chunk_rows = xcd_chunk_rows(lr, ldY, L.elem, a.nt_out);
            if (on_dia && j + 1 < j1) {
                // steps j and j+1 in one update of the gradient: the launch writes
                // rbar_j+1, a plain step then makes rbar_j+2 (if a later step needs it)
                a.mode = ADJ_PLAIN2;
                a.w2 = r[j + 1 - j0];
                a.last = j + 2 >= m;   // rbar_j+1 feeds no later step
                LD_CHECK(sweep(a));
                if (j + 2 < m) LD_CHECK(plain_step(B.rb[1 - rc], B.rb[rc], j + 1, ldY, k));
                j += 2;   // rbar_j+2 sits in B.rb[rc]
            } else {
                a.mode = ADJ_PLAIN;
                a.last = j == m - 1;
                LD_CHECK(sweep(a));
                rc = 1 - rc;
                j += 1;
            }
        }
    }
    int hsym = 0;
    LD_CHECK_HIP(hipMemcpyAsync(&hsym, S.flag + 3, sizeof(int), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    if (hsym) return fail(LD_EINVAL, "the gradient needs a symmetric sparsity pattern (an entry has no mirror)");
    return LD_OK;
}

// Estimate (and, with grad != nullptr, its gradient): the body of both entry points.
int run_logdet(const ld_csr* A, double lmin, double lmax, int degree, int n_matvec, uint64_t seed,
               const ld_options& o, void* workspace, size_t ws_bytes, hipStream_t st,
               double* out_logdet, void* grad, ld_stats* stats, bool timed = true) {
    const auto t0 = std::chrono::steady_clock::now();
    const bool want_grad = grad != nullptr;
    EstimateState S;
    S.timed = timed;
    LD_CHECK(make_plan(lmin, lmax, degree, o, S.plan));
    S.L = layout_envelope(A, degree, n_matvec, want_grad, o);
    S.mode = choose_dot_mode(S.plan, o.dot_mode, S.coef);
    if (o.probe_dist != LD_PROBE_RADEMACHER && o.probe_dist != LD_PROBE_GAUSSIAN)
        return fail(LD_EINVAL, "probe_dist must be LD_PROBE_RADEMACHER or LD_PROBE_GAUSSIAN");
    S.probe = o.probe_dist;
    OwnedWs own;
    Arena ar;
    LD_CHECK(get_workspace(workspace, ws_bytes, layout_bytes(S.L, want_grad), own, ar));
    carve(ar, S.L, S);
    GradBufs B;
    // the squared path takes [Q_b | U] as one block of at most 64 columns (one
    // column-sum launch per step); wider sketches and ill-conditioned squared
    // coefficients take the Newton form
    const bool sq_grad = want_grad && S.mode == LD_DOT_SQUARED && S.L.nc <= kMaxDotBlock;
    if (want_grad) {
        S.L.FX.base = ar.take(S.L.FX.bytes());
        S.L.Gm.base = ar.take(S.L.Gm.bytes());
        S.L.T1.base = ar.take(S.L.T1.bytes());
        B.mask2 = ar.take(S.L.mask);
        B.grad64 = S.L.grad64 ? (double*)ar.take(S.L.grad64) : (double*)grad;
        B.ghalf = S.L.ghalf ? (double*)ar.take(S.L.ghalf) : nullptr;
        // the chosen path's vectors share one region
        Arena reg{(char*)ar.take(std::max(S.L.sqb, S.L.fwdb)), std::max(S.L.sqb, S.L.fwdb), 0};
        if (sq_grad) {
            carve_store(reg, B.rs, degree, S.L.sq_stride, S.L.Y.bytes());
            carve_store(reg, B.us, S.L.H, S.L.sq_stride, S.L.X.bytes());
            for (void*& b : B.mu) b = reg.take(S.L.X.bytes());
            for (void*& b : B.rb) b = reg.take(S.L.Y.bytes());
        } else {
            B.Lg = reg.take(S.L.gblk);
            B.Rg = reg.take(S.L.gblk);
            B.lam0 = reg.take(S.L.gblk);
            B.lam1 = reg.take(S.L.gblk);
            for (int i = 0; i < S.L.nckpt - 1; ++i) B.ckpt.push_back(reg.take(S.L.gblk));
            for (int i = 0; i < S.L.stride - 1; ++i) B.seg.push_back(reg.take(S.L.gblk));
        }
        if (reg.used > reg.size) return fail(LD_EINVAL, "internal: gradient region overflow");
    }
    if (ar.base && ar.used > layout_bytes(S.L, want_grad))
        return fail(LD_EINVAL, "internal: workspace layout overflow");
    if (!o.trusted_csr) LD_CHECK(validate_csr(A, S.flag, st));
    LD_CHECK(prepare_rows(A, o, ar, st, S.longrows));
    if (!want_grad) LD_CHECK(fit_blocks(A, degree, n_matvec, o, S.longrows, S.L));
    Timer tm(st, timed);
    tm.mark();
    LD_CHECK(estimate_front(A, seed, S, st, tm, sq_grad ? &B.rs : nullptr));
    const EstLayout& L = S.L;
    double t_low = 0.0, t_res = 0.0;
    if (!want_grad || sq_grad) {
        std::vector<double> nu;
        LD_CHECK(estimate_dots(A, S, st, nu, sq_grad ? &B.us : nullptr));
        tm.mark();
        const int ncoef = S.plan.degree + 1;
        KahanSum tl, tr;
        for (int col = 0; col < L.nc; ++col)
            for (int i = 0; i < ncoef; ++i) {
                const double v = S.coef[i] * nu[(size_t)i * L.nc + col];
                if (col < L.k)
                    tl.add(v);
                else
                    tr.add(v);
            }
        t_low = tl.value();
        t_res = tr.value() / L.kg;
        if (sq_grad) {
            LD_CHECK(gradient_squared(A, seed, S, B, st));
            tm.mark();
        }
    } else {
        tm.mark();   // no separate quadratic-form pass
        LD_CHECK(gradient_newton_form(A, seed, S, B, st, &t_low, &t_res));
        tm.mark();
    }
    if (want_grad && S.L.grad64)   // FP32 matrix: the FP64 accumulator rounded once
        LD_CHECK_HIP(launch_narrow(A->nnz, B.grad64, (float*)grad, st));
    // ---- combine (Alg. 3 step 7): n log(sigma) + t_low + t_res
    KahanSum tot;
    tot.add((double)A->n * std::log(S.plan.sigma));
    tot.add(t_low);
    tot.add(t_res);
    *out_logdet = tot.value();
    LD_CHECK_HIP(hipStreamSynchronize(st));
    // statistics: to the caller, and one line on stderr when LD_PROFILE is set
    const char* prof = std::getenv("LD_PROFILE");
    const bool print = prof && prof[0] && std::strcmp(prof, "0") != 0;
    if (stats || print) {
        ld_stats local;
        ld_stats* const out = stats ? stats : &local;
        std::memset(out, 0, sizeof(*out));
        out->ms_phase1 = tm.ms(0, 1);
        out->ms_qr = tm.ms(1, 2);
        out->ms_phase23 = tm.ms(2, 3);
        out->ms_adjoint = want_grad ? tm.ms(3, 4) : 0.0;
        out->bytes_alg = S.bytes_alg;
        out->taylor_terms = S.plan.taylor_terms;
        out->sigma = S.plan.sigma;
        out->lo = S.plan.lo;
        out->hi = S.plan.hi;
        out->k = L.k;
        out->k_G = L.kg;
        out->dot_mode_used = S.mode;
        out->dia_diagonals = S.longrows.dia_nd;
        out->dia_constant = S.longrows.dia_pres != nullptr;
        out->tile_order_used = S.longrows.tile_order == LD_TILES_INTERLEAVED ||
                                         (S.longrows.tile_order == LD_TILES_AUTO && S.longrows.skewed)
                                     ? LD_TILES_INTERLEAVED
                                     : LD_TILES_XCD_BANDS;
        // the chunk rows the quadratic-form launches take (chunks of whole tiles only)
        const int crows =
            out->tile_order_used == LD_TILES_XCD_BANDS
                ? xcd_chunk_rows(S.longrows, L.X.ld, L.elem,
                                 alg_bytes_step(A, L.X.bw, S.mode == LD_DOT_SQUARED ? STEP_DOT_SQ : STEP_DOT_FWD,
                                                L.elem, S.longrows.dia_nd, S.longrows.dia_pres != nullptr) >
                                     kMallBudget)
                : 0;
        out->xcd_chunk_rows = crows > 0 && crows % step_tile_rows(L.X.bw, (int)L.elem) == 0 ? crows : 0;
        out->block_cols1 = L.Y.bw;
        out->block_cols23 = L.X.bw;
        out->ranges23 = S.ranges23;
        out->spmm_launches = S.spmm_launches;
        out->t_low = t_low;
        out->t_res = t_res;
        out->ms_steps1 = elapsed(S, 0, 1);
        out->ms_steps23 = elapsed(S, 2, 3);
        out->launches1 = S.launches1;
        out->launches23 = S.launches23;
        out->bytes1 = S.bytes1;
        out->bytes23 = S.bytes23;
        out->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (print)
            std::fprintf(stderr,
                         "ld_profile: %s n=%lld degree=%d m_vec=%d | sketch %.3f ms, CholQR+deflation %.3f ms, "
                         "quadratic forms %.3f ms, gradient %.3f ms, call %.3f ms | steps %d+%d, %.1f GB/s "
                         "(algorithmic) | storage %s%s, tiles %s\n",
                         want_grad ? "estimate+gradient" : "estimate", (long long)A->n, degree, n_matvec,
                         out->ms_phase1, out->ms_qr, out->ms_phase23, out->ms_adjoint, out->ms_total,
                         out->launches1, out->launches23,
                         (out->bytes1 + out->bytes23) / ((out->ms_steps1 + out->ms_steps23) * 1e-3 + 1e-30) / 1e9,
                         out->dia_diagonals ? "diagonal" : "csr", out->dia_constant ? " (constant values)" : "",
                         out->tile_order_used == LD_TILES_INTERLEAVED ? "interleaved"
                         : out->xcd_chunk_rows                          ? "xcd-chunks"
                                                                        : "xcd-bands");
    }
    return LD_OK;
}

}  // namespace
}  // namespace ld

using namespace ld;

// ---------------------------------------------------------------------------
// Scratch of ld_logdet_estimate_noalloc, for callers that cannot allocate
// device memory: a file-scope device array of the library (each GPU the
// library runs on holds its own copy, until the process ends).  Host code
// never passes `scratch` itself to a kernel (in host code the name is only a
// stand-in): its device address is looked up once per device with
// hipGetSymbolAddress and that address is used everywhere.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made on that device, with it current).
int scratch_address(void** out) {
    int dev = -1;
    LD_CHECK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(LD_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return LD_OK;
}
}  // namespace

// ---------------------------------------------------------------------------
// Lanczos refinement of the upper end of the spectrum (App. A): `steps`
// steps of the symmetric Lanczos recurrence in FP64 (an FP32 matrix's values
// are widened once) from the unit Rademacher vector of generator stream 2
// (seed 0), no reorthogonalisation; the largest Ritz
// value theta of the tridiagonal projection plus its residual norm
// beta_k |s_k| (s the Ritz vector in the Krylov basis) and a rounding margin.
// The Ritz value alone underestimates lambda_max; the residual term is the
// usual practical upper bound, not a guaranteed one, which is why the caller
// caps it by Gershgorin's.  Allocates its own vectors.
// ---------------------------------------------------------------------------
constexpr int kMaxLanczos = 512;

int lanczos_upper(const ld_csr* A_in, int steps, double abs_bound, hipStream_t st, double* out) {
    const bool f64 = true;
    const long long n = A_in->n;
    const size_t elem = 8;
    const size_t vb = align_up((size_t)n * elem);
    const size_t pb = align_up((size_t)cross_num_wg((int)n) * sizeof(double));
    const size_t wb = A_in->dtype == LD_F64 ? 0 : align_up((size_t)A_in->nnz * 8);
    OwnedWs own;
    if (hipMalloc(&own.p, 3 * vb + align_up((size_t)n * 8) + pb + 256 + wb) != hipSuccess)
        return fail(LD_ENOMEM, "hipMalloc failed");
    char* base = (char*)own.p;
    ld_csr A64 = *A_in;
    if (wb) {
        double* v64 = (double*)(base + 3 * vb + align_up((size_t)n * 8) + pb + 256);
        LD_CHECK_HIP(launch_widen(A_in->nnz, (const float*)A_in->val, v64, st));
        A64.val = v64;
        A64.dtype = LD_F64;
    }
    const ld_csr* A = &A64;
    void* vec[3] = {base, base + vb, base + 2 * vb};     // v_{j-1}, v_j, w
    uint64_t* mask = (uint64_t*)(base + 3 * vb);
    double* part = (double*)(base + 3 * vb + align_up((size_t)n * 8));
    double* scal = (double*)((char*)part + pb);
    const Blk one = Blk::plain(1);
    LD_CHECK_HIP(launch_sign_mask((int)n, 1, probe_stream_key(0, 2), mask, st));
    LD_CHECK_HIP(launch_fill_signs(f64, (int)n, 1, 1, 0, mask, 1.0 / std::sqrt((double)n), vec[1], st));
    const int k_max = (int)std::min<long long>(steps, n);
    std::vector<double> a, b;   // diagonal, off-diagonal of the projection
    double beta = 0.0;
    auto dot = [&](const void* x, const void* y, double* r) -> int {
        LD_CHECK(cross_product(f64, (int)n, x, one, 1, y, one, 1, nullptr, part, scal, st));
        LD_CHECK_HIP(hipMemcpyAsync(r, scal, sizeof(double), hipMemcpyDeviceToHost, st));
        LD_CHECK_HIP(hipStreamSynchronize(st));
        return LD_OK;
    };
    for (int j = 0; j < k_max; ++j) {
        StepArgs s{};
        s.kind = STEP_PLAIN;
        s.win = vec[1];
        s.wout = vec[2];
        s.ld = 1;
        s.alpha = 1.0;
        s.beta = 0.0;
        LD_CHECK(run_step(f64, A, s, 1, 1, st, nullptr, LongRows{}));      // w = A v_j
        double alpha = 0.0;
        LD_CHECK(dot(vec[1], vec[2], &alpha));
        LD_CHECK_HIP(launch_axpby(f64, n, -alpha, vec[1], 1.0, vec[2], st));
        if (j > 0) LD_CHECK_HIP(launch_axpby(f64, n, -beta, vec[0], 1.0, vec[2], st));
        a.push_back(alpha);
        double bb = 0.0;
        LD_CHECK(dot(vec[2], vec[2], &bb));
        beta = std::sqrt(std::fmax(bb, 0.0));
        if (!std::isfinite(alpha) || !std::isfinite(beta))
            return fail(LD_EINVAL, "non-finite value in the Lanczos recurrence (non-finite entries of A?)");
        if (j + 1 == k_max || beta <= 1e-14 * std::fmax(std::fabs(alpha), abs_bound)) break;   // done / invariant subspace
        b.push_back(beta);
        // v_{j+1} = w / beta into the buffer of v_{j-1}; then rotate
        LD_CHECK_HIP(launch_scale_copy(f64, (int)n, 1, vec[2], 1, 1.0 / beta, vec[0], 1, st));
        std::swap(vec[0], vec[1]);   // vec[1] = v_{j+1}, vec[0] = v_j
    }
    double theta = 0.0, last = 0.0;
    tridiag_top_eigenpair(a, b, &theta, &last);
    *out = theta + beta * std::fabs(last) + 8.0 * 0x1p-53 * abs_bound * std::sqrt((double)a.size());
    LD_CHECK_HIP(hipStreamSynchronize(st));
    return LD_OK;
}

// Workspace of the adaptive apply: two n x ncols blocks, step partials for
// 64 columns, Gram partials, small sums, the mask, degrees, flag, long rows.
constexpr int kAdaptPoll = 8;   // steps between host checks of the active mask (after the first few)

size_t adaptive_ws_bytes(const ld_csr* A, int ncols, const ld_options& o) {
    const size_t elem = A->dtype == LD_F64 ? 8 : 4;
    const int n = (int)A->n;
    return 2 * align_up((size_t)n * ncols * elem) +
           align_up((size_t)step_num_wg_any(n) * 64 * 8) +
           align_up((size_t)cross_num_wg(n) * 64 * 64 * 8) + align_up(64 * 64 * 8) + align_up(256) +
           align_up((size_t)ncols * 4) + align_up(256) + long_rows_bytes(A) + dia_bytes(A, o);
}

// Buffers of Alg. 2's adaptive loop: two n x ld temporaries (ld of the
// input), step partials (step_num_wg_any(n) x 64 doubles), Gram partials
// (cross_num_wg(n) x 64 x 64 doubles), 64 x 64 sums, the active mask, degrees.
struct AdaptBufs {
    void* W[2] = {nullptr, nullptr};
    double *part = nullptr, *gpart = nullptr, *sums = nullptr;
    uint64_t* mask = nullptr;
    int* deg = nullptr;
};

// Alg. 2 with each column's own stopping rule on the n x nc block V (leading
// dimension ld) into P (leading dimension ldp): column c starts with w_0 = v,
// P = (d_0 + shift) v and, while |d_m| ||w_m||_2 > tol and m < p.degree, takes
// w_{m+1} = (T - xi_m) w_m, m += 1, P += d_m w_m.  hdeg[c] = the m it stopped
// at.  Chunks of 64 columns; the host polls the active mask before the first
// step, after steps 1, 2, 4 and then every kAdaptPoll steps, and stops a
// chunk once no column is active.  `launches` counts the Newton steps.
int adaptive_apply(const ld_csr* A, const Plan& p, double tol, double shift, const void* V, int ld, int nc,
                   void* P, int ldp, const AdaptBufs& b, const LongRows& lr, hipStream_t st,
                   std::vector<int>& hdeg, int* launches) {
    const bool f64 = A->dtype == LD_F64;
    const size_t elem = f64 ? 8 : 4;
    const int n = (int)A->n;
    const int nwg_max = step_num_wg_any(n);
    const int m = p.degree;
    const std::vector<int> deg0((size_t)nc, m);   // columns that never meet tol stop at the cap
    LD_CHECK_HIP(hipMemcpyAsync(b.deg, deg0.data(), (size_t)nc * 4, hipMemcpyHostToDevice, st));
    const uint64_t all = ~0ull;
    const uint8_t* v8 = (const uint8_t*)V;
    uint8_t* p8 = (uint8_t*)P;
    for (int q0 = 0; q0 < nc; q0 += 64) {
        const int qc = std::min(64, nc - q0);
        const uint8_t* Vq = v8 + (size_t)q0 * elem;
        uint8_t* Pq = p8 + (size_t)q0 * elem;
        // P_0 = (d_0 + shift) w_0, w_0 = v
        LD_CHECK_HIP(launch_scale_copy(f64, n, qc, Vq, ld, p.d[0] + shift, Pq, ldp, st));
        // e_0 = |d_0| ||v||: the diagonal of the chunk's Gram matrix
        LD_CHECK(cross_product(f64, n, Vq, Blk::plain(ld), qc, Vq, Blk::plain(ld), qc, nullptr, b.gpart, b.sums,
                               st));
        LD_CHECK_HIP(hipMemcpyAsync(b.mask, &all, 8, hipMemcpyHostToDevice, st));
        LD_CHECK_HIP(launch_adapt_decide(b.sums, qc + 1, qc, std::fabs(p.d[0]), tol, 0, b.mask, b.deg + q0, st));
        {   // columns that stop at degree 0 need no product at all
            uint64_t h = 0;
            LD_CHECK_HIP(hipMemcpyAsync(&h, b.mask, 8, hipMemcpyDeviceToHost, st));
            LD_CHECK_HIP(hipStreamSynchronize(st));
            if (h == 0) continue;
        }
        const uint8_t* cur = Vq;
        for (int j = 0; j < m; ++j) {
            uint8_t* out = (uint8_t*)b.W[j % 2] + (size_t)q0 * elem;
            StepArgs s{};
            s.kind = STEP_ACC_NORM;
            s.win = cur;
            s.wout = out;
            s.ld = ld;
            s.alpha = p.alpha;
            s.beta = p.beta[j];
            s.dj = p.d[j + 1];
            s.acc = Pq;
            s.ldacc = ldp;
            s.acc_cols = qc;
            s.active = b.mask;
            s.ps1 = b.part;
            s.part_ld = 64;
            int nwg = 0;
            LD_CHECK(run_step(f64, A, s, qc, qc, st, &nwg, lr));
            if (nwg > nwg_max) return fail(LD_EINVAL, "internal: partial sums overflow");
            if (launches) *launches += 1;
            LD_CHECK_HIP(launch_reduce(b.part, nwg, qc, 64, 1, 0, b.sums, qc, st));
            LD_CHECK_HIP(
                launch_adapt_decide(b.sums, 1, qc, std::fabs(p.d[j + 1]), tol, j + 1, b.mask, b.deg + q0, st));
            cur = out;
            const int done = j + 1;   // poll after steps 1, 2, 4, then every kAdaptPoll: stop once all columns are done
            if (done < m && (done == 1 || done == 2 || done == 4 || done % kAdaptPoll == 0)) {
                uint64_t h = 0;
                LD_CHECK_HIP(hipMemcpyAsync(&h, b.mask, 8, hipMemcpyDeviceToHost, st));
                LD_CHECK_HIP(hipStreamSynchronize(st));
                if (h == 0) break;
            }
        }
    }
    hdeg.assign((size_t)nc, 0);
    LD_CHECK_HIP(hipMemcpyAsync(hdeg.data(), b.deg, (size_t)nc * 4, hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));   // also keeps deg0 and `all` alive until their copies ran
    return LD_OK;
}

// Alg. 3 with Alg. 2's stopping rule in its three applications of log(Q~)
// (steps 3, 5, 6): the estimate's column blocks and CholQR2/deflation, the
// sketch Y = P(Q~)S and F[Q_b | U] by adaptive_apply (forward Newton form,
// each column its own degree, at most p.degree), then the quadratic forms
// x^T F x as the diagonal of block cross products.  Workspace: the
// estimate's, a copy of X's blocks for F[Q_b | U], and the adaptive buffers.
EstLayout layout_adaptive(const ld_csr* A, int max_degree, int n_matvec, const ld_options& o) {
    // blocks sized by the CSR bytes whatever the storage: the loop polls each
    // block's columns, and narrower blocks would multiply the polls
    return layout_estimate(A, max_degree, n_matvec, false, o, matrix_bytes(A, A->dtype == LD_F64 ? 8 : 4));
}

size_t adaptive_estimate_ws_bytes(const ld_csr* A, int max_degree, int n_matvec, const ld_options& o) {
    const EstLayout L = layout_adaptive(A, max_degree, n_matvec, o);
    const int n = (int)A->n;
    return layout_bytes(L, false) + align_up(L.xb) + align_up((size_t)step_num_wg_any(n) * 64 * 8) +
           align_up((size_t)cross_num_wg(n) * 64 * 64 * 8) + align_up(64 * 64 * 8) + 2 * align_up(256) + 256;
}

int run_logdet_adaptive(const ld_csr* A, double lmin, double lmax, int max_degree, double tol, int n_matvec,
                        uint64_t seed, const ld_options& o, void* workspace, size_t ws_bytes, hipStream_t st,
                        double* out_logdet, int32_t* degrees, ld_stats* stats) {
    const auto t0 = std::chrono::steady_clock::now();
    const bool f64 = A->dtype == LD_F64;
    const int n = (int)A->n;
    EstimateState S;
    LD_CHECK(make_plan(lmin, lmax, max_degree, o, S.plan));
    S.L = layout_adaptive(A, max_degree, n_matvec, o);
    S.mode = LD_DOT_FORWARD;
    if (o.probe_dist != LD_PROBE_RADEMACHER && o.probe_dist != LD_PROBE_GAUSSIAN)
        return fail(LD_EINVAL, "probe_dist must be LD_PROBE_RADEMACHER or LD_PROBE_GAUSSIAN");
    S.probe = o.probe_dist;
    OwnedWs own;
    Arena ar;
    LD_CHECK(get_workspace(workspace, ws_bytes, adaptive_estimate_ws_bytes(A, max_degree, n_matvec, o), own, ar));
    carve(ar, S.L, S);
    const EstLayout& L = S.L;
    BlkMat PX = L.X;   // F [Q_b | U], the layout of X
    PX.base = ar.take(L.xb);
    AdaptBufs b;
    b.W[0] = S.W0;
    b.W[1] = S.W1;
    b.part = (double*)ar.take((size_t)step_num_wg_any(n) * 64 * 8);
    b.gpart = (double*)ar.take((size_t)cross_num_wg(n) * 64 * 64 * 8);
    b.sums = (double*)ar.take(64 * 64 * 8);
    b.mask = (uint64_t*)ar.take(256);
    b.deg = (int*)ar.take(256);   // one block's columns (at most 64)
    if (ar.base && ar.used > adaptive_estimate_ws_bytes(A, max_degree, n_matvec, o))
        return fail(LD_EINVAL, "internal: workspace layout overflow");
    if (!o.trusted_csr) LD_CHECK(validate_csr(A, S.flag, st));
    LD_CHECK(prepare_rows(A, o, ar, st, S.longrows));
    Timer tm(st, true);
    tm.mark();
    std::vector<int> deg_all((size_t)n_matvec, 0), hdeg;
    // ---- step 3: Y = F S column block by column block; S written out in Q1's block
    S.key0 = probe_stream_key(seed, 0);
    if (S.probe == LD_PROBE_RADEMACHER) LD_CHECK_HIP(launch_sign_mask(n, L.k, S.key0, (uint64_t*)S.mask, st));
    for (int blk = 0; blk < L.Y.nblocks(); ++blk) {
        const int cols = L.Y.bcols(blk), gcol = blk * L.Y.bw;
        void* const sblk = L.Q1.block(blk);
        if (S.probe == LD_PROBE_GAUSSIAN)
            LD_CHECK_HIP(launch_gauss_fill(f64, n, cols, S.key0, gcol, 1.0, sblk, Blk::plain(L.Q1.ld), st));
        else
            LD_CHECK_HIP(launch_fill_signs(f64, n, cols, L.Q1.ld, gcol, (const uint64_t*)S.mask, 1.0, sblk, st));
        LD_CHECK(adaptive_apply(A, S.plan, tol, 0.0, sblk, L.Q1.ld, cols, L.Y.block(blk), L.Y.ld, b, S.longrows,
                                st, hdeg, &S.launches1));
        for (int c = 0; c < cols; ++c) deg_all[(size_t)(gcol + c)] = hdeg[(size_t)c];
    }
    tm.mark();
    // ---- steps 4 and 6: Q_b and U into X
    LD_CHECK(orthonormalize_and_deflate(A, seed, S, st));
    tm.mark();
    // ---- steps 5 and 6: F [Q_b | U] and the quadratic forms x^T F x
    std::vector<double> nu((size_t)L.nc, 0.0), g(64 * 64);
    for (int blk = 0; blk < L.X.nblocks(); ++blk) {
        const int cols = L.X.bcols(blk), gcol = blk * L.X.bw;
        LD_CHECK(adaptive_apply(A, S.plan, tol, 0.0, L.X.block(blk), L.X.ld, cols, PX.block(blk), L.X.ld, b,
                                S.longrows, st, hdeg, &S.launches23));
        for (int c = 0; c < cols; ++c) deg_all[(size_t)(L.k + gcol + c)] = hdeg[(size_t)c];
        LD_CHECK(cross_product(f64, n, L.X.block(blk), Blk::plain(L.X.ld), cols, PX.block(blk), Blk::plain(L.X.ld),
                               cols, nullptr, b.gpart, b.sums, st));
        LD_CHECK_HIP(hipMemcpyAsync(g.data(), b.sums, (size_t)cols * cols * 8, hipMemcpyDeviceToHost, st));
        LD_CHECK_HIP(hipStreamSynchronize(st));
        for (int c = 0; c < cols; ++c) nu[(size_t)(gcol + c)] = g[(size_t)c * cols + c];
    }
    int hflag[2] = {0, 0};
    LD_CHECK_HIP(hipMemcpyAsync(hflag, S.flag + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    LD_CHECK(cholqr_status(hflag));
    tm.mark();
    // ---- step 7: n log(sigma) + t_low + t_res
    KahanSum tl, tr, tot;
    for (int c = 0; c < L.nc; ++c) (c < L.k ? tl : tr).add(nu[(size_t)c]);
    const double t_low = tl.value(), t_res = tr.value() / L.kg;
    tot.add((double)A->n * std::log(S.plan.sigma));
    tot.add(t_low);
    tot.add(t_res);
    *out_logdet = tot.value();
    if (degrees)
        for (int c = 0; c < n_matvec; ++c) degrees[c] = deg_all[(size_t)c];
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->ms_phase1 = tm.ms(0, 1);
        stats->ms_qr = tm.ms(1, 2);
        stats->ms_phase23 = tm.ms(2, 3);
        stats->taylor_terms = S.plan.taylor_terms;
        stats->sigma = S.plan.sigma;
        stats->lo = S.plan.lo;
        stats->hi = S.plan.hi;
        stats->k = L.k;
        stats->k_G = L.kg;
        stats->dot_mode_used = LD_DOT_FORWARD;
        stats->dia_diagonals = S.longrows.dia_nd;
        stats->block_cols1 = L.Y.bw;
        stats->block_cols23 = L.X.bw;
        stats->dia_constant = S.longrows.dia_pres != nullptr;
        stats->spmm_launches = S.launches1 + S.launches23;
        stats->launches1 = S.launches1;
        stats->launches23 = S.launches23;
        stats->t_low = t_low;
        stats->t_res = t_res;
        stats->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return LD_OK;
}

extern "C" {

int ld_workspace_size(const ld_csr* A, int32_t degree, int32_t n_matvec, int32_t want_grad,
                      const ld_options* opts, size_t* bytes) {
    clear_error();
    if (!bytes) return fail(LD_EINVAL, "bytes is null");
    LD_CHECK(check_csr_args(A));
    if (degree < 1) return fail(LD_EINVAL, "degree must be >= 1");
    const ld_options o = resolve(opts);
    if (n_matvec < 0 && want_grad) {
        *bytes = adaptive_ws_bytes(A, (int)(-(int64_t)n_matvec), o);
        return LD_OK;
    }
    if (n_matvec < 0) {
        const size_t elem = A->dtype == LD_F64 ? 8 : 4;
        *bytes = 2 * align_up((size_t)A->n * (size_t)(-(int64_t)n_matvec) * elem) + align_up(256) +
                 long_rows_bytes(A) + dia_bytes(A, o);
        return LD_OK;
    }
    if (n_matvec < 3) return fail(LD_EINVAL, "n_matvec must be >= 3");
    const EstLayout L = layout_envelope(A, degree, n_matvec, want_grad != 0, o);
    *bytes = layout_bytes(L, want_grad != 0);
    return LD_OK;
}

int ld_apply_log(const ld_csr* A, double lmin, double lmax, int32_t degree, const void* V, void* PV,
                 int64_t ncols, const ld_options* opts, void* workspace, size_t ws_bytes,
                 void* stream) {
    clear_error();
    LD_CHECK(check_csr_args(A));
    if (ncols < 0 || ncols > (1 << 20)) return fail(LD_EINVAL, "bad ncols");
    if (ncols > 0 && (!V || !PV)) return fail(LD_EINVAL, "V or PV is null");
    const ld_options o = resolve(opts);
    Plan p;
    LD_CHECK(make_plan(lmin, lmax, degree, o, p));
    if (ncols == 0) return LD_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = A->dtype == LD_F64;
    const size_t elem = f64 ? 8 : 4;
    const int n = (int)A->n, nc = (int)ncols;
    const size_t blk = (size_t)n * nc * elem;
    const uint8_t* v8 = (const uint8_t*)V;
    const uint8_t* p8 = (const uint8_t*)PV;
    if (v8 < p8 + blk && p8 < v8 + blk) return fail(LD_EINVAL, "V and PV overlap");
    const size_t need = 2 * align_up(blk) + align_up(256) + long_rows_bytes(A) + dia_bytes(A, o);
    OwnedWs own;
    Arena ar;
    LD_CHECK(get_workspace(workspace, ws_bytes, need, own, ar));
    void* B0 = ar.take(blk);
    void* B1 = ar.take(blk);
    int* flag = (int*)ar.take(256);
    if (!o.trusted_csr) LD_CHECK(validate_csr(A, flag, st));
    LongRows lr;
    LD_CHECK(prepare_rows(A, o, ar, st, lr));
    const int m = p.degree;
    const int cb = (o.block_cols > 0 && o.block_cols < std::min(nc, 64)) ? o.block_cols : std::min(nc, 64);
    // Horner: r_m = d_m V; r_j = (T - xi_j) r_{j+1} + d_j V, with d_0 carrying
    // log(sigma); r_m starts in B0, the steps ping-pong B0/B1, step 0 writes PV.
    LD_CHECK_HIP(launch_scale_copy(f64, n, nc, V, nc, p.d[m], B0, nc, st));
    const void* cur = B0;
    for (int j = m - 1; j >= 0; --j) {
        void* out = j == 0 ? PV : (cur == B0 ? B1 : B0);
        StepArgs s{};
        s.kind = STEP_HORNER_VEC;
        s.win = cur;
        s.wout = out;
        s.ld = nc;
        s.alpha = p.alpha;
        s.beta = p.beta[j];
        s.dj = j == 0 ? p.d[0] + std::log(p.sigma) : p.d[j];
        s.vsrc = V;
        s.ldv = nc;
        LD_CHECK(run_step(f64, A, s, nc, cb, st, nullptr, lr));
        cur = out;
    }
    if (!workspace) LD_CHECK_HIP(hipStreamSynchronize(st));
    return LD_OK;
}

int ld_apply_log_adaptive(const ld_csr* A, double lmin, double lmax, int32_t max_degree, double tol,
                          const void* V, void* PV, int64_t ncols, const ld_options* opts, void* workspace,
                          size_t ws_bytes, void* stream, int32_t* degrees) {
    clear_error();
    LD_CHECK(check_csr_args(A));
    if (ncols < 0 || ncols > (1 << 20)) return fail(LD_EINVAL, "bad ncols");
    if (ncols > 0 && (!V || !PV)) return fail(LD_EINVAL, "V or PV is null");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and >= 0");
    const ld_options o = resolve(opts);
    Plan p;
    LD_CHECK(make_plan(lmin, lmax, max_degree, o, p));
    if (ncols == 0) return LD_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = A->dtype == LD_F64;
    const size_t elem = f64 ? 8 : 4;
    const int n = (int)A->n, nc = (int)ncols;
    const size_t blk = (size_t)n * nc * elem;
    const uint8_t* v8 = (const uint8_t*)V;
    const uint8_t* p8 = (const uint8_t*)PV;
    if (v8 < p8 + blk && p8 < v8 + blk) return fail(LD_EINVAL, "V and PV overlap");
    OwnedWs own;
    Arena ar;
    LD_CHECK(get_workspace(workspace, ws_bytes, adaptive_ws_bytes(A, nc, o), own, ar));
    AdaptBufs b;
    b.W[0] = ar.take(blk);
    b.W[1] = ar.take(blk);
    b.part = (double*)ar.take((size_t)step_num_wg_any(n) * 64 * 8);
    b.gpart = (double*)ar.take((size_t)cross_num_wg(n) * 64 * 64 * 8);
    b.sums = (double*)ar.take(64 * 64 * 8);
    b.mask = (uint64_t*)ar.take(256);
    b.deg = (int*)ar.take((size_t)nc * 4);
    int* flag = (int*)ar.take(256);
    if (!o.trusted_csr) LD_CHECK(validate_csr(A, flag, st));
    LongRows lr;
    LD_CHECK(prepare_rows(A, o, ar, st, lr));
    std::vector<int> hdeg;
    LD_CHECK(adaptive_apply(A, p, tol, std::log(p.sigma), V, nc, nc, PV, nc, b, lr, st, hdeg, nullptr));
    if (degrees)
        for (int c = 0; c < nc; ++c) degrees[c] = hdeg[(size_t)c];
    return LD_OK;
}

int ld_adaptive_workspace_size(const ld_csr* A, int32_t max_degree, int32_t n_matvec, const ld_options* opts,
                               size_t* bytes) {
    clear_error();
    if (!bytes) return fail(LD_EINVAL, "bytes is null");
    LD_CHECK(check_csr_args(A));
    if (max_degree < 1) return fail(LD_EINVAL, "max_degree must be >= 1");
    if (n_matvec < 3) return fail(LD_EINVAL, "n_matvec must be >= 3");
    *bytes = adaptive_estimate_ws_bytes(A, max_degree, n_matvec, resolve(opts));
    return LD_OK;
}

int ld_logdet_estimate_adaptive(const ld_csr* A, double lmin, double lmax, int32_t max_degree, double tol,
                                int32_t n_matvec, uint64_t seed, const ld_options* opts, void* workspace,
                                size_t ws_bytes, void* stream, double* out_logdet, int32_t* degrees,
                                ld_stats* stats) {
    clear_error();
    if (!out_logdet) return fail(LD_EINVAL, "out_logdet is null");
    LD_CHECK(check_estimate_args(A, lmin, lmax, max_degree, n_matvec));
    if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(LD_EINVAL, "tol must be finite and >= 0");
    return run_logdet_adaptive(A, lmin, lmax, max_degree, tol, n_matvec, seed, resolve(opts), workspace, ws_bytes,
                               (hipStream_t)stream, out_logdet, degrees, stats);
}

int ld_logdet_estimate(const ld_csr* A, double lmin, double lmax, int32_t degree,
                       int32_t n_matvec, uint64_t seed, const ld_options* opts, void* workspace,
                       size_t ws_bytes, void* stream, double* out_logdet, ld_stats* stats) {
    clear_error();
    if (!out_logdet) return fail(LD_EINVAL, "out_logdet is null");
    LD_CHECK(check_estimate_args(A, lmin, lmax, degree, n_matvec));
    return run_logdet(A, lmin, lmax, degree, n_matvec, seed, resolve(opts), workspace, ws_bytes,
                      (hipStream_t)stream, out_logdet, nullptr, stats);
}

int ld_logdet_estimate_noalloc(const ld_csr* A, double lmin, double lmax, int32_t degree,
                               int32_t n_matvec, uint64_t seed, const ld_options* opts, void* stream,
                               double* out_logdet, ld_stats* stats) {
    clear_error();
    if (!out_logdet) return fail(LD_EINVAL, "out_logdet is null");
    LD_CHECK(check_estimate_args(A, lmin, lmax, degree, n_matvec));
    const ld_options o = resolve(opts);
    const size_t need = layout_bytes(layout_envelope(A, degree, n_matvec, false, o), false);
    if (need > kNoAllocScratchBytes)
        return fail(LD_EWORKSPACE, "the estimate needs " + std::to_string(need) +
                                       " bytes of scratch; the library's static scratch holds " +
                                       std::to_string(kNoAllocScratchBytes));
    hipStream_t st = (hipStream_t)stream;
    int dev = -1, sdev = -1;
    LD_CHECK_HIP(hipGetDevice(&dev));
    LD_CHECK_HIP(hipStreamGetDevice(st, &sdev));
    if (sdev != dev) return fail(LD_EINVAL, "the stream must belong to the current device");
    void* ws = nullptr;
    LD_CHECK(scratch_address(&ws));
    return run_logdet(A, lmin, lmax, degree, n_matvec, seed, o, ws, kNoAllocScratchBytes, st, out_logdet,
                      nullptr, stats, /*timed=*/false);
}

int ld_spectral_bounds(const ld_csr* A, int32_t lanczos_steps, void* stream, double* lmin,
                       double* lmax) {
    clear_error();
    LD_CHECK(check_csr_args(A));
    if (!lmin || !lmax || lanczos_steps < 0 || lanczos_steps > kMaxLanczos)
        return fail(LD_EINVAL, "need lmin, lmax non-null and 0 <= lanczos_steps <= " +
                                   std::to_string(kMaxLanczos));
    hipStream_t st = (hipStream_t)stream;
    const int nwg = gersh_num_wg((int)A->n);
    OwnedWs own;
    if (hipMalloc(&own.p, (size_t)2 * nwg * sizeof(double) + 256) != hipSuccess)
        return fail(LD_ENOMEM, "hipMalloc failed");
    int* flag = (int*)((char*)own.p + (size_t)2 * nwg * sizeof(double));
    LD_CHECK(validate_csr(A, flag, st));
    LD_CHECK_HIP(launch_gershgorin(A->dtype == LD_F64, dev_of(A), (double*)own.p, st));
    std::vector<double> h((size_t)2 * nwg);
    LD_CHECK_HIP(hipMemcpyAsync(h.data(), own.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
    LD_CHECK_HIP(hipStreamSynchronize(st));
    double lo = INFINITY, hi = -INFINITY;
    for (int i = 0; i < nwg; ++i) {
        lo = std::fmin(lo, h[2 * i]);
        hi = std::fmax(hi, h[2 * i + 1]);
    }
    *lmin = lo;
    *lmax = hi;
    if (lanczos_steps > 0 && A->n > 0) {
        double top = hi;
        LD_CHECK(lanczos_upper(A, lanczos_steps, std::fmax(std::fabs(lo), std::fabs(hi)), st, &top));
        *lmax = std::fmin(hi, top);
    }
    if (!(lo > 0.0)) return fail(LD_EINDEF, "Gershgorin lower bound is not positive");
    return LD_OK;
}

int ld_logdet_grad(const ld_csr* A, double lmin, double lmax, int32_t degree, int32_t n_matvec,
                   uint64_t seed, const ld_options* opts, void* workspace, size_t ws_bytes,
                   void* stream, double* out_logdet, void* grad_val, ld_stats* stats) {
    clear_error();
    if (!out_logdet) return fail(LD_EINVAL, "out_logdet is null");
    LD_CHECK(check_estimate_args(A, lmin, lmax, degree, n_matvec));
    if (!grad_val && A->nnz > 0) return fail(LD_EINVAL, "grad_val is null");
    return run_logdet(A, lmin, lmax, degree, n_matvec, seed, resolve(opts), workspace, ws_bytes,
                      (hipStream_t)stream, out_logdet, grad_val, stats);
}

}  // extern "C"
