// Launchers of the gfx950 kernels (kernels.hip).  All launches are
// asynchronous on `stream`; shapes are checked by the caller (api.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ld {

// Kinds of Newton step (one SpMM pass over a block of columns).
enum StepKind : int {
    STEP_HORNER_SIGNS = 0,  // out = alpha*A*in - beta*in + dj*S   (S from the sign mask)
    STEP_HORNER_VEC = 1,    // out = alpha*A*in - beta*in + dj*V   (V in memory)
    STEP_DOT_FWD = 2,       // out = alpha*A*in - beta*in; <X,out> (and <X,in> if first)
    STEP_DOT_SQ = 3,        // out = alpha*A*in - beta*in; <in,out>, <out,out> (and <in,in>)
    STEP_PLAIN = 4,         // out = alpha*A*in - beta*in
    STEP_PLAIN_ACC = 5,     // PLAIN, and acc[r, c] += dj*out[r, c] for columns c < acc_cols
    STEP_ACC_NORM = 6,      // PLAIN, acc += dj*out on the columns active in *active, <out,out>
};

// A dense n x cols matrix stored as column blocks of width bw: element
// (r, c) lives at (C / bw) * bstride + r * ld + C % bw (in elements), with
// C = c + c0 (c0 selects a column range).  A plain row-major matrix is the
// single-block case.
struct Blk {
    int ld;
    int bw;
    long long bstride;
    int c0;
    __host__ __device__ size_t offset(int c) const {
        const int C = c + c0;
        return (size_t)(C / bw) * (size_t)bstride + (size_t)(C % bw);
    }
    static Blk plain(int ld, int c0 = 0) { return Blk{ld, 1 << 30, 0, c0}; }
    Blk shifted(int dc) const { return Blk{ld, bw, bstride, c0 + dc}; }
};

struct CsrDev {
    int n;
    int nnz;
    const int* row_ptr;
    const int* col_idx;
    const void* val;
};

constexpr int kMaxDiag = 9;
constexpr int kXcds = 8;     // XCDs of the MI355X; workgroup w runs on XCD w % 8      // diagonals of the diagonal storage (9-point stencils, 7-point 3-D)

// Geometry of a Newton step launch over columns [c0, c0+bcols) of row-major
// blocks with leading dimension ld (elements).
struct StepArgs {
    int kind;
    bool first;
    const void* win;
    void* wout;
    int ld, c0, bcols;
    int gshift;                // global column = local column + gshift
    double alpha, beta, dj;
    const void* vsrc;          // HORNER_VEC: V;  DOT_FWD: X
    int ldv;
    const uint64_t* mask;      // HORNER_SIGNS: one word of sign bits per row
    // HORNER_SIGNS on the diagonal storage, when non-null: the same bits as
    // eight byte planes (plane p, n bytes: byte p of every row's word), so a
    // step reads one byte per row and 16-byte chunk instead of the word
    const uint8_t* planes = nullptr;
    double* ps0;               // partial sums [nwg][part_ld], may be null
    double* ps1;
    double* ps2;
    int part_ld;
    // Rows with more than kLongRow entries, when listed here, are skipped by the
    // row-group kernel and done by a workgroup each (partial rows after the
    // regular ones: kLongWgs of them).
    const int* long_rows;      // device list of long rows (ascending), or null
    const int* long_count;     // device count of the list
    void* acc;                 // PLAIN_ACC / ACC_NORM: row-major accumulator (column c of the step = column c)
    int ldacc, acc_cols;
    const uint64_t* active;    // ACC_NORM: device word, bit (c - c0) set = column c still accumulates
    // Diagonal storage of A (dia_nd > 0): row r holds dia[r*dia_nd + q] at
    // column r + dia_off[q] (offsets ascending; 0 where absent); replaces the
    // CSR arrays in the gather.
    const void* dia;
    int dia_nd;
    int dia_off[kMaxDiag];
    // every diagonal one constant (dia_pres non-null): row r holds dia_cval[q]
    // on diagonal q when bit q of dia_pres[r] is set; dia is not read
    const uint16_t* dia_pres;
    double dia_cval[kMaxDiag];
    // tile order: 0 = XCD x (blockIdx % 8) walks the x-th contiguous band of
    // row tiles (stencil neighbours stay in that XCD's L2); 1 = workgroup w
    // takes tiles w, w + grid, ... (spreads each tile's neighbours over the
    // XCDs; faster once the blocks stream from HBM)
    int interleave;
    // with interleave = 0: > 0 cuts the bands into chunks of about this many
    // rows, chunk c going to XCD c % 8 (each XCD walks its chunks in order);
    // 0 = one contiguous band per XCD
    int chunk_rows;
    // 1: the output block is written with non-temporal (streaming) stores
    int nt_out;
    // when non-null: set to the number of launches over consecutive row
    // ranges the step took (1 but for streaming steps with column sums)
    int* ranges_out = nullptr;
};

constexpr int kLongRow = 64;     // entries above which a row is "long"
constexpr int kLongWgs = 1024;   // workgroups of the long-row launch

// Deterministic list of the rows with more than kLongRow entries:
// list[0..count) ascending, *count on the device.  tmp: >= n/256 + 2 ints.
hipError_t launch_long_rows(const CsrDev& A, int* tmp, int* list, int* count, hipStream_t st);

// Widest column range of one launch (a row group spans at most one wave).
int step_max_cols(bool f64, const StepArgs& s);
// Partial rows a column-sum launch writes (one per workgroup), at most: for
// 16-byte aligned blocks of at most bcols columns, and for any layout.
int step_num_wg_bound(int n, int bcols, int elem_bytes);
int step_num_wg_any(int n);
// Rows of one tile of the column-sum kinds over bcols columns of 16-byte aligned blocks.
int step_tile_rows(int bcols, int elem_bytes);

// *nwg_out (may be null): workgroup partial rows the launch wrote (dot kinds:
// the grid, which is the number of resident workgroups or less, plus the
// long-row launch's kLongWgs).
hipError_t launch_step(bool f64, const CsrDev& A, const StepArgs& s, hipStream_t st, int* nwg_out = nullptr);

// Sign mask of stream `key`: bit c of word r = (probe(r, c) == -1), c < k <= 64.
// With `planes` non-null also its eight byte planes: planes[p*n + r] = byte p
// of word r (8n bytes).
hipError_t launch_sign_mask(int n, int k, uint64_t key, uint64_t* mask, hipStream_t st,
                            uint8_t* planes = nullptr);

// out[r*ld + c] = scale * S[r, c + gshift] for c < k (other columns untouched).
hipError_t launch_fill_signs(bool f64, int n, int k, int ld, int gshift, const uint64_t* mask,
                             double scale, void* out, hipStream_t st);

// out[r, c] = scale * g(key, (c + col0)*n + r + 1), c < k, out column-blocked:
// standard normal entries by Box-Muller (FP64) on the two 32-bit halves of
// SplitMix64 output number (c + col0)*n + r + 1 of the stream key.
hipError_t launch_gauss_fill(bool f64, int n, int k, uint64_t key, int col0, double scale, void* out, Blk bo,
                             hipStream_t st);

// out[r, c] = scale * V[r, c] (row-major, V with ldv, out with ldo), c < ncols.
hipError_t launch_scale_copy(bool f64, int n, int ncols, const void* V, int ldv, double scale,
                             void* out, int ldo, hipStream_t st);

// Partial cross products X^T Z per workgroup, FP64: part[wg][i*kz+j],
// cross_num_wg(n) rows.  Z is a second block, or, with zmask (one word per
// row, bit j set = -1), the signs of columns [0, kz); Z is then ignored.
int cross_num_wg(int n);
hipError_t launch_cross(bool f64, int n, const void* X, Blk bx, int kx, const void* Z, Blk bz,
                        int kz, const uint64_t* zmask, double* part, hipStream_t st);

// out[o*out_ld + j] = sum_wg part[o*outer_stride + wg*part_ld + j], j < len
// (Neumaier, fixed order).
hipError_t launch_reduce(const double* part, int nwg, int len, int part_ld, int outer,
                         long long outer_stride, double* out, int out_ld, hipStream_t st);

// G = R^T R for a k x k FP64 Gram (k <= 64, row-major): R (may be null) and
// R^{-1}, both upper triangular; *flag = 0, 1 (non-finite entry) or 2 (pivot
// not positive or below 1e-7 sqrt(G_jj)), R^{-1} zero unless 0.
hipError_t launch_chol_factor(const double* G, int k, double* R, double* Rinv, int* flag,
                              hipStream_t st);

// out[r, j] = (base ? base[r, j] : 0) + (zmask ? sign of bit j of zmask[r] : 0)
//             + sign_m * sum_i Y[r, i] M[i, j],
// M k_y x k_out FP64 (device), j < k_out; Y, base and out column-blocked
// (base may alias out: each element is read before it is written).
hipError_t launch_rowmat(bool f64, int n, const void* Y, Blk by, int ky, const double* M, int kout,
                         double sign_m, const uint64_t* zmask, const void* base, Blk bb,
                         void* out, Blk bo, hipStream_t st);

// CSR structure check: *flag (device int) set to 1 on any violation.
hipError_t launch_validate_csr(const CsrDev& A, int* flag, hipStream_t st);

// Gershgorin: per-workgroup (min(a_ii - r_i), max(a_ii + r_i)) into part[2*wg].
int gersh_num_wg(int n);
hipError_t launch_gershgorin(bool f64, const CsrDev& A, double* part, hipStream_t st);

// Gradient sweep step (all blocks n x ld row-major, ncols used; grad FP64):
//   grad[nz(r,c)] (+)= alpha * sum_cols own[r, col] * w[c, col]
//   ADJ_HORNER:  lam_out = alpha*A*lam_in - beta*lam_in + dj*L,  own = lam_in
//   ADJ_PLAIN:   lam_out = alpha*A*lam_in - beta*lam_in,         own = lam_in
//   ADJ_SQUARED: lam_out = alpha*A*lam_in - beta*lam_in + q0*w + q1*(alpha*A*w - beta*w),
//                own = wgt(col) * (lam_in + p1*w), wgt = 1 for col < wsplit, else whi
//   ADJ_PLAIN2 (diagonal storage only): ADJ_PLAIN, and the entry also picks up
//                alpha * sum_cols lam_out[r, col] * w2[c, col] (two steps of the
//                sketch's adjoint per read and write of the gradient)
//   ADJ_SQUARED_SYM (diagonal storage with offsets symmetric about the main
//                diagonal): ADJ_SQUARED's step, and each mirrored pair is summed
//                into the half accumulator of its upper entry: for c > r the
//                slot (r, c) picks up alpha * sum_cols (own[r] w[c] + own[c] w[r]),
//                the diagonal slot alpha * sum_cols own[r] w[r]; slots are
//                grad[r * nh + h] for the h-th non-negative offset (the lower
//                entries have no slot)
enum AdjMode : int { ADJ_HORNER = 0, ADJ_PLAIN = 1, ADJ_SQUARED = 2, ADJ_PLAIN2 = 3, ADJ_SQUARED_SYM = 4 };
struct AdjArgs {
    int mode;
    const void* lam_in;
    void* lam_out;
    const void* w;
    const void* w2;      // ADJ_PLAIN2
    const void* L;
    double* grad;
    int ld, ncols;
    double alpha, beta, dj;
    double q0, q1, p1;   // ADJ_SQUARED coefficients
    int wsplit;          // ADJ_SQUARED column weights: 1 before wsplit, whi after
    double whi;
    bool first;      // grad is overwritten instead of accumulated
    bool last;       // no lam_out needed (only the SDDMM)
    bool nt_out;     // lam_out written with non-temporal (streaming) stores
    double lam_scale = 1.0;   // lam = lam_scale * lam_in (0: a zero block, lam_in not read)
};
hipError_t launch_adjoint(bool f64, const CsrDev& A, const AdjArgs& a, hipStream_t st);

// The same step on the diagonal storage (modes ADJ_PLAIN, ADJ_PLAIN2,
// ADJ_SQUARED, ADJ_SQUARED_SYM): presence bits per row (pres), the values either one per
// diagonal (constant) or dia[r*nd + q]; the gradient at A's CSR positions
// (row_ptr of A).
struct AdjDia {
    int nd;
    int off[kMaxDiag];
    const uint16_t* pres;
    const void* dia;
    bool constant;
    double cval[kMaxDiag];
    int chunk_rows;   // > 0: chunked XCD bands of this many rows (0: contiguous bands)
    int qh0 = 0, nh = 0;   // ADJ_SQUARED_SYM: index of offset 0, number of offsets >= 0
};
hipError_t launch_adjoint_dia(bool f64, const CsrDev& A, const AdjArgs& a, const AdjDia& dg, hipStream_t st);

// Every stored entry of the gradient from the half accumulator of
// ADJ_SQUARED_SYM (half[r * nh + h], nh = dg.nh): g at the CSR position of
// (r, c) = half of the upper entry's pair sum for r != c, the diagonal slot
// for r = c (a mean of mirrored pairs, as launch_symmetrize gives); *flag
// (device int) set to 1 when an entry's mirror is absent.
hipError_t launch_expand_half(const CsrDev& A, const AdjDia& dg, const double* half, double* g, int* flag,
                              hipStream_t st);

// Mean of every mirrored pair g[(r,c)], g[(c,r)] (FP64, CSR positions); *flag
// (device int) set to 1 when some entry has no mirror.
hipError_t launch_symmetrize(const CsrDev& A, double* g, int* flag, hipStream_t st);

// y[i] = (float)x[i], i < len.
hipError_t launch_narrow(long long len, const double* x, float* y, hipStream_t st);

// Row probe (info: device, 64 ints, preset to 0 by the caller): info[0] =
// number of diagonals nd (distinct offsets col - row of 64 sampled rows,
// ascending, in info[1..nd]; -1 if more than kMaxDiag),
// info[kBandInfo + i] = row_ptr[i*n/8], i = 0..8 (entries per XCD band), and
// at info + kConstInfo nd doubles: each diagonal's value in the first sampled
// row that stores it.  Then the diagonal storage: dia[r*nd + q] =
// A[r, r + info[1+q]] or 0, pres[r] bit q = row r stores diagonal q;
// info[kDiaFlag] = 1 when some stored entry lies on none of the diagonals (the
// storage is then unusable), info[kConstFlag] = 1 when some entry differs from
// its diagonal's sampled value (else every diagonal is one constant).
constexpr int kBandInfo = 16;
constexpr int kConstFlag = 13;
constexpr int kConstInfo = 32;   // int index; 8-byte aligned doubles
hipError_t launch_rows_probe(bool f64, const CsrDev& A, int* info, hipStream_t st);
hipError_t launch_dia_build(bool f64, const CsrDev& A, void* dia, uint16_t* pres, int* info, hipStream_t st);

// Alg. 2's stopping test after the step that produced w_m: for columns c < qc
// still active in *mask, e = |d_m| sqrt(sums[c*stride]) <= tol clears the bit
// and sets deg[c] = m (deg of the columns that never stop is left as set by
// the caller).  One wave; sums are FP64 column sums of w_m^2.
hipError_t launch_adapt_decide(const double* sums, int stride, int qc, double dm_abs, double tol, int m,
                               uint64_t* mask, int* deg, hipStream_t st);

// y[i] = (double)x[i], i < len.
hipError_t launch_widen(long long len, const float* x, double* y, hipStream_t st);

// y = a*x + b*y elementwise on contiguous arrays of length len.
hipError_t launch_axpby(bool f64, long long len, double a, const void* x, double b, void* y,
                        hipStream_t st);

}  // namespace ld
