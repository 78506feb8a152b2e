// gfx950 kernels of the Léja + Hutch++ hot path.
//
// Data layout: dense blocks are row-major n x ld (a row's columns are
// contiguous), so one sparse row's gather W[col_idx[k], c0:c0+b] is a single
// contiguous run of b elements.  A wave64 is split into row groups of
// lpr = ceil(b/VEC) lanes; each lane owns VEC adjacent columns (16-byte
// vectors), so a row group reads a gathered row with one coalesced access.
//
// Work distribution is XCD-aware: workgroups are issued round-robin over the
// 8 XCDs, so the logical row tile of a workgroup is remapped such that each
// XCD walks one contiguous band of rows.  Stencil neighbours (rows r +- N)
// are then mostly found in that XCD's own L2.  Matrices whose entries crowd
// into a few bands take interleaved tiles instead (balanced XCD load).
//
// Reductions never use atomics: each workgroup writes FP64 partial sums and a
// separate kernel adds them in a fixed order (Neumaier), so every result is
// deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <mutex>
#include <type_traits>
#include <unordered_map>

#include "kernels.h"

namespace ld {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

template <typename T, int V>
struct alignas(sizeof(T) * V) Pack {
    T v[V];
};

template <typename T, int V>
__device__ __forceinline__ Pack<T, V> load_pack(const T* p) {
    return *reinterpret_cast<const Pack<T, V>*>(p);
}
template <typename T, int V>
__device__ __forceinline__ void store_pack(T* p, const Pack<T, V>& x) {
    *reinterpret_cast<Pack<T, V>*>(p) = x;
}
// Streaming store (non-temporal hint): the line is not kept in L2, which then
// holds more of the rows the next tiles gather.
template <typename T, int V>
__device__ __forceinline__ void store_pack_nt(T* p, const Pack<T, V>& x) {
    typedef T vt __attribute__((ext_vector_type(V)));
    vt v;
#pragma unroll
    for (int e = 0; e < V; ++e) v[e] = x.v[e];
    __builtin_nontemporal_store(v, reinterpret_cast<vt*>(p));
}

// Logical tile of this workgroup: XCD x (= blockIdx % 8) gets the contiguous
// tile range [x*(nwg/8) + min(x, nwg%8), ...).
__device__ __forceinline__ int xcd_tile(int bid, int nwg) {
    const int x = bid % kXcds;
    const int i = bid / kXcds;
    const int base = nwg / kXcds, rem = nwg % kXcds;
    return x * base + (x < rem ? x : rem) + i;
}

// SplitMix64 output number i of the generator seeded with key.
__device__ __forceinline__ uint64_t probe_bits(uint64_t key, uint64_t i) {
    uint64_t z = key + i * 0x9E3779B97F4A7C15ull;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

int div_up(long long a, long long b) { return (int)((a + b - 1) / b); }
__device__ __forceinline__ int div_up_dev(int a, int b) { return (int)(((long long)a + b - 1) / b); }

// rows of one row group iteration
inline int lanes_per_row(int bcols, int vec) { return (bcols + vec - 1) / vec; }

constexpr int kStepIters = 2;      // row groups per wave and launch
constexpr int kRangeTiles = 48;    // tiles per workgroup and launch of a streaming step with column sums
constexpr int kWaveNz = 384;       // CSR entries one wave stages in LDS
constexpr int kMaxDotCols = 64;    // columns of one launch of the kinds with column sums
constexpr int kAdjBatch = 4;       // CSR entries of a row whose gathers the adjoint issues together
constexpr int kAdjStageNz = 1536;  // CSR entries one adjoint workgroup stages in LDS

constexpr bool is_dot(int kind) { return kind == STEP_DOT_FWD || kind == STEP_DOT_SQ || kind == STEP_ACC_NORM; }
// kinds with a first-step variant (it adds the sums of the input block itself)
constexpr bool has_first(int kind) { return kind == STEP_DOT_FWD || kind == STEP_DOT_SQ; }
constexpr int threads_of(int) { return 256; }
// Kinds with column sums run a fixed grid of at most kDotWgs workgroups (all
// resident on the 256 CUs), each looping over row tiles and reducing its
// column sums once; the others launch one workgroup per tile.
constexpr int kDotWgs = 2048;
inline int grid_of(int kind, int ntiles) { return is_dot(kind) && ntiles > kDotWgs ? kDotWgs : ntiles; }

// ---------------------------------------------------------------------------
// Newton step: out = alpha*A*in - beta*in (+ dj*source), optional dot partials
// or accumulation acc += dj*out.
//
// Wave w of a workgroup owns the contiguous rows R0 + w*rpw*ITERS + [0,
// rpw*ITERS).  Each wave stages its own slice of row_ptr and, when it fits,
// of col_idx/val in LDS (coalesced loads, no workgroup barrier); each row
// group then reads its row's entries from LDS (one address per row group, a
// broadcast) and issues the gathers.  Slices with more than kWaveNz entries
// (long rows) read the CSR arrays directly.
//
// Column sums (dot kinds): each wave reduces its row groups through its own
// LDS region, stores its column sums, and bumps an LDS counter; the last wave
// to arrive adds the NW wave sums in wave order and writes the workgroup's
// partial row.  No wave ever waits at a barrier, and the order of every
// addition is fixed.  Global column of local column c: c + gshift.
// ---------------------------------------------------------------------------
struct DiaOff {
    int o[kMaxDiag];
};
// one value per diagonal (constant-coefficient storage)
template <typename T>
struct DiaVal {
    T c[kMaxDiag];
};

// ND > 0: gather from the diagonal storage, at most ND diagonals (compile-time
// width of the per-row gather batch); ND = 0: from the CSR arrays.
template <typename T, int VEC, int KIND, bool FIRST, int ITERS, int NT, int ND>
__global__ __launch_bounds__(NT) void step_kernel(
    int n, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
    const T* __restrict__ val, const T* __restrict__ win, T* __restrict__ wout, int ld, int c0,
    int bcols, int gshift, T alpha, T beta, T dj, const T* __restrict__ vsrc, int ldv,
    const uint64_t* __restrict__ mask, double* __restrict__ ps0, double* __restrict__ ps1,
    double* __restrict__ ps2, int part_ld, int lpr, int rpw, int skip_long, T* __restrict__ accum,
    int ldacc, int acc_cols, int ntiles, const uint64_t* __restrict__ active, const T* __restrict__ dia, int nd,
    DiaOff off, int interleave, int chunk, int nt_out, const uint16_t* __restrict__ dpres, DiaVal<T> cv,
    int tile0, int add_parts) {
    constexpr bool kDot = is_dot(KIND);
    constexpr int NW = NT / 64;
    constexpr int kSums = kDot ? ((FIRST ? 1 : 0) + 1 + (KIND == STEP_DOT_SQ ? 1 : 0)) : 0;
    static_assert(KIND != STEP_ACC_NORM || !FIRST, "ACC_NORM has no first-step variant");
    constexpr int kStageBytes = kWaveNz * (int)(sizeof(T) + 4);
    constexpr int kLaneBytes = 64 * VEC * 8;                  // per-lane sums of one wave
    constexpr int kWaveBytes = kStageBytes > kLaneBytes ? kStageBytes : kLaneBytes;
    __shared__ int s_rp[NW][64 * ITERS + 1];
    __shared__ __align__(16) unsigned char s_wave[NW][kWaveBytes];
    __shared__ double s_cols[kDot ? NW * kSums * kMaxDotCols : 1];
    __shared__ unsigned s_count;

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane / lpr;
    const int li = lane - g * lpr;
    const bool lane_ok = g < rpw;
    const int col = c0 + li * VEC;
    const int rows_per_wave = rpw * ITERS;
    if constexpr (kDot) {
        if (threadIdx.x == 0) s_count = 0;
        __syncthreads();   // the only workgroup barrier: the counter is set before any wave can finish
    }

    T* const s_val = reinterpret_cast<T*>(s_wave[wave]);
    int* const s_col = reinterpret_cast<int*>(s_wave[wave] + kWaveNz * sizeof(T));
    int* const rp = s_rp[wave];
    double s0[VEC], s1[VEC], s2[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) s0[e] = s1[e] = s2[e] = 0.0;

    // Tiles of NW*rows_per_wave rows.  Banded order (chunk = 0): XCD x (=
    // blockIdx % 8) owns the contiguous band of tiles [x*base + min(x, rem),
    // ...) and its workgroups take the band's tiles round-robin in order, so
    // the XCD's active rows stay a narrow window.  Chunked bands (chunk > 0):
    // the tiles are cut into chunks of `chunk` tiles, chunk c belongs to XCD
    // c % 8, and each XCD's workgroups take its chunks' tiles round-robin in
    // order, so an XCD's consecutive chunks lie 8 chunks apart (a 3-D
    // stencil's plane: the plane neighbours of a row were gathered by the
    // same XCD one chunk earlier, in its L2).  Interleaved order: workgroup w
    // takes tiles w, w + grid, ...  With one workgroup per tile each takes one.
    const int xcd = blockIdx.x % kXcds;
    const int base = ntiles / kXcds, rem = ntiles % kXcds;
    const int band0 = interleave ? 0 : xcd * base + (xcd < rem ? xcd : rem);
    const int band_len = interleave ? ntiles : base + (xcd < rem ? 1 : 0);
    const int wgs_here =
        interleave ? (int)gridDim.x : (int)(gridDim.x / kXcds) + (xcd < (int)(gridDim.x % kXcds) ? 1 : 0);
    for (int t = interleave ? (int)blockIdx.x : (int)(blockIdx.x / kXcds);; t += wgs_here) {
    int tile;
    if (interleave) {
        if (t >= ntiles) break;
        tile = t;
    } else if (chunk > 0) {
        const int c = (t / chunk) * kXcds + xcd;
        if ((long long)c * chunk >= ntiles) break;   // later chunks of this XCD lie further out
        tile = c * chunk + t % chunk;
        if (tile >= ntiles) continue;                // the tail of the last, partial chunk
    } else {
        if (t >= band_len) break;
        tile = band0 + t;
    }
    const int W0 = (tile0 + tile) * (NW * rows_per_wave) + wave * rows_per_wave;   // first row of this wave
    const int nrows = max(0, min(rows_per_wave, n - W0));
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // the previous tile's LDS reads come first
    __builtin_amdgcn_wave_barrier();
    int K0 = 0;
    bool staged;
    if constexpr (ND > 0) {
        // the wave's rows are one contiguous run of nrows*nd diagonal values
        staged = !dpres && nrows * nd <= kWaveNz;   // constant values: nothing to stage
        if (staged) {   // read once per step: streamed past L2 when the launch works from HBM
            if (nt_out)
                for (int k = lane; k < nrows * nd; k += 64) s_val[k] = __builtin_nontemporal_load(dia + (size_t)W0 * nd + k);
            else
                for (int k = lane; k < nrows * nd; k += 64) s_val[k] = dia[(size_t)W0 * nd + k];
        }
    } else {
        if (nrows > 0)   // waves past the last row read nothing
            for (int t2 = lane; t2 <= nrows; t2 += 64) rp[t2] = row_ptr[W0 + t2];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        K0 = nrows > 0 ? rp[0] : 0;
        const int K1 = nrows > 0 ? rp[nrows] : 0;
        staged = (K1 - K0) <= kWaveNz;
        if (staged) {   // read once per step: streamed past L2 when the launch works from HBM
            if (nt_out) {
                for (int k = K0 + lane; k < K1; k += 64) {
                    s_col[k - K0] = __builtin_nontemporal_load(col_idx + k);
                    s_val[k - K0] = __builtin_nontemporal_load(val + k);
                }
            } else {
                for (int k = K0 + lane; k < K1; k += 64) {
                    s_col[k - K0] = col_idx[k];
                    s_val[k - K0] = val[k];
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();

#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
        const int lr = it * rpw + g;
        if (!lane_ok || lr >= nrows) continue;
        const int row = W0 + lr;
        T acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = T(0);
        if constexpr (ND > 0) {
            // offsets ascending = the CSR column order: the same sums in the same
            // order (a diagonal absent from the row, or leaving the matrix, adds an
            // exact zero product of the row's own vector).  All gathers are issued
            // before the first product.
            int cq[ND];
            T aq[ND];
            const unsigned pbits = dpres ? dpres[row] : 0u;
#pragma unroll
            for (int q = 0; q < ND; ++q) {
                const int c = row + off.o[q];
                const bool ok = q < nd && (unsigned)c < (unsigned)n;
                cq[q] = ok ? c : row;
                if (dpres)
                    aq[q] = ok && ((pbits >> q) & 1u) ? cv.c[q] : T(0);
                else
                    aq[q] = ok ? (staged ? s_val[lr * nd + q] : dia[(size_t)row * nd + q]) : T(0);
            }
            Pack<T, VEC> xq[ND];
#pragma unroll
            for (int q = 0; q < ND; ++q) xq[q] = load_pack<T, VEC>(win + (size_t)cq[q] * ld + col);
#pragma unroll
            for (int q = 0; q < ND; ++q) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = fma(aq[q], xq[q].v[e], acc[e]);
            }
        } else {
        const int beg = rp[lr], end = rp[lr + 1];
        if (skip_long && end - beg > kLongRow) continue;   // done by long_row_kernel
        if (staged) {
            // batches of four entries: their gathers are issued before their
            // products (same order of the sums as one entry at a time)
            int k = beg - K0;
            const int kend = end - K0;
            for (; k + 4 <= kend; k += 4) {
                Pack<T, VEC> x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = load_pack<T, VEC>(win + (size_t)s_col[k + u] * ld + col);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const T a = s_val[k + u];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = fma(a, x[u].v[e], acc[e]);
                }
            }
            for (; k < kend; ++k) {
                const Pack<T, VEC> x = load_pack<T, VEC>(win + (size_t)s_col[k] * ld + col);
                const T a = s_val[k];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = fma(a, x.v[e], acc[e]);
            }
        } else {
            for (int base = beg; base < end; base += 8) {
                int cidx[8];
                T a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    cidx[u] = row;
                    a[u] = T(0);
                    if (base + u < end) {
                        cidx[u] = col_idx[base + u];
                        a[u] = val[base + u];
                    }
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    if (base + u < end) {
                        const Pack<T, VEC> x = load_pack<T, VEC>(win + (size_t)cidx[u] * ld + col);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[e] = fma(a[u], x.v[e], acc[e]);
                    }
                }
            }
        }
        }   // CSR
        const Pack<T, VEC> w = load_pack<T, VEC>(win + (size_t)row * ld + col);
        Pack<T, VEC> o;
#pragma unroll
        for (int e = 0; e < VEC; ++e) o.v[e] = alpha * acc[e] - beta * w.v[e];
        if constexpr (KIND == STEP_HORNER_SIGNS) {
            const uint64_t bits = mask[row];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T sgn = ((bits >> ((col + gshift + e) & 63)) & 1ull) ? T(-1) : T(1);
                o.v[e] = fma(dj, sgn, o.v[e]);
            }
        } else if constexpr (KIND == STEP_HORNER_VEC) {
            const Pack<T, VEC> v = load_pack<T, VEC>(vsrc + (size_t)row * ldv + col);
#pragma unroll
            for (int e = 0; e < VEC; ++e) o.v[e] = fma(dj, v.v[e], o.v[e]);
        } else if constexpr (KIND == STEP_DOT_FWD) {
            const Pack<T, VEC> x = load_pack<T, VEC>(vsrc + (size_t)row * ldv + col);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if (FIRST) s0[e] += (double)x.v[e] * (double)w.v[e];
                s1[e] += (double)x.v[e] * (double)o.v[e];
            }
        } else if constexpr (KIND == STEP_DOT_SQ) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                if (FIRST) s0[e] += (double)w.v[e] * (double)w.v[e];
                s1[e] += (double)w.v[e] * (double)o.v[e];
                s2[e] += (double)o.v[e] * (double)o.v[e];
            }
        } else if constexpr (KIND == STEP_ACC_NORM) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) s1[e] += (double)o.v[e] * (double)o.v[e];
        }
        if constexpr (KIND == STEP_PLAIN_ACC || KIND == STEP_ACC_NORM) {
            if (col < acc_cols) {
                // ACC_NORM: only the columns still active in Alg. 2's loop accumulate
                const uint64_t bits = KIND == STEP_ACC_NORM ? *active : ~0ull;
                T* const pa = accum + (size_t)row * ldacc + col;
                const Pack<T, VEC> a0 = load_pack<T, VEC>(pa);
                Pack<T, VEC> a1;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int b = col - c0 + e;
                    const bool on = KIND == STEP_PLAIN_ACC || (b < 64 && ((bits >> (b & 63)) & 1ull));
                    a1.v[e] = on ? fma(dj, o.v[e], a0.v[e]) : a0.v[e];
                }
                store_pack<T, VEC>(pa, a1);
            }
        }
        // Every lane stores its whole vector: ld and c0 are multiples of VEC, so
        // the vector never leaves the row, and columns past c0+bcols in it get
        // the value of the same recurrence (real columns of a wider block, or
        // padding that no one reads).
        if (nt_out)
            store_pack_nt<T, VEC>(wout + (size_t)row * ld + col, o);
        else
            store_pack<T, VEC>(wout + (size_t)row * ld + col, o);
    }
    }   // tiles

    if constexpr (kDot) {
        // 1) per wave: the row groups' sums of each column, in group order
        double* const lanes = reinterpret_cast<double*>(s_wave[wave]);   // staging is dead
        int q = 0;
        auto wave_sum = [&](const double (&v)[VEC]) __attribute__((always_inline)) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) lanes[lane * VEC + e] = v[e];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int t = lane; t < bcols; t += 64) {
                const int tl = t / VEC, te = t - tl * VEC;
                double acc = 0.0;
                for (int gg = 0; gg < rpw; ++gg) acc += lanes[(gg * lpr + tl) * VEC + te];
                s_cols[(wave * kSums + q) * kMaxDotCols + t] = acc;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            ++q;
        };
        if constexpr (FIRST) wave_sum(s0);
        wave_sum(s1);
        if constexpr (KIND == STEP_DOT_SQ) wave_sum(s2);
        // 2) the last wave of the workgroup to get here adds the wave sums in
        //    wave order and writes the workgroup's partial row
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        unsigned ticket = 0;
        if (lane == 0) ticket = atomicAdd(&s_count, 1u);
        ticket = __shfl(ticket, 0, 64);
        if (ticket == NW - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            double* const outs[3] = {FIRST ? ps0 : ps1, FIRST ? ps1 : ps2, ps2};
            for (int t = lane; t < kSums * bcols; t += 64) {
                const int qq = t / bcols, cc = t - qq * bcols;
                double acc = 0.0;
#pragma unroll
                for (int wv = 0; wv < NW; ++wv) acc += s_cols[(wv * kSums + qq) * kMaxDotCols + cc];
                double* const dst = qq == 0 ? outs[0] : (qq == 1 ? outs[1] : outs[2]);
                const size_t at = (size_t)blockIdx.x * part_ld + c0 + gshift + cc;
                dst[at] = add_parts ? dst[at] + acc : acc;   // later row ranges of one step add on
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Long rows: one workgroup per row (grid-stride over the list).  The row's
// entries are dealt round-robin to the workgroup's row groups, each group
// gathers and accumulates its share, and the group sums are added in group
// order through LDS.  Column sums accumulate over the workgroup's rows and go
// to partial row part_row0 + blockIdx.x.
// ---------------------------------------------------------------------------
template <typename T, int VEC, int KIND, bool FIRST>
__global__ __launch_bounds__(256) void long_row_kernel(
    int n, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
    const T* __restrict__ val, const T* __restrict__ win, T* __restrict__ wout, int ld, int c0,
    int bcols, int gshift, T alpha, T beta, T dj, const T* __restrict__ vsrc, int ldv,
    const uint64_t* __restrict__ mask, double* __restrict__ ps0, double* __restrict__ ps1,
    double* __restrict__ ps2, int part_ld, int lpr, int rpw, const int* __restrict__ list,
    const int* __restrict__ count, int part_row0, T* __restrict__ accum, int ldacc, int acc_cols,
    const uint64_t* __restrict__ active) {
    constexpr int NW = 4;
    __shared__ T s_acc[NW * 64 * VEC];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane / lpr;
    const int li = lane - g * lpr;
    const bool lane_ok = g < rpw;
    const int col = c0 + li * VEC;
    const int groups = NW * rpw;
    const int gid = wave * rpw + g;
    const int nlong = *count;
    double s0[VEC], s1[VEC], s2[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) s0[e] = s1[e] = s2[e] = 0.0;
    for (int i = blockIdx.x; i < nlong; i += gridDim.x) {
        const int row = list[i];
        const int beg = row_ptr[row], end = row_ptr[row + 1];
        T acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = T(0);
        if (lane_ok) {
            int k = beg + gid;
            for (; k + 3 * groups < end; k += 4 * groups) {
                int cc[4];
                T aa[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    cc[u] = col_idx[k + u * groups];
                    aa[u] = val[k + u * groups];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const Pack<T, VEC> x = load_pack<T, VEC>(win + (size_t)cc[u] * ld + col);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) acc[e] = fma(aa[u], x.v[e], acc[e]);
                }
            }
            for (; k < end; k += groups) {
                const Pack<T, VEC> x = load_pack<T, VEC>(win + (size_t)col_idx[k] * ld + col);
                const T a = val[k];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = fma(a, x.v[e], acc[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) s_acc[threadIdx.x * VEC + e] = acc[e];
        __syncthreads();
        if (wave == 0 && g == 0) {
            // group sums in group order, then the Newton update of the row
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                T t = T(0);
                for (int q = 0; q < groups; ++q) {
                    const int wv = q / rpw, gg = q - wv * rpw;
                    t += s_acc[(wv * 64 + gg * lpr + li) * VEC + e];
                }
                acc[e] = t;
            }
            const Pack<T, VEC> w = load_pack<T, VEC>(win + (size_t)row * ld + col);
            Pack<T, VEC> o;
#pragma unroll
            for (int e = 0; e < VEC; ++e) o.v[e] = alpha * acc[e] - beta * w.v[e];
            if constexpr (KIND == STEP_HORNER_SIGNS) {
                const uint64_t bits = mask[row];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T sgn = ((bits >> ((col + gshift + e) & 63)) & 1ull) ? T(-1) : T(1);
                    o.v[e] = fma(dj, sgn, o.v[e]);
                }
            } else if constexpr (KIND == STEP_HORNER_VEC) {
                const Pack<T, VEC> v = load_pack<T, VEC>(vsrc + (size_t)row * ldv + col);
#pragma unroll
                for (int e = 0; e < VEC; ++e) o.v[e] = fma(dj, v.v[e], o.v[e]);
            } else if constexpr (KIND == STEP_DOT_FWD) {
                const Pack<T, VEC> x = load_pack<T, VEC>(vsrc + (size_t)row * ldv + col);
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    if (FIRST) s0[e] += (double)x.v[e] * (double)w.v[e];
                    s1[e] += (double)x.v[e] * (double)o.v[e];
                }
            } else if constexpr (KIND == STEP_DOT_SQ) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    if (FIRST) s0[e] += (double)w.v[e] * (double)w.v[e];
                    s1[e] += (double)w.v[e] * (double)o.v[e];
                    s2[e] += (double)o.v[e] * (double)o.v[e];
                }
            } else if constexpr (KIND == STEP_ACC_NORM) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) s1[e] += (double)o.v[e] * (double)o.v[e];
            }
            if constexpr (KIND == STEP_PLAIN_ACC || KIND == STEP_ACC_NORM) {
                if (col < acc_cols) {
                    const uint64_t bits = KIND == STEP_ACC_NORM ? *active : ~0ull;
                    T* const pa = accum + (size_t)row * ldacc + col;
                    const Pack<T, VEC> a0 = load_pack<T, VEC>(pa);
                    Pack<T, VEC> a1;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int b = col - c0 + e;
                        const bool on = KIND == STEP_PLAIN_ACC || (b < 64 && ((bits >> (b & 63)) & 1ull));
                        a1.v[e] = on ? fma(dj, o.v[e], a0.v[e]) : a0.v[e];
                    }
                    store_pack<T, VEC>(pa, a1);
                }
            }
            store_pack<T, VEC>(wout + (size_t)row * ld + col, o);
        }
        __syncthreads();
    }
    if constexpr (is_dot(KIND)) {
        if (wave == 0 && g == 0) {
            const size_t prow = (size_t)(part_row0 + blockIdx.x) * part_ld + c0 + gshift;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int t = li * VEC + e;
                if (t >= bcols) continue;
                if (FIRST) ps0[prow + t] = s0[e];
                ps1[prow + t] = s1[e];
                if (KIND == STEP_DOT_SQ) ps2[prow + t] = s2[e];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Newton step on the diagonal storage, kinds without column sums (HORNER_SIGNS,
// HORNER_VEC, PLAIN, PLAIN_ACC): one 16-byte chunk of a row per thread, chunk
// i = row*lpr + q over the whole block, so a wave's accesses are 64
// consecutive chunks (no idle lanes, one contiguous 1 KB run per load) and a
// workgroup is a single pass with no tile loop.  Measured on gfx950 at the
// 1024^2 bench shape (20 FP32 columns, constant diagonals): 28.5 us per step
// against 31.5 us for the row-group mapping of step_kernel, whose waves leave
// 64 mod lpr lanes idle.  The rows r +- 1 share cache lines with r and cost no
// extra traffic.  Per row the arithmetic and the order of the sums are those
// of step_kernel, so the results are the same bits.
// ---------------------------------------------------------------------------
template <typename T, int VEC, int KIND, int ND, bool PLANES>
__global__ __launch_bounds__(kThreads) void dia_flat_kernel(
    int n, const T* __restrict__ win, T* __restrict__ wout, int ld, int lpr, int gshift, T alpha, T beta, T dj,
    const T* __restrict__ vsrc, int ldv, const uint64_t* __restrict__ mask, T* __restrict__ accum, int ldacc,
    int acc_cols, const T* __restrict__ dia, int nd, DiaOff off, int interleave, int chunk, int nt_out,
    const uint16_t* __restrict__ dpres, DiaVal<T> cv, const uint8_t* __restrict__ planes) {
    static_assert(KIND == STEP_HORNER_SIGNS || KIND == STEP_HORNER_VEC || KIND == STEP_PLAIN ||
                  KIND == STEP_PLAIN_ACC, "kinds without column sums");
    unsigned blk = blockIdx.x;
    if (!interleave) {
        const unsigned x = blk % kXcds, i = blk / kXcds;   // the i-th workgroup dispatched to XCD x
        if (chunk > 0) {   // chunk c of `chunk` workgroups belongs to XCD c % 8, walked in order
            blk = ((i / (unsigned)chunk) * kXcds + x) * (unsigned)chunk + i % (unsigned)chunk;
        } else {           // XCD x takes the x-th contiguous band of workgroups
            const unsigned per = gridDim.x / kXcds;   // the grid is a multiple of 8
            blk = x * per + i;
        }
    }
    const unsigned i = blk * kThreads + threadIdx.x;
    if (i >= (unsigned)n * (unsigned)lpr) return;   // the launch checks n * lpr < 2^31
    const int row = (int)(i / (unsigned)lpr);
    const int col = (int)(i - (unsigned)row * (unsigned)lpr) * VEC;
    // HORNER_SIGNS from byte planes: the chunk's VEC columns start at a
    // multiple of VEC, so their sign bits lie in one byte of the row's word,
    // read from its plane (issued up front)
    unsigned sbits = 0;
    if constexpr (KIND == STEP_HORNER_SIGNS && PLANES) {
        const int g = col + gshift;
        sbits = (unsigned)planes[(size_t)((g >> 3) & 7) * n + row] >> (g & 7);
    }
    int cq[ND];
    T aq[ND];
    const unsigned pbits = dpres ? dpres[row] : 0u;
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        const int c = row + off.o[q];
        const bool ok = q < nd && (unsigned)c < (unsigned)n;
        cq[q] = ok ? c : row;
        if (dpres)
            aq[q] = ok && ((pbits >> q) & 1u) ? cv.c[q] : T(0);
        else
            aq[q] = ok ? (nt_out ? __builtin_nontemporal_load(dia + (size_t)row * nd + q) : dia[(size_t)row * nd + q])
                       : T(0);
    }
    Pack<T, VEC> xq[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q) xq[q] = load_pack<T, VEC>(win + (size_t)cq[q] * ld + col);
    T acc[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = T(0);
#pragma unroll
    for (int q = 0; q < ND; ++q) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = fma(aq[q], xq[q].v[e], acc[e]);
    }
    const Pack<T, VEC> w = load_pack<T, VEC>(win + (size_t)row * ld + col);
    Pack<T, VEC> o;
#pragma unroll
    for (int e = 0; e < VEC; ++e) o.v[e] = alpha * acc[e] - beta * w.v[e];
    if constexpr (KIND == STEP_HORNER_SIGNS && PLANES) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T sgn = ((sbits >> e) & 1u) ? T(-1) : T(1);
            o.v[e] = fma(dj, sgn, o.v[e]);
        }
    } else if constexpr (KIND == STEP_HORNER_SIGNS) {
        const uint64_t bits = mask[row];
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T sgn = ((bits >> ((col + gshift + e) & 63)) & 1ull) ? T(-1) : T(1);
            o.v[e] = fma(dj, sgn, o.v[e]);
        }
    } else if constexpr (KIND == STEP_HORNER_VEC) {
        const Pack<T, VEC> v = load_pack<T, VEC>(vsrc + (size_t)row * ldv + col);
#pragma unroll
        for (int e = 0; e < VEC; ++e) o.v[e] = fma(dj, v.v[e], o.v[e]);
    } else if constexpr (KIND == STEP_PLAIN_ACC) {
        if (col < acc_cols) {
            T* const pa = accum + (size_t)row * ldacc + col;
            const Pack<T, VEC> a0 = load_pack<T, VEC>(pa);
            Pack<T, VEC> a1;
#pragma unroll
            for (int e = 0; e < VEC; ++e) a1.v[e] = fma(dj, o.v[e], a0.v[e]);
            store_pack<T, VEC>(pa, a1);
        }
    }
    if (nt_out)
        store_pack_nt<T, VEC>(wout + (size_t)row * ld + col, o);
    else
        store_pack<T, VEC>(wout + (size_t)row * ld + col, o);
}

// Workgroups of a kernel that are resident at once on the device (blocks per
// CU at full occupancy x CUs), at most kDotWgs; cached per kernel (one device).
int resident_wgs(const void* fn, int nt) {
    static std::mutex mu;
    static std::unordered_map<const void*, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    const auto it = cache.find(fn);
    if (it != cache.end()) return it->second;
    int dev = 0, cus = 0, per_cu = 0;
    int r = kDotWgs;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) == hipSuccess && per_cu > 0 && cus > 0)
        r = std::max(kXcds, std::min(kDotWgs, per_cu * cus));
    cache[fn] = r;
    return r;
}

template <typename T, int VEC, int KIND, bool FIRST>
hipError_t launch_step_t(const CsrDev& A, const StepArgs& s, hipStream_t st, int* nwg_out) {
    constexpr int kIters = kStepIters;
    constexpr int NT = threads_of(KIND);
    if (nwg_out) *nwg_out = 0;
    if (is_dot(KIND) && s.bcols > kMaxDotCols) return hipErrorInvalidValue;
    const int lpr = lanes_per_row(s.bcols, VEC);
    if (lpr > 64) return hipErrorInvalidValue;
    const int rpw = 64 / lpr;
    const int rows_per_wg = (NT / 64) * rpw * kIters;
    const int ntiles = div_up(A.n, rows_per_wg);
    if (ntiles == 0) return hipSuccess;
    // the kinds with column sums run as many workgroups as are resident at once
    // (each loops over its tiles); the others one workgroup per tile.  The
    // occupancy is the smaller of the first and the other steps' variants, so
    // every step of a phase writes the same number of partial rows (they are
    // reduced together) and every launch's workgroups are all resident.
    // Measured at 20 and 22 FP32 columns (first step 78 VGPRs: 6 workgroups
    // per CU; the others 70: 7): the other steps' occupancy as the grid made
    // them slower, 34 -> 41 us at the 1024^2 bench shape and 205 -> 252 us on
    // the 2048^2 GMRF, with 96- or 48-row tiles alike; a grid balanced to
    // whole rounds of tiles (1368 workgroups) took 36.5 us.
    auto grid = [&](const void* fn_first, const void* fn_rest) {
        return is_dot(KIND) ? std::min({ntiles, resident_wgs(fn_first, NT), resident_wgs(fn_rest, NT)}) : ntiles;
    };
    // chunked bands: s.chunk_rows rows per chunk, in tiles (only when a chunk is
    // a whole number of tiles, so that an XCD's consecutive chunks lie exactly
    // chunk_rows * 8 rows apart; else contiguous bands)
    const int ctiles = s.chunk_rows > 0 && !s.interleave && s.chunk_rows % rows_per_wg == 0
                           ? s.chunk_rows / rows_per_wg
                           : 0;
    // A step with column sums that streams from HBM, on a stencil whose widest
    // offset reaches beyond a tile, goes in launches over consecutive row
    // ranges of at most kRangeTiles tiles per workgroup, each adding its sums
    // to the same partial rows: a persistent workgroup that walks many tiles
    // drifts away from the others, and the XCD's active rows then spread
    // beyond what its L2 holds of their neighbour rows.  Measured on gfx950
    // (FP32 quadratic-form step): 5000^2 GMRF, about 170 tiles per workgroup,
    // 1176 us in one launch, 1056 us at 24 or 48 tiles per range, 1125 us at
    // 12; ranges cost 2-3% where the workgroups walk few tiles or the
    // neighbours are near (2048^2 GMRF in one block, 28 tiles: 205 -> 209 us at
    // 24; pentadiagonal n = 10^7: 412 -> 425 us).  XCD bands only; chunked
    // bands keep one launch.
    int reach = 0;
    for (int q = 0; q < s.dia_nd && q < kMaxDiag; ++q) reach = std::max(reach, std::abs(s.dia_off[q]));
    auto row_ranges = [&](int nwg) {
        if (!is_dot(KIND) || !s.nt_out || s.interleave || ctiles > 0 || reach <= rows_per_wg || nwg <= 0) return 1;
        return std::max(1, div_up(div_up(ntiles, nwg), kRangeTiles));
    };
    DiaOff off{};
    for (int q = 0; q < kMaxDiag; ++q) off.o[q] = q < s.dia_nd ? s.dia_off[q] : 0;
    DiaVal<T> cv{};
    for (int q = 0; q < kMaxDiag; ++q) cv.c[q] = (T)(q < s.dia_nd ? s.dia_cval[q] : 0.0);
    if (s.dia_nd > 0) {   // no row has more than kMaxDiag entries: no long rows either
        if (s.dia_nd > kMaxDiag || !s.dia) return hipErrorInvalidValue;
        constexpr bool kFlat = !is_dot(KIND) && KIND != STEP_ACC_NORM && VEC * sizeof(T) == 16;
        if constexpr (kFlat) {
            // one chunk per thread (the column range starts at c0 = 0 or at a
            // whole number of chunks: the chunk index counts from c0)
            const long long chunks = (long long)A.n * lpr;
            if (chunks < (1LL << 31)) {
                const int need = div_up(chunks, kThreads);
                // chunked bands: s.chunk_rows rows per chunk, in workgroups; the grid
                // covers whole rounds of 8 chunks (workgroups past the end return)
                // (only when a chunk is a whole number of workgroups: otherwise the
                // XCD's consecutive chunks would not lie a stencil offset apart)
                const int cwg = s.chunk_rows > 0 && !s.interleave && (long long)s.chunk_rows * lpr % kThreads == 0
                                    ? (int)((long long)s.chunk_rows * lpr / kThreads)
                                    : 0;
                const int nwg = cwg > 0 ? div_up(div_up(need, cwg), kXcds) * kXcds * cwg
                                        : div_up(need, kXcds) * kXcds;
                // byte planes of the sign words (HORNER_SIGNS): a chunk's columns must
                // start at a multiple of VEC (then they lie in one byte)
                const uint8_t* const planes =
                    KIND == STEP_HORNER_SIGNS && (s.gshift + s.c0) % VEC == 0 ? s.planes : nullptr;
#define LD_FLAT_LAUNCH_P(ND_, P_)                                                                              \
    hipLaunchKernelGGL((dia_flat_kernel<T, VEC, KIND, ND_, P_>), dim3(nwg), dim3(kThreads), 0, st, A.n,       \
                       (const T*)s.win + s.c0, (T*)s.wout + s.c0, s.ld, lpr, s.gshift + s.c0, (T)s.alpha,     \
                       (T)s.beta, (T)s.dj, s.vsrc ? (const T*)s.vsrc + s.c0 : nullptr, s.ldv, s.mask,         \
                       s.acc ? (T*)s.acc + s.c0 : nullptr, s.ldacc, s.acc_cols - s.c0, (const T*)s.dia,        \
                       s.dia_nd, off, s.interleave, cwg, s.nt_out, s.dia_pres, cv, planes)
#define LD_FLAT_LAUNCH(ND_)                                                                                    \
    do {                                                                                                       \
        if (planes)                                                                                            \
            LD_FLAT_LAUNCH_P(ND_, KIND == STEP_HORNER_SIGNS);                                                  \
        else                                                                                                   \
            LD_FLAT_LAUNCH_P(ND_, false);                                                                      \
    } while (0)
                if (s.dia_nd <= 3)
                    LD_FLAT_LAUNCH(3);
                else if (s.dia_nd <= 5)
                    LD_FLAT_LAUNCH(5);
                else if (s.dia_nd <= 7)
                    LD_FLAT_LAUNCH(7);
                else
                    LD_FLAT_LAUNCH(9);
#undef LD_FLAT_LAUNCH
#undef LD_FLAT_LAUNCH_P
                if (nwg_out) *nwg_out = 0;   // no partial rows
                return hipGetLastError();
            }
        }
#define LD_DIA_LAUNCH(ND_)                                                                                     \
    {                                                                                                          \
        const auto fn = step_kernel<T, VEC, KIND, FIRST, kIters, NT, ND_>;                                     \
        const int nwg = grid(reinterpret_cast<const void*>(step_kernel<T, VEC, KIND, has_first(KIND), kIters, NT, ND_>), \
                             reinterpret_cast<const void*>(step_kernel<T, VEC, KIND, false, kIters, NT, ND_>));  \
        const int nsub = row_ranges(nwg);                                                                      \
        for (int k = 0; k < nsub; ++k) {                                                                       \
            const int t0 = (int)((long long)ntiles * k / nsub), t1 = (int)((long long)ntiles * (k + 1) / nsub); \
            hipLaunchKernelGGL(fn, dim3(nwg), dim3(NT), 0, st, A.n, A.row_ptr, A.col_idx, (const T*)A.val,     \
                               (const T*)s.win, (T*)s.wout, s.ld, s.c0, s.bcols, s.gshift, (T)s.alpha,         \
                               (T)s.beta, (T)s.dj, (const T*)s.vsrc, s.ldv, s.mask, s.ps0, s.ps1, s.ps2,       \
                               s.part_ld, lpr, rpw, 0, (T*)s.acc, s.ldacc, s.acc_cols, t1 - t0, s.active,      \
                               (const T*)s.dia, s.dia_nd, off, s.interleave, ctiles, s.nt_out, s.dia_pres, cv, \
                               t0, k > 0 ? 1 : 0);                                                            \
        }                                                                                                      \
        if (nwg_out) *nwg_out = nwg;                                                                           \
        if (s.ranges_out) *s.ranges_out = nsub;                                                                \
    }
        if (s.dia_nd <= 3)
            LD_DIA_LAUNCH(3)
        else if (s.dia_nd <= 5)
            LD_DIA_LAUNCH(5)
        else if (s.dia_nd <= 7)
            LD_DIA_LAUNCH(7)
        else
            LD_DIA_LAUNCH(9)
#undef LD_DIA_LAUNCH
        return hipGetLastError();
    }
    if (s.ranges_out) *s.ranges_out = 1;
    const int skip = s.long_rows != nullptr;
    const auto fn = step_kernel<T, VEC, KIND, FIRST, kIters, NT, 0>;
    const int nwg = grid(reinterpret_cast<const void*>(step_kernel<T, VEC, KIND, has_first(KIND), kIters, NT, 0>),
                         reinterpret_cast<const void*>(step_kernel<T, VEC, KIND, false, kIters, NT, 0>));
    if (nwg_out) *nwg_out = nwg + (skip ? kLongWgs : 0);
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(NT), 0, st,
                       A.n, A.row_ptr, A.col_idx, (const T*)A.val, (const T*)s.win, (T*)s.wout, s.ld,
                       s.c0, s.bcols, s.gshift, (T)s.alpha, (T)s.beta, (T)s.dj, (const T*)s.vsrc,
                       s.ldv, s.mask, s.ps0, s.ps1, s.ps2, s.part_ld, lpr, rpw, skip, (T*)s.acc,
                       s.ldacc, s.acc_cols, ntiles, s.active, (const T*)nullptr, 0, off, s.interleave, ctiles,
                       s.nt_out, (const uint16_t*)nullptr, cv, 0, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !skip) return e;
    hipLaunchKernelGGL((long_row_kernel<T, VEC, KIND, FIRST>), dim3(kLongWgs), dim3(256), 0, st,
                       A.n, A.row_ptr, A.col_idx, (const T*)A.val, (const T*)s.win, (T*)s.wout, s.ld,
                       s.c0, s.bcols, s.gshift, (T)s.alpha, (T)s.beta, (T)s.dj, (const T*)s.vsrc,
                       s.ldv, s.mask, s.ps0, s.ps1, s.ps2, s.part_ld, lpr, rpw, s.long_rows,
                       s.long_count, nwg, (T*)s.acc, s.ldacc, s.acc_cols, s.active);
    return hipGetLastError();
}

template <typename T, int VEC>
hipError_t launch_step_v(const CsrDev& A, const StepArgs& s, hipStream_t st, int* nw) {
    switch (s.kind) {
        case STEP_HORNER_SIGNS: return launch_step_t<T, VEC, STEP_HORNER_SIGNS, false>(A, s, st, nw);
        case STEP_HORNER_VEC: return launch_step_t<T, VEC, STEP_HORNER_VEC, false>(A, s, st, nw);
        case STEP_PLAIN: return launch_step_t<T, VEC, STEP_PLAIN, false>(A, s, st, nw);
        case STEP_PLAIN_ACC: return launch_step_t<T, VEC, STEP_PLAIN_ACC, false>(A, s, st, nw);
        case STEP_ACC_NORM:
            if (!s.active || !s.acc) return hipErrorInvalidValue;
            return launch_step_t<T, VEC, STEP_ACC_NORM, false>(A, s, st, nw);
        case STEP_DOT_FWD:
            return s.first ? launch_step_t<T, VEC, STEP_DOT_FWD, true>(A, s, st, nw)
                           : launch_step_t<T, VEC, STEP_DOT_FWD, false>(A, s, st, nw);
        case STEP_DOT_SQ:
            return s.first ? launch_step_t<T, VEC, STEP_DOT_SQ, true>(A, s, st, nw)
                           : launch_step_t<T, VEC, STEP_DOT_SQ, false>(A, s, st, nw);
        default: return hipErrorInvalidValue;
    }
}

// widest vector (16 bytes max) compatible with the leading dimensions,
// column offset and pointer alignment
inline int pick_vec(const StepArgs& s, int elem_bytes) {
    int vec = 16 / elem_bytes;
    auto ok = [&](int v) {
        const uintptr_t align = (uintptr_t)v * elem_bytes;
        if (s.ld % v || s.c0 % v) return false;
        if ((uintptr_t)s.win % align || (uintptr_t)s.wout % align) return false;
        if (s.vsrc && (s.ldv % v || (uintptr_t)s.vsrc % align)) return false;
        if (s.acc && (s.ldacc % v || (uintptr_t)s.acc % align)) return false;
        return true;
    };
    while (vec > 1 && !ok(vec)) vec /= 2;
    return vec;
}

}  // namespace

int step_num_wg_bound(int n, int bcols, int elem_bytes) {
    // blocks aligned to the 16-byte vector (the estimator's internal layout),
    // plus the partial rows of the long-row launch
    const int rows = (threads_of(STEP_PLAIN) / 64) * (64 / lanes_per_row(bcols, 16 / elem_bytes)) * kStepIters;
    return grid_of(STEP_DOT_SQ, div_up(n, rows)) + kLongWgs;
}

int step_max_cols(bool f64, const StepArgs& s) { return 64 * pick_vec(s, f64 ? 8 : 4); }

int step_tile_rows(int bcols, int elem_bytes) {
    return (threads_of(STEP_DOT_SQ) / 64) * (64 / lanes_per_row(bcols, 16 / elem_bytes)) * kStepIters;
}

int step_num_wg_any(int n) {
    // any vector width and column count: at most 8 rows per tile, at most kDotWgs tiles' workgroups
    return grid_of(STEP_DOT_SQ, div_up(n, (threads_of(STEP_PLAIN) / 64) * kStepIters)) + kLongWgs;
}

hipError_t launch_step(bool f64, const CsrDev& A, const StepArgs& s, hipStream_t st, int* nwg_out) {
    if (f64) {
        const int vec = pick_vec(s, 8);
        return vec == 2 ? launch_step_v<double, 2>(A, s, st, nwg_out) : launch_step_v<double, 1>(A, s, st, nwg_out);
    }
    const int vec = pick_vec(s, 4);
    if (vec == 4) return launch_step_v<float, 4>(A, s, st, nwg_out);
    if (vec == 2) return launch_step_v<float, 2>(A, s, st, nwg_out);
    return launch_step_v<float, 1>(A, s, st, nwg_out);
}

// ---------------------------------------------------------------------------
// deterministic list of long rows: per-block counts, one-block scan, scatter
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void long_count_kernel(int n, const int* __restrict__ row_ptr,
                                                              int* __restrict__ cnt) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    const bool is_long = r < n && row_ptr[r + 1] - row_ptr[r] > kLongRow;
    __shared__ int s[kThreads / 64];
    const unsigned long long b = __ballot(is_long);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(b);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int i = 0; i < kThreads / 64; ++i) t += s[i];
        cnt[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void long_scan_kernel(int nb, int* __restrict__ cnt,
                                                         int* __restrict__ count) {
    // exclusive scan of cnt[0..nb) in place, one block: contiguous chunks per thread
    __shared__ int s[1024];
    const int per = (nb + 1023) / 1024;
    const int b0 = threadIdx.x * per, b1 = min(nb, b0 + per);
    int local = 0;
    for (int i = b0; i < b1; ++i) local += cnt[i];
    s[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    int run = s[threadIdx.x] - local;   // exclusive prefix of this chunk
    for (int i = b0; i < b1; ++i) {
        const int c = cnt[i];
        cnt[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *count = s[1023];
}

__global__ __launch_bounds__(kThreads) void long_scatter_kernel(int n, const int* __restrict__ row_ptr,
                                                                const int* __restrict__ off,
                                                                int* __restrict__ list) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    const bool is_long = r < n && row_ptr[r + 1] - row_ptr[r] > kLongRow;
    __shared__ int s[kThreads / 64];
    const unsigned long long b = __ballot(is_long);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s[wave] = __popcll(b);
    __syncthreads();
    int base = off[blockIdx.x];
    for (int i = 0; i < wave; ++i) base += s[i];
    if (is_long) list[base + __popcll(b & ((1ull << lane) - 1ull))] = r;
}

hipError_t launch_long_rows(const CsrDev& A, int* tmp, int* list, int* count, hipStream_t st) {
    const int nb = div_up(A.n, kThreads);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(long_count_kernel, dim3(nb), dim3(kThreads), 0, st, A.n, A.row_ptr, tmp);
    hipLaunchKernelGGL(long_scan_kernel, dim3(1), dim3(1024), 0, st, nb, tmp, count);
    hipLaunchKernelGGL(long_scatter_kernel, dim3(nb), dim3(kThreads), 0, st, A.n, A.row_ptr, tmp, list);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// probe signs
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void sign_mask_kernel(int n, int k, uint64_t key,
                                                             uint64_t* __restrict__ mask,
                                                             uint8_t* __restrict__ planes) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    uint64_t bits = 0;
    for (int c = 0; c < k; ++c) {
        const uint64_t x = probe_bits(key, (uint64_t)c * (uint64_t)n + (uint64_t)r + 1ull);
        bits |= (x >> 63) << c;
    }
    mask[r] = bits;
    if (planes)
        for (int p = 0; p < 8; ++p) planes[(size_t)p * n + r] = (uint8_t)(bits >> (8 * p));
}

hipError_t launch_sign_mask(int n, int k, uint64_t key, uint64_t* mask, hipStream_t st, uint8_t* planes) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(sign_mask_kernel, dim3(div_up(n, kThreads)), dim3(kThreads), 0, st, n, k,
                       key, mask, planes);
    return hipGetLastError();
}

// One thread per 16-byte chunk of a row (VEC columns): a vector store when the
// chunk lies inside [0, k) and out's rows are 16-byte aligned, else per column.
template <typename T>
__global__ __launch_bounds__(kThreads) void fill_signs_kernel(int n, int k, int ld, int gshift,
                                                              const uint64_t* __restrict__ mask,
                                                              T scale, T* __restrict__ out, int chunks,
                                                              int vec_ok) {
    constexpr int V = 16 / (int)sizeof(T);
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (long long)n * chunks) return;
    const int r = (int)(i / chunks), c0 = (int)(i - (long long)r * chunks) * V;
    const uint64_t w = mask[r];
    T* const dst = out + (size_t)r * ld + c0;
    if (vec_ok && c0 + V <= k) {
        Pack<T, V> p;
#pragma unroll
        for (int q = 0; q < V; ++q) p.v[q] = ((w >> ((c0 + q + gshift) & 63)) & 1ull) ? -scale : scale;
        store_pack<T, V>(dst, p);
    } else {
        for (int q = 0; q < V && c0 + q < k; ++q) dst[q] = ((w >> ((c0 + q + gshift) & 63)) & 1ull) ? -scale : scale;
    }
}

// Gaussian probe entries: one thread per row of a column (grid.y = column).
template <typename T>
__global__ __launch_bounds__(kThreads) void gauss_fill_kernel(int n, uint64_t key, int col0, double scale,
                                                              T* __restrict__ out, Blk bo) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= n) return;
    const uint64_t x = probe_bits(key, (uint64_t)(c + col0) * (uint64_t)n + (uint64_t)r + 1ull);
    const double u1 = ((double)(x >> 32) + 0.5) * 0x1p-32;
    const double u2 = ((double)(x & 0xFFFFFFFFull) + 0.5) * 0x1p-32;
    const double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    out[bo.offset(c) + (size_t)r * bo.ld] = (T)(scale * g);
}

hipError_t launch_gauss_fill(bool f64, int n, int k, uint64_t key, int col0, double scale, void* out, Blk bo,
                             hipStream_t st) {
    if ((long long)n * k == 0) return hipSuccess;
    if (k > 65535) return hipErrorInvalidValue;
    const dim3 grid(div_up(n, kThreads), k);
    if (f64)
        hipLaunchKernelGGL(gauss_fill_kernel<double>, grid, dim3(kThreads), 0, st, n, key, col0, scale,
                           (double*)out, bo);
    else
        hipLaunchKernelGGL(gauss_fill_kernel<float>, grid, dim3(kThreads), 0, st, n, key, col0, scale,
                           (float*)out, bo);
    return hipGetLastError();
}

hipError_t launch_fill_signs(bool f64, int n, int k, int ld, int gshift, const uint64_t* mask,
                             double scale, void* out, hipStream_t st) {
    if ((long long)n * k == 0) return hipSuccess;
    const int v = f64 ? 2 : 4;
    const int chunks = (k + v - 1) / v;
    const int vec_ok = ((uintptr_t)out % 16 == 0) && ld % v == 0;
    const int nb = div_up((long long)n * chunks, kThreads);
    if (f64)
        hipLaunchKernelGGL(fill_signs_kernel<double>, dim3(nb), dim3(kThreads), 0, st, n, k, ld,
                           gshift, mask, scale, (double*)out, chunks, vec_ok);
    else
        hipLaunchKernelGGL(fill_signs_kernel<float>, dim3(nb), dim3(kThreads), 0, st, n, k, ld,
                           gshift, mask, (float)scale, (float*)out, chunks, vec_ok);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void scale_copy_kernel(int n, int ncols,
                                                              const T* __restrict__ V, int ldv,
                                                              T scale, T* __restrict__ out,
                                                              int ldo) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= (long long)n * ncols) return;
    const int r = (int)(i / ncols), c = (int)(i - (long long)r * ncols);
    out[(size_t)r * ldo + c] = scale * V[(size_t)r * ldv + c];
}

hipError_t launch_scale_copy(bool f64, int n, int ncols, const void* V, int ldv, double scale,
                             void* out, int ldo, hipStream_t st) {
    const long long tot = (long long)n * ncols;
    if (tot == 0) return hipSuccess;
    const int nb = div_up(tot, kThreads);
    if (f64)
        hipLaunchKernelGGL(scale_copy_kernel<double>, dim3(nb), dim3(kThreads), 0, st, n, ncols,
                           (const double*)V, ldv, scale, (double*)out, ldo);
    else
        hipLaunchKernelGGL(scale_copy_kernel<float>, dim3(nb), dim3(kThreads), 0, st, n, ncols,
                           (const float*)V, ldv, (float)scale, (float*)out, ldo);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// X^T Z on FP64 MFMA (v_mfma_f64_16x16x4_f64).  Operand layout of the 16x16x4
// instruction: lane l holds A[l%16][l/16] and B[l/16][l%16]; the 16x16 result
// has D[l/16 + 4v][l%16] in accumulator element v (checked on gfx950).  With
// A = X^T and B = Z over a chunk of 4 rows, lane l simply loads
// X[r0 + l/16][16*t + l%16].
// ---------------------------------------------------------------------------
constexpr int kCrossRows = 256;    // rows per tile
constexpr int kCrossWgs = 2048;    // workgroups of a launch at most (each loops over tiles)
constexpr int kCrossChunks = 4;    // 4-row chunks a wave loads before their MFMAs

typedef double double4_t __attribute__((ext_vector_type(4)));

// SAME: Z is X (a Gram matrix): one load feeds both operands.
template <typename T, int TX, int TZ, bool ZSIGNS, bool SAME>
__global__ __launch_bounds__(kThreads) void cross_kernel(int n, const T* __restrict__ X, Blk bx,
                                                         int kx, const T* __restrict__ Z, Blk bz,
                                                         int kz, const uint64_t* __restrict__ zmask,
                                                         double* __restrict__ part) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int sub = lane >> 4;       // row within a chunk of 4
    const int cit = lane & 15;       // column within a 16-wide tile
    double4_t acc[TX][TZ];
#pragma unroll
    for (int a = 0; a < TX; ++a)
#pragma unroll
        for (int b = 0; b < TZ; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};

    size_t xoff[TX], zoff[TZ];
#pragma unroll
    for (int a = 0; a < TX; ++a) xoff[a] = bx.offset(a * 16 + cit);
#pragma unroll
    for (int b = 0; b < TZ; ++b) zoff[b] = (ZSIGNS || SAME) ? 0 : bz.offset(b * 16 + cit);
    const int ntiles = div_up_dev(n, kCrossRows);
    constexpr int kStep = kWaves * 4 * kCrossChunks;   // rows of one pass of the workgroup
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int row0 = tile * kCrossRows;
        const int row1 = min(row0 + kCrossRows, n);
        for (int r0 = row0 + wave * 4 * kCrossChunks; r0 < row1; r0 += kStep) {
            double xa[kCrossChunks][TX], zb[kCrossChunks][TZ];
#pragma unroll
            for (int h = 0; h < kCrossChunks; ++h) {
                const int r = r0 + 4 * h + sub;
                const bool rok = r < row1;
#pragma unroll
                for (int a = 0; a < TX; ++a) {
                    const int c = a * 16 + cit;
                    xa[h][a] = (rok && c < kx) ? (double)X[xoff[a] + (size_t)r * bx.ld] : 0.0;
                }
                if constexpr (!SAME) {
#pragma unroll
                    for (int b = 0; b < TZ; ++b) {
                        const int c = b * 16 + cit;
                        double z = 0.0;
                        if (rok && c < kz) {
                            if constexpr (ZSIGNS) {
                                z = ((zmask[r] >> c) & 1ull) ? -1.0 : 1.0;
                            } else {
                                z = (double)Z[zoff[b] + (size_t)r * bz.ld];
                            }
                        }
                        zb[h][b] = z;
                    }
                }
            }
#pragma unroll
            for (int h = 0; h < kCrossChunks; ++h)
#pragma unroll
                for (int a = 0; a < TX; ++a)
#pragma unroll
                    for (int b = 0; b < TZ; ++b)
                        if (!SAME || a <= b)   // a Gram matrix: the tiles below the diagonal are mirrors
                            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                xa[h][a], SAME ? xa[h][b] : zb[h][b], acc[a][b], 0, 0, 0);
        }
    }

    // sum the four waves in a fixed order through LDS
    __shared__ double sh[TX * TZ * 256];
    for (int wv = 0; wv < kWaves; ++wv) {
        if (wave == wv) {
#pragma unroll
            for (int a = 0; a < TX; ++a)
#pragma unroll
                for (int b = 0; b < TZ; ++b)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = ((a * TZ + b) * 4 + v) * 64 + lane;
                        sh[idx] = (wv == 0) ? acc[a][b][v] : sh[idx] + acc[a][b][v];
                    }
        }
        __syncthreads();
    }
    // scatter to part[workgroup][i*kz + j]; element (il, jl) of tile (a, b) sits at
    // lane 16*(il%4) + jl, accumulator element il/4
    for (int e = threadIdx.x; e < TX * TZ * 256; e += kThreads) {
        const int l = e & 63;
        const int v = (e >> 6) & 3;
        const int ab = e >> 8;
        const int a = ab / TZ, b = ab - a * TZ;
        const int il = (l >> 4) + 4 * v, jl = l & 15;
        const int i = a * 16 + il;
        const int j = b * 16 + jl;
        if (i >= kx || j >= kz) continue;
        double val;
        if (SAME && a > b)   // mirror of element (jl, il) of tile (b, a)
            val = sh[((b * TZ + a) * 4 + jl / 4) * 64 + 16 * (jl % 4) + il];
        else
            val = sh[e];
        part[(size_t)blockIdx.x * kx * kz + i * kz + j] = val;
    }
}

template <typename T, int TX, int TZ>
hipError_t launch_cross_t(int n, const void* X, Blk bx, int kx, const void* Z, Blk bz, int kz,
                          const uint64_t* zmask, double* part, hipStream_t st) {
    const bool zsigns = zmask != nullptr;
    const int nwg = cross_num_wg(n);
    if (nwg == 0) return hipSuccess;
    const bool same = !zsigns && X == Z && kx == kz && bx.ld == bz.ld && bx.bw == bz.bw &&
                      bx.bstride == bz.bstride && bx.c0 == bz.c0;
    if (zsigns)
        hipLaunchKernelGGL((cross_kernel<T, TX, TZ, true, false>), dim3(nwg), dim3(kThreads), 0, st, n,
                           (const T*)X, bx, kx, (const T*)Z, bz, kz, zmask, part);
    else if (same && TX == TZ)
        hipLaunchKernelGGL((cross_kernel<T, TX, TZ, false, TX == TZ>), dim3(nwg), dim3(kThreads), 0, st, n,
                           (const T*)X, bx, kx, (const T*)Z, bz, kz, zmask, part);
    else
        hipLaunchKernelGGL((cross_kernel<T, TX, TZ, false, false>), dim3(nwg), dim3(kThreads), 0, st, n,
                           (const T*)X, bx, kx, (const T*)Z, bz, kz, zmask, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cross_tx(int n, const void* X, Blk bx, int kx, const void* Z, Blk bz, int kz,
                           const uint64_t* zmask, double* part, hipStream_t st) {
    const int tx = (kx + 15) / 16, tz = (kz + 15) / 16;
#define LD_CROSS_CASE(A, B) \
    if (tx == A && tz == B) return launch_cross_t<T, A, B>(n, X, bx, kx, Z, bz, kz, zmask, part, st);
    LD_CROSS_CASE(1, 1) LD_CROSS_CASE(1, 2) LD_CROSS_CASE(1, 3) LD_CROSS_CASE(1, 4)
    LD_CROSS_CASE(2, 1) LD_CROSS_CASE(2, 2) LD_CROSS_CASE(2, 3) LD_CROSS_CASE(2, 4)
    LD_CROSS_CASE(3, 1) LD_CROSS_CASE(3, 2) LD_CROSS_CASE(3, 3) LD_CROSS_CASE(3, 4)
    LD_CROSS_CASE(4, 1) LD_CROSS_CASE(4, 2) LD_CROSS_CASE(4, 3) LD_CROSS_CASE(4, 4)
#undef LD_CROSS_CASE
    return hipErrorInvalidValue;
}

int cross_num_wg(int n) { return (int)std::min<long long>(div_up(n, kCrossRows), kCrossWgs); }

// ---------------------------------------------------------------------------
// Narrow cross products (kx, kz <= 32) from LDS-staged tiles on the FP64
// vector units.  A tile of RT rows is staged whole (X's block rows with
// 16-byte vectors; probe signs expanded once per row from its sign word), and each
// thread accumulates one 4x4 block of X^T Z in FP64 over a fixed subset of
// the tile's rows (its phase).  The phases are summed in order at the end,
// so partial row wg (one per workgroup, as cross_kernel's) is repeatable.
// At 20 columns the FP64 MFMA tiles of cross_kernel are 61% padding; here
// the padding is at most 3 columns per side.
// ---------------------------------------------------------------------------
constexpr int kGramMaxK = 32;
constexpr int kGramKS = kGramMaxK + 5;   // LDS row stride: odd, and room for a 4-column block past a view's end

template <typename T, bool SAME, bool ZSIGNS, int RT>
__global__ __launch_bounds__(kThreads) void gram_kernel(int n, const T* __restrict__ X, Blk bx, int kx,
                                                        const T* __restrict__ Z, Blk bz, int kz,
                                                        const uint64_t* __restrict__ zmask, double* __restrict__ part) {
    constexpr int V = 16 / (int)sizeof(T);
    using P = Pack<T, V>;
    constexpr int NV = (RT * kGramMaxK / V + kThreads - 1) / kThreads;   // vectors per thread and tile
    constexpr int kTileBytes = (SAME ? 1 : 2) * RT * kGramKS * (int)sizeof(T);
    constexpr int kRedBytes = kThreads * 17 * 8;
    __shared__ __align__(16) unsigned char smem[kTileBytes > kRedBytes ? kTileBytes : kRedBytes];
    T* const xs = reinterpret_cast<T*>(smem);
    T* const zs = SAME ? xs : xs + RT * kGramKS;
    double* const red = reinterpret_cast<double*>(smem);

    const int tid = threadIdx.x;
    const int bix = (kx + 3) / 4, biz = (kz + 3) / 4;
    const int nblk = SAME ? bix * (bix + 1) / 2 : bix * biz;
    const int nph = kThreads / nblk;   // row phases, >= 4
    const int blk = tid % nblk, phase = tid / nblk;
    int bi, bj;
    if (SAME) {   // upper-triangular blocks in row order
        int b = blk;
        bi = 0;
        while (b >= bix - bi) {
            b -= bix - bi;
            ++bi;
        }
        bj = bi + b;
    } else {
        bi = blk / biz;
        bj = blk - bi * biz;
    }
    const int ldx = bx.ld, cx = bx.c0 % bx.bw;
    const T* const xblk = X + (size_t)(bx.c0 / bx.bw) * (size_t)bx.bstride;
    const int ldz = bz.ld, cz = (SAME || ZSIGNS) ? 0 : bz.c0 % bz.bw;
    const T* const zblk = (SAME || ZSIGNS) ? nullptr : Z + (size_t)(bz.c0 / bz.bw) * (size_t)bz.bstride;
    const int xcol = cx + 4 * bi, zcol = (SAME ? cx : cz) + 4 * bj;

    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const int ntiles = div_up_dev(n, RT);
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int row0 = t * RT, nr = min(RT, n - row0);
        {   // X's block rows [row0, row0 + nr), whole
            const int nvec = nr * ldx / V;
            const T* src = xblk + (size_t)row0 * ldx;
            P v[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = tid + u * kThreads;
                if (e < nvec) v[u] = load_pack<T, V>(src + (size_t)e * V);
            }
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = tid + u * kThreads;
                if (e < nvec) {
                    const int x = e * V, r = x / ldx, c = x - r * ldx;
#pragma unroll
                    for (int q = 0; q < V; ++q) xs[r * kGramKS + c + q] = v[u].v[q];
                }
            }
        }
        if constexpr (ZSIGNS) {   // one thread per row expands the row's sign word
            for (int r = tid; r < nr; r += kThreads) {
                const uint64_t w = zmask[row0 + r];
                for (int j = 0; j < kz; ++j) zs[r * kGramKS + j] = ((w >> j) & 1ull) ? T(-1) : T(1);
            }
        } else if constexpr (!SAME) {
            const int nvec = nr * ldz / V;
            const T* src = zblk + (size_t)row0 * ldz;
            P v[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = tid + u * kThreads;
                if (e < nvec) v[u] = load_pack<T, V>(src + (size_t)e * V);
            }
#pragma unroll
            for (int u = 0; u < NV; ++u) {
                const int e = tid + u * kThreads;
                if (e < nvec) {
                    const int x = e * V, r = x / ldz, c = x - r * ldz;
#pragma unroll
                    for (int q = 0; q < V; ++q) zs[r * kGramKS + c + q] = v[u].v[q];
                }
            }
        }
        __syncthreads();
        if (phase < nph) {
            for (int r = phase; r < nr; r += nph) {
                double xv[4], zv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xv[q] = (double)xs[r * kGramKS + xcol + q];
                    zv[q] = (double)zs[r * kGramKS + zcol + q];
                }
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a * 4 + b] = fma(xv[a], zv[b], acc[a * 4 + b]);
            }
        }
        __syncthreads();   // the tiles are restaged (or become the reduction buffer)
    }
    // phases of each block summed in order; entries past kx / kz are dropped
#pragma unroll
    for (int q = 0; q < 16; ++q) red[tid * 17 + q] = acc[q];
    __syncthreads();
    for (int e = tid; e < kx * kz; e += kThreads) {
        const int i = e / kz, j = e - i * kz;
        int a = i, b = j;
        if (SAME && a / 4 > b / 4) {   // below the diagonal blocks: the mirror entry
            a = j;
            b = i;
        }
        const int pi = a / 4, pj = b / 4;
        const int pb = SAME ? pi * bix - pi * (pi - 1) / 2 + (pj - pi) : pi * biz + pj;
        double s = 0.0;
        for (int p = 0; p < nph; ++p) s += red[(p * nblk + pb) * 17 + (a % 4) * 4 + (b % 4)];
        part[(size_t)blockIdx.x * kx * kz + e] = s;
    }
}

// The staged kernel applies when both views lie in one block each whose rows
// (16-byte multiple, at most kGramMaxK wide) can be staged whole.
template <typename T>
bool gram_fits(const void* X, Blk bx, int kx, const void* Z, Blk bz, int kz, bool zsigns) {
    constexpr int V = 16 / (int)sizeof(T);
    auto view_ok = [](const void* p, const Blk& b, int k) {
        return ((uintptr_t)p & 15) == 0 && b.ld % V == 0 && b.ld <= kGramMaxK && b.c0 % b.bw + k <= b.bw &&
               b.bw <= b.ld;
    };
    return kx <= kGramMaxK && kz <= kGramMaxK && view_ok(X, bx, kx) && (zsigns || view_ok(Z, bz, kz));
}

template <typename T>
void launch_gram_t(int n, const void* X, Blk bx, int kx, const void* Z, Blk bz, int kz,
                   const uint64_t* zmask, double* part, int nwg, hipStream_t st) {
    const bool zsigns = zmask != nullptr;
    constexpr int RT = sizeof(T) == 8 ? 64 : 128;
    const bool same = !zsigns && X == Z && kx == kz && bx.ld == bz.ld && bx.bw == bz.bw &&
                      bx.bstride == bz.bstride && bx.c0 == bz.c0;
    if (zsigns)
        hipLaunchKernelGGL((gram_kernel<T, false, true, RT>), dim3(nwg), dim3(kThreads), 0, st, n, (const T*)X,
                           bx, kx, (const T*)Z, bz, kz, zmask, part);
    else if (same)
        hipLaunchKernelGGL((gram_kernel<T, true, false, RT>), dim3(nwg), dim3(kThreads), 0, st, n, (const T*)X,
                           bx, kx, (const T*)Z, bz, kz, zmask, part);
    else
        hipLaunchKernelGGL((gram_kernel<T, false, false, RT>), dim3(nwg), dim3(kThreads), 0, st, n, (const T*)X,
                           bx, kx, (const T*)Z, bz, kz, zmask, part);
}

hipError_t launch_cross(bool f64, int n, const void* X, Blk bx, int kx, const void* Z, Blk bz,
                        int kz, const uint64_t* zmask, double* part, hipStream_t st) {
    if (kx < 1 || kz < 1 || kx > 64 || kz > 64) return hipErrorInvalidValue;
    const int nwg = cross_num_wg(n);
    if (nwg == 0) return hipSuccess;
    const bool zsigns = zmask != nullptr;
    if (f64 ? gram_fits<double>(X, bx, kx, Z, bz, kz, zsigns) : gram_fits<float>(X, bx, kx, Z, bz, kz, zsigns)) {
        if (f64)
            launch_gram_t<double>(n, X, bx, kx, Z, bz, kz, zmask, part, nwg, st);
        else
            launch_gram_t<float>(n, X, bx, kx, Z, bz, kz, zmask, part, nwg, st);
        return hipGetLastError();
    }
    return f64 ? launch_cross_tx<double>(n, X, bx, kx, Z, bz, kz, zmask, part, st)
               : launch_cross_tx<float>(n, X, bx, kx, Z, bz, kz, zmask, part, st);
}

// ---------------------------------------------------------------------------
// fixed-order compensated reduction over workgroup partials
// ---------------------------------------------------------------------------
// A block owns 16 outputs; its 16 lane groups take the partial rows
// q, q+16, q+32, ... (Neumaier), then one thread adds the 16 group sums in
// order.  The summation order depends only on nwg, so results are repeatable.
constexpr int kRedJ = 16, kRedQ = kThreads / kRedJ;

__device__ __forceinline__ void neumaier(double& s, double& c, double x) {
    const double t = s + x;
    c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(kThreads) void reduce_kernel(const double* __restrict__ part, int nwg,
                                                          int len, int part_ld,
                                                          long long outer_stride,
                                                          double* __restrict__ out, int out_ld) {
    const int jj = threadIdx.x % kRedJ, q = threadIdx.x / kRedJ;
    const int j = blockIdx.x * kRedJ + jj;
    const int o = blockIdx.y;
    double s = 0.0, c = 0.0;
    if (j < len) {
        const double* p = part + (size_t)o * outer_stride + j;
#pragma unroll 8
        for (int w = q; w < nwg; w += kRedQ) neumaier(s, c, p[(size_t)w * part_ld]);
    }
    __shared__ double ss[kThreads], cc[kThreads];
    ss[threadIdx.x] = s;
    cc[threadIdx.x] = c;
    __syncthreads();
    if (q == 0 && j < len) {
        double S = 0.0, C = 0.0;
        for (int t = 0; t < kRedQ; ++t) {
            neumaier(S, C, ss[t * kRedJ + jj]);
            neumaier(S, C, cc[t * kRedJ + jj]);
        }
        out[(size_t)o * out_ld + j] = S + C;
    }
}

hipError_t launch_reduce(const double* part, int nwg, int len, int part_ld, int outer,
                         long long outer_stride, double* out, int out_ld, hipStream_t st) {
    if ((long long)outer * len == 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_kernel, dim3(div_up(len, kRedJ), outer), dim3(kThreads), 0, st, part,
                       nwg, len, part_ld, outer_stride, out, out_ld);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// CholQR's small factorisation on the device: G = R^T R (upper R) and R^{-1},
// k <= 64, one workgroup.  Right-looking elimination subtracts the rank-one
// terms R[t][i] R[t][l] in increasing t, the order of the textbook
// column-oriented Cholesky; R^{-1} solves R X = I row by row from the last,
// each row's contribution subtracted from all rows above it at once.  A non-finite Gram entry sets *flag = 1 and a non-positive or
// relatively tiny pivot (rank-deficient sketch: r_jj <= 1e-7 sqrt(G_jj))
// sets 2; then R^{-1} is left zero.  *flag is written on every call.
// ---------------------------------------------------------------------------
constexpr int kCholMax = 64;
constexpr int kCholThreads = 256;   // a 16 x 16 grid over the entries
constexpr int kCholLd = kCholMax + 1;

__global__ __launch_bounds__(kCholThreads) void chol_factor_kernel(const double* __restrict__ G, int k,
                                                                   double* __restrict__ R,
                                                                   double* __restrict__ Rinv,
                                                                   int* __restrict__ flag) {
    // R in the upper triangle of a; R^{-1} transposed in its strict lower
    // triangle, inv(j, i) at a[i][j], with the diagonal of R^{-1} in invd.
    // Threads form a 16 x 16 grid (tx, ty) over the matrix entries.
    __shared__ double a[kCholMax * kCholLd];
    __shared__ double invd[kCholMax];
    __shared__ double gdiag[kCholMax];   // the Gram's diagonal, for the relative pivot test
    __shared__ int bad;
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int r = ty; r < k; r += 16)
        for (int c = tx; c < k; c += 16) {
            const double v = G[r * k + c];
            if (!isfinite(v)) bad = 1;
            a[r * kCholLd + c] = v;
            if (r == c) gdiag[r] = v;
        }
    __syncthreads();
    for (int j = 0; j < k && bad == 0; ++j) {
        const double s = a[j * kCholLd + j];
        const double rjj = sqrt(s);
        const bool ok = s > 0.0 && isfinite(s) && rjj > 1e-7 * sqrt(fabs(gdiag[j]));
        __syncthreads();   // every lane has read the pivot before row j changes
        if (!ok) {
            if (tid == 0) bad = 2;
            __syncthreads();
            break;
        }
        for (int i = j + tid; i < k; i += kCholThreads)
            a[j * kCholLd + i] = i == j ? rjj : a[j * kCholLd + i] / rjj;
        __syncthreads();
        for (int r = j + 1 + ty; r < k; r += 16)
            for (int c = j + 1 + tx; c < k; c += 16)
                if (c >= r) a[r * kCholLd + c] -= a[j * kCholLd + r] * a[j * kCholLd + c];
        __syncthreads();
    }
    const int ok = bad == 0;
    // R X = I solved by rows, last first: row j of X is final once the rows
    // below it have been subtracted from the right-hand side B (= I at the
    // start); then every row i < j takes away R[i][j] X[j][:].  B and X are
    // upper triangular: B[i][c] (i < c) lives at a[c][i], its diagonal in invd.
    if (ok) {
        for (int r = ty; r < k; r += 16)
            for (int c = tx; c < r; c += 16) a[r * kCholLd + c] = 0.0;
        for (int i = tid; i < k; i += kCholThreads) invd[i] = 1.0;
        __syncthreads();
        for (int j = k - 1; j >= 0; --j) {
            const double rjj = a[j * kCholLd + j];
            for (int c = j + tid; c < k; c += kCholThreads) {
                if (c == j)
                    invd[j] = invd[j] / rjj;
                else
                    a[c * kCholLd + j] = a[c * kCholLd + j] / rjj;
            }
            __syncthreads();
            for (int i = ty; i < j; i += 16)
                for (int c = j + tx; c < k; c += 16) {
                    const double xjc = c == j ? invd[j] : a[c * kCholLd + j];
                    a[c * kCholLd + i] -= a[i * kCholLd + j] * xjc;
                }
            __syncthreads();
        }
    }
    __syncthreads();
    for (int r = ty; r < k; r += 16)
        for (int c = tx; c < k; c += 16) {
            const bool on = ok && c >= r;
            if (R) R[r * k + c] = on ? a[r * kCholLd + c] : 0.0;
            Rinv[r * k + c] = on ? (c == r ? invd[r] : a[c * kCholLd + r]) : 0.0;
        }
    if (tid == 0) *flag = bad;
}

hipError_t launch_chol_factor(const double* G, int k, double* R, double* Rinv, int* flag,
                              hipStream_t st) {
    if (k < 1 || k > kCholMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(chol_factor_kernel, dim3(1), dim3(kCholThreads), 0, st, G, k, R, Rinv, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// row block times a small FP64 matrix (TRSM with R^{-1}; deflation G - Q C)
// ---------------------------------------------------------------------------
// Tiles of RT rows (one row per thread); a grid of at most kRowmatWgs
// workgroups loops over them, staging M once per workgroup.  The tile of Y is
// loaded into LDS with coalesced accesses (consecutive threads read
// consecutive columns; each thread issues all its loads before it stores any,
// so a tile costs one memory round trip), each thread multiplies its row by M
// (one row of M per step, read from LDS at the same address by every lane),
// the results go back into the tile, and the tile is written out
// coalesced, adding the optional base matrix and probe signs.  Y, base and
// out are column-blocked (Blk).
constexpr int kRowmatWgs = 1024;
constexpr int kRowmatBatch = 8;    // loads a thread keeps in flight while staging (16: 151-214 VGPRs, 19-21% slower)

// FAST: Y's columns lie in one block whose rows (ld <= max(KY, KO), 16-byte
// multiple) the tile holds whole, and out (and base) cover whole rows of
// their block: a tile is then one contiguous run in each, moved with 16-byte
// vectors in a single batch per thread.
template <typename T, int KY, int KO, bool SIGNS, int RT, bool FAST>
__global__ __launch_bounds__(RT) void rowmat_kernel(int n, const T* __restrict__ Y, Blk by,
                                                    int ky, const double* __restrict__ M,
                                                    int kout, double sign_m, const uint64_t* __restrict__ zmask,
                                                    const T* base, Blk bb, T* out, Blk bo) {
    constexpr int KS = (KY > KO ? KY : KO) + 1;      // padded row stride of the tile
    __shared__ T ms[KY * KO];
    __shared__ T tile[RT * KS];
    __shared__ size_t yoff[KY], ooff[KO], boff[KO];
    for (int e = threadIdx.x; e < KY * KO; e += RT) {
        const int i = e / KO, j = e - i * KO;
        ms[e] = (i < ky && j < kout) ? (T)(sign_m * M[i * kout + j]) : T(0);
    }
    for (int i = threadIdx.x; i < KY; i += RT) yoff[i] = i < ky ? by.offset(i) : 0;
    for (int j = threadIdx.x; j < KO; j += RT) {
        ooff[j] = j < kout ? bo.offset(j) : 0;
        boff[j] = j < kout ? bb.offset(j) : 0;
    }
    __syncthreads();
    const int ntiles = div_up_dev(n, RT);
    // element e = tid + u*RT of a tile is (row e / k, column e % k); RT = qa*k + qb
    const int qa_y = RT / ky, qb_y = RT - qa_y * ky;
    const int qa_o = RT / kout, qb_o = RT - qa_o * kout;
    const int cy = FAST ? by.c0 % by.bw : 0;   // first column of Y's view within a staged row
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int row0 = t * RT;
    const int nr = min(RT, n - row0);
    constexpr int V = 16 / (int)sizeof(T);
    using P = Pack<T, V>;
    if constexpr (FAST) {   // the tile is rows [row0, row0+nr) of Y's block, whole
        constexpr int NV = (KS - 1 + V - 1) / V;
        const int ldy = by.ld;
        const T* src = Y + (size_t)(by.c0 / by.bw) * (size_t)by.bstride + (size_t)row0 * ldy;
        const int nvec = nr * ldy / V;
        P v[NV];
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = threadIdx.x + u * RT;
            if (e < nvec) v[u] = load_pack<T, V>(src + (size_t)e * V);
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = threadIdx.x + u * RT;
            if (e < nvec) {
                const int x = e * V, r = x / ldy, c = x - r * ldy;
#pragma unroll
                for (int q = 0; q < V; ++q) tile[r * KS + c + q] = v[u].v[q];
            }
        }
    } else
    {   // stage the tile of Y: a batch of loads in flight, then their LDS stores
        int r = threadIdx.x / ky, i = threadIdx.x - (threadIdx.x / ky) * ky;
#pragma nounroll
        for (int u0 = 0; u0 < KY && u0 * RT < nr * ky; u0 += kRowmatBatch) {
            T v[kRowmatBatch];
            const int r0 = r, i0 = i;
#pragma unroll
            for (int u = 0; u < kRowmatBatch; ++u) {
                v[u] = r < nr ? Y[yoff[i] + (size_t)(row0 + r) * by.ld] : T(0);
                r += qa_y;
                i += qb_y;
                if (i >= ky) {
                    i -= ky;
                    ++r;
                }
            }
            r = r0;
            i = i0;
#pragma unroll
            for (int u = 0; u < kRowmatBatch; ++u) {
                if (r < nr) tile[r * KS + i] = v[u];
                r += qa_y;
                i += qb_y;
                if (i >= ky) {
                    i -= ky;
                    ++r;
                }
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < nr) {   // row times M: one row of M (LDS broadcast) per step
        T acc[KO];
#pragma unroll
        for (int j = 0; j < KO; ++j) acc[j] = T(0);
#pragma nounroll
        for (int i = 0; i < ky; ++i) {
            const T yi = tile[threadIdx.x * KS + cy + i];
#pragma unroll
            for (int j = 0; j < KO; ++j) acc[j] = fma(yi, ms[i * KO + j], acc[j]);
        }
#pragma unroll
        for (int j = 0; j < KO; ++j)
            if (j < kout) tile[threadIdx.x * KS + j] = acc[j];
    }
    __syncthreads();
    if constexpr (FAST) {   // out's tile is rows [row0, row0+nr) of its block, kout == ld
        constexpr int NV = (KO + V - 1) / V;
        T* dst = out + (size_t)(bo.c0 / bo.bw) * (size_t)bo.bstride + (size_t)row0 * kout;
        const T* bsrc = base ? base + (size_t)(bb.c0 / bb.bw) * (size_t)bb.bstride + (size_t)row0 * kout : nullptr;
        const int nvec = nr * kout / V;
        P b[NV];
        uint64_t w[SIGNS ? NV : 1];   // sign words, loaded with the base values before any store
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = threadIdx.x + u * RT;
#pragma unroll
            for (int q = 0; q < V; ++q) b[u].v[q] = T(0);
            if (bsrc && e < nvec) b[u] = load_pack<T, V>(bsrc + (size_t)e * V);
            if constexpr (SIGNS) w[u] = e < nvec ? zmask[row0 + (e * V) / kout] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int e = threadIdx.x + u * RT;
            if (e < nvec) {
                const int x = e * V, r = x / kout, c = x - r * kout;
                P o;
#pragma unroll
                for (int q = 0; q < V; ++q) {
                    T v = tile[r * KS + c + q] + b[u].v[q];
                    if constexpr (SIGNS) v += ((w[u] >> (c + q)) & 1ull) ? T(-1) : T(1);
                    o.v[q] = v;
                }
                store_pack<T, V>(dst + (size_t)x, o);
            }
        }
    } else
    {   // write out: a batch of base values loaded first (base may alias out), then the stores
        int r = threadIdx.x / kout, j = threadIdx.x - (threadIdx.x / kout) * kout;
#pragma nounroll
        for (int u0 = 0; u0 < KO && u0 * RT < nr * kout; u0 += kRowmatBatch) {
            T b[kRowmatBatch];
            uint64_t w[SIGNS ? kRowmatBatch : 1];
            const int r0 = r, j0 = j;
#pragma unroll
            for (int u = 0; u < kRowmatBatch; ++u) {
                b[u] = (base && r < nr) ? base[boff[j] + (size_t)(row0 + r) * bb.ld] : T(0);
                if constexpr (SIGNS) w[u] = r < nr ? zmask[row0 + r] : 0ull;
                r += qa_o;
                j += qb_o;
                if (j >= kout) {
                    j -= kout;
                    ++r;
                }
            }
            r = r0;
            j = j0;
#pragma unroll
            for (int u = 0; u < kRowmatBatch; ++u) {
                if (r < nr) {
                    const int row = row0 + r;
                    T v = tile[r * KS + j] + b[u];
                    if constexpr (SIGNS) v += ((w[u] >> j) & 1ull) ? T(-1) : T(1);
                    out[ooff[j] + (size_t)row * bo.ld] = v;
                }
                r += qa_o;
                j += qb_o;
                if (j >= kout) {
                    j -= kout;
                    ++r;
                }
            }
        }
    }
    __syncthreads();   // the tile is reused by the next iteration
    }
}

template <typename T, int KY, int KO>
void launch_rowmat_t(int n, hipStream_t st, const void* Y, Blk by, int ky, const double* M,
                     int kout, double sign_m, const uint64_t* zmask, const void* base, Blk bb,
                     void* out, Blk bo) {
    constexpr int RT = (sizeof(T) == 8 && KY == 64 && KO == 64) ? 128 : 256;
    const int nwg = std::min(div_up(n, RT), kRowmatWgs);
    constexpr int V = 16 / (int)sizeof(T);
    auto aligned = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    // a view covers whole rows of its block: starts a block, as wide as its rows
    auto whole_rows = [&](const Blk& b, int k) { return b.c0 % b.bw == 0 && k == b.ld && k <= b.bw && b.ld % V == 0; };
    // at most 16 vectors per thread in a batch (FP64 with 64 columns keeps the general path)
    constexpr bool kFastFits = (KY > KO ? KY : KO) / V <= 16;
    const bool fast = kFastFits && aligned(Y) && aligned(out) && by.ld % V == 0 && by.ld <= (KY > KO ? KY : KO) &&
                      by.c0 % by.bw + ky <= by.bw && whole_rows(bo, kout) &&
                      (!base || (aligned(base) && whole_rows(bb, kout)));
#define LD_RM_GO(S_, F_)                                                                                     \
    hipLaunchKernelGGL((rowmat_kernel<T, KY, KO, S_, RT, F_>), dim3(nwg), dim3(RT), 0, st, n, (const T*)Y, by, \
                       ky, M, kout, sign_m, zmask, (const T*)base, bb, (T*)out, bo)
    if constexpr (kFastFits) {
        if (fast) {
            if (zmask)
                LD_RM_GO(true, true);
            else
                LD_RM_GO(false, true);
            return;
        }
    }
    if (zmask)
        LD_RM_GO(true, false);
    else
        LD_RM_GO(false, false);
#undef LD_RM_GO
}

template <typename T>
hipError_t launch_rowmat_ty(hipStream_t st, int n, const void* Y, Blk by, int ky,
                            const double* M, int kout, double sign_m, const uint64_t* zmask,
                            const void* base, Blk bb, void* out, Blk bo) {
    const int a = ky <= 16 ? 16 : ky <= 32 ? 32 : 64;
    const int b = kout <= 16 ? 16 : kout <= 32 ? 32 : 64;
#define LD_RM(A_, B_) \
    if (a == A_ && b == B_) launch_rowmat_t<T, A_, B_>(n, st, Y, by, ky, M, kout, sign_m, zmask, base, bb, out, bo);
    LD_RM(16, 16) LD_RM(16, 32) LD_RM(16, 64) LD_RM(32, 16) LD_RM(32, 32) LD_RM(32, 64)
    LD_RM(64, 16) LD_RM(64, 32) LD_RM(64, 64)
#undef LD_RM
    return hipGetLastError();
}

hipError_t launch_rowmat(bool f64, int n, const void* Y, Blk by, int ky, const double* M, int kout,
                         double sign_m, const uint64_t* zmask, const void* base, Blk bb,
                         void* out, Blk bo, hipStream_t st) {
    if (ky < 1 || kout < 1 || ky > 64 || kout > 64) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    return f64 ? launch_rowmat_ty<double>(st, n, Y, by, ky, M, kout, sign_m, zmask, base, bb, out, bo)
               : launch_rowmat_ty<float>(st, n, Y, by, ky, M, kout, sign_m, zmask, base, bb, out, bo);
}

// ---------------------------------------------------------------------------
// CSR structure check (reads col_idx only inside [0, nnz))
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void validate_kernel(int n, int nnz,
                                                            const int* __restrict__ row_ptr,
                                                            const int* __restrict__ col_idx,
                                                            int* __restrict__ flag) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    const int b = row_ptr[r], e = row_ptr[r + 1];
    bool bad = (b < 0) || (e < b) || (e > nnz) || (r == 0 && b != 0) || (r == n - 1 && e != nnz);
    if (!bad) {
        int prev = -1;
        for (int k = b; k < e; ++k) {
            const int c = col_idx[k];
            if (c < 0 || c >= n || c <= prev) {
                bad = true;
                break;
            }
            prev = c;
        }
    }
    if (bad) *flag = 1;
}

hipError_t launch_validate_csr(const CsrDev& A, int* flag, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(validate_kernel, dim3(div_up(A.n, kThreads)), dim3(kThreads), 0, st, A.n,
                       A.nnz, A.row_ptr, A.col_idx, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gershgorin discs
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void gersh_kernel(int n, const int* __restrict__ row_ptr,
                                                         const int* __restrict__ col_idx,
                                                         const T* __restrict__ val,
                                                         double* __restrict__ part) {
    const int r = blockIdx.x * kThreads + threadIdx.x;
    double lo = __builtin_inf(), hi = -__builtin_inf();
    if (r < n) {
        double diag = 0.0, rad = 0.0;
        for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            const double v = (double)val[k];
            if (col_idx[k] == r)
                diag += v;
            else
                rad += fabs(v);
        }
        lo = diag - rad;
        hi = diag + rad;
    }
    __shared__ double slo[kThreads], shi[kThreads];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
            shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = slo[0];
        part[2 * blockIdx.x + 1] = shi[0];
    }
}

int gersh_num_wg(int n) { return div_up(n, kThreads); }

hipError_t launch_gershgorin(bool f64, const CsrDev& A, double* part, hipStream_t st) {
    const int nwg = gersh_num_wg(A.n);
    if (nwg == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(gersh_kernel<double>, dim3(nwg), dim3(kThreads), 0, st, A.n, A.row_ptr,
                           A.col_idx, (const double*)A.val, part);
    else
        hipLaunchKernelGGL(gersh_kernel<float>, dim3(nwg), dim3(kThreads), 0, st, A.n, A.row_ptr,
                           A.col_idx, (const float*)A.val, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise y = a x + b y
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void axpby_kernel(long long len, T a, const T* __restrict__ x,
                                                         T b, T* __restrict__ y) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < len) y[i] = a * x[i] + b * y[i];
}

// Candidate diagonals: the distinct offsets col - row of 64 rows scattered
// over the matrix, merged in ascending order by one lane; info[0] = their number,
// or -1 when a sampled row or the union exceeds kMaxDiag.
__global__ __launch_bounds__(64) void dia_probe_kernel(int n, const int* __restrict__ row_ptr,
                                                       const int* __restrict__ col_idx, const void* __restrict__ val,
                                                       int f64, int* __restrict__ info) {
    // one wave: lane t samples one row (golden-ratio stride: no alignment with
    // a grid's rows, whatever its width) and holds its column offsets
    const int t = threadIdx.x;
    const int r = (int)(((uint64_t)(t + 1) * 0x9E3779B97F4A7C15ull) % (uint64_t)n);
    const int b = row_ptr[r], e = row_ptr[r + 1];
    const bool fits = e - b <= kMaxDiag;
    int off[kMaxDiag];
#pragma unroll
    for (int q = 0; q < kMaxDiag; ++q) off[q] = (fits && b + q < e) ? col_idx[b + q] - r : INT_MAX;
    // the distinct offsets in increasing order: repeatedly the wave's smallest
    // offset above the last one found
    int nu = __any(!fits) ? -1 : 0;
    int u[kMaxDiag];
    long long last = LLONG_MIN;
    while (nu >= 0) {
        int m = INT_MAX;
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q)
            if ((long long)off[q] > last && off[q] < m) m = off[q];
        for (int d = 32; d >= 1; d >>= 1) m = min(m, __shfl_xor(m, d, 64));
        if (m == INT_MAX) break;
        if (nu == kMaxDiag) {
            nu = -1;
            break;
        }
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q)
            if (q == nu) u[q] = m;
        ++nu;
        last = m;
    }
    if (t == 0) {
        info[0] = nu;
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q) info[1 + q] = (nu > 0 && q < nu) ? u[q] : 0;
    }
    // candidate constant of each diagonal: its value in the first sampled row
    // that has it (the build checks every other entry against it)
    double* const cval = reinterpret_cast<double*>(info + kConstInfo);
#pragma unroll
    for (int q = 0; q < kMaxDiag; ++q) {
        if (q >= nu) break;   // uniform
        int at = -1;
#pragma unroll
        for (int j = 0; j < kMaxDiag; ++j)
            if (off[j] == u[q]) at = j;
        const double v = at < 0 ? 0.0
                                : (f64 ? static_cast<const double*>(val)[b + at]
                                       : (double)static_cast<const float*>(val)[b + at]);
        const uint64_t has = __ballot(at >= 0);
        const int first = __ffsll((unsigned long long)has) - 1;   // at least one lane: u[q] came from a sample
        const double c = __shfl(v, first, 64);
        if (t == 0) cval[q] = c;
    }
    // row_ptr at the boundaries of eight equal row bands (balance of the
    // entries over the XCD bands)
    if (t <= kXcds) info[kBandInfo + t] = row_ptr[(int)((long long)t * n / kXcds)];
}

// Diagonal storage for the offsets of info (ascending): dia[r*nd + q] =
// A[r, r + off[q]] or 0, pres[r] bit q set when row r stores diagonal q;
// info[kDiaFlag] = 1 when a stored entry lies on none of them (or there are
// no candidates), info[kConstFlag] = 1 when some entry differs from its
// diagonal's candidate constant.
constexpr int kDiaFlag = 12;

template <typename T>
__global__ __launch_bounds__(kThreads) void dia_build_kernel(int n, const int* __restrict__ row_ptr,
                                                             const int* __restrict__ col_idx,
                                                             const T* __restrict__ val, T* __restrict__ dia,
                                                             uint16_t* __restrict__ pres, int* __restrict__ info) {
    // each thread places its row's entries in registers; the workgroup's rows
    // are one contiguous run of the storage, written through LDS with
    // consecutive threads on consecutive elements
    __shared__ T sv[kThreads * kMaxDiag];
    const int nd = info[0];
    if (nd <= 0) {   // uniform: no candidate diagonals
        if (blockIdx.x == 0 && threadIdx.x == 0) info[kDiaFlag] = 1;
        return;
    }
    const int r0 = blockIdx.x * kThreads;
    const int nr = min(kThreads, n - r0);
    const int r = r0 + threadIdx.x;
    if (threadIdx.x < nr) {
        int off[kMaxDiag];
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q) off[q] = info[1 + q];
        T v[kMaxDiag], cv[kMaxDiag];
        const double* const cinfo = reinterpret_cast<const double*>(info + kConstInfo);
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q) {
            v[q] = T(0);
            cv[q] = q < nd ? (T)cinfo[q] : T(0);
        }
        bool bad = false, varies = false;
        unsigned bits = 0;
        for (int k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            const int o = col_idx[k] - r;
            const T x = val[k];
            bool hit = false;
#pragma unroll
            for (int q = 0; q < kMaxDiag; ++q)
                if (q < nd && off[q] == o) {
                    v[q] = x;
                    hit = true;
                    bits |= 1u << q;
                    varies |= !(x == cv[q]);
                }
            bad |= !hit;
        }
        if (bad) info[kDiaFlag] = 1;
        if (varies) info[kConstFlag] = 1;
        pres[r] = (uint16_t)bits;
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q)
            if (q < nd) sv[threadIdx.x * nd + q] = v[q];
    }
    __syncthreads();
    T* const out = dia + (size_t)r0 * nd;
    for (int e = threadIdx.x; e < nr * nd; e += kThreads) out[e] = sv[e];
}

hipError_t launch_rows_probe(bool f64, const CsrDev& A, int* info, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    hipLaunchKernelGGL(dia_probe_kernel, dim3(1), dim3(64), 0, st, A.n, A.row_ptr, A.col_idx, A.val, (int)f64, info);
    return hipGetLastError();
}

hipError_t launch_dia_build(bool f64, const CsrDev& A, void* dia, uint16_t* pres, int* info, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    const int nb = div_up(A.n, kThreads);
    if (f64)
        hipLaunchKernelGGL(dia_build_kernel<double>, dim3(nb), dim3(kThreads), 0, st, A.n, A.row_ptr, A.col_idx,
                           (const double*)A.val, (double*)dia, pres, info);
    else
        hipLaunchKernelGGL(dia_build_kernel<float>, dim3(nb), dim3(kThreads), 0, st, A.n, A.row_ptr, A.col_idx,
                           (const float*)A.val, (float*)dia, pres, info);
    return hipGetLastError();
}

__global__ __launch_bounds__(64) void adapt_decide_kernel(const double* __restrict__ sums, int stride, int qc,
                                                          double dm_abs, double tol, int m,
                                                          uint64_t* __restrict__ mask, int* __restrict__ deg) {
    const int c = threadIdx.x;
    const uint64_t old = *mask;
    const bool was = c < qc && ((old >> c) & 1ull);
    bool keep = false;
    if (was) {
        const double e = dm_abs * sqrt(fmax(sums[(size_t)c * stride], 0.0));
        keep = e > tol;
        if (!keep) deg[c] = m;
    }
    const uint64_t now = __ballot(keep);
    if (c == 0) *mask = now;
}

hipError_t launch_adapt_decide(const double* sums, int stride, int qc, double dm_abs, double tol, int m,
                               uint64_t* mask, int* deg, hipStream_t st) {
    if (qc < 1 || qc > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(adapt_decide_kernel, dim3(1), dim3(64), 0, st, sums, stride, qc, dm_abs, tol, m, mask,
                       deg);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void widen_kernel(long long len, const float* __restrict__ x,
                                                         double* __restrict__ y) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < len) y[i] = (double)x[i];
}

hipError_t launch_widen(long long len, const float* x, double* y, hipStream_t st) {
    if (len == 0) return hipSuccess;
    hipLaunchKernelGGL(widen_kernel, dim3(div_up(len, kThreads)), dim3(kThreads), 0, st, len, x, y);
    return hipGetLastError();
}

hipError_t launch_axpby(bool f64, long long len, double a, const void* x, double b, void* y,
                        hipStream_t st) {
    if (len == 0) return hipSuccess;
    const int nb = div_up(len, kThreads);
    if (f64)
        hipLaunchKernelGGL(axpby_kernel<double>, dim3(nb), dim3(kThreads), 0, st, len, a,
                           (const double*)x, b, (double*)y);
    else
        hipLaunchKernelGGL(axpby_kernel<float>, dim3(nb), dim3(kThreads), 0, st, len, (float)a,
                           (const float*)x, (float)b, (float*)y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient sweep step: one Newton step of a block `lam` fused with an SDDMM on
// A's pattern.  For each stored entry (r, c) of A the gradient (FP64) picks up
//   alpha * sum_cols own[r, col] * w[c, col]
// and the block moves on (A symmetric):
//   ADJ_HORNER:  out = alpha*A*lam - beta*lam + dj*L,        own = lam[r]
//                (the Horner adjoint of the Newton form: lam_i from lam_{i+1})
//   ADJ_PLAIN:   out = alpha*A*lam - beta*lam,               own = lam[r]
//                (the forward Newton vectors of the sketch's cotangent)
//   ADJ_SQUARED: out = alpha*A*lam - beta*lam + q0*w[r] + q1*(alpha*A*w - beta*w)[r],
//                own = wgt(col) * (lam[r] + p1*w[r])
//                (the adjoint of the quadratic forms in the squared Newton basis:
//                lam = mu~_{i+1}, w = u_i, q0 = 2c_{2i}, q1 = 2c_{2i+1}, p1 = c_{2i+1},
//                wgt = 1 on the first wsplit columns and whi after them)
// Row groups of LPR lanes (a power of two) own one row; lane li holds the
// columns (q*LPR + li)*VEC + [0, VEC) for q < CPL (chunks at or past ld are
// not loaded).  A row's entries go in batches of NB = min(LPR, kAdjBatch):
// the batch's gathers of w and lam are issued together, then the NB per-lane
// partial dot products (the lane's own columns in the block's precision, FP64
// from there on) are reduced across the row group (butterfly
// over the lane bits >= NB, then a reduce-scatter over the low bits, NB-1
// shuffles) so that lane li ends with entry li's sum and the batch's gradient
// entries are read (ahead of the gathers) and written by NB adjacent lanes.
// Each entry's gradient is owned by one lane: no atomics.  The workgroup's
// CSR slice is staged in LDS when it fits.
// ---------------------------------------------------------------------------
template <typename T, int VEC, int LPR, int CPL, int MODE>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(
    int n, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
    const T* __restrict__ val, const T* __restrict__ lam_in, T* __restrict__ lam_out,
    const T* __restrict__ w, const T* __restrict__ L, double* __restrict__ grad, int ld, int ncols,
    T alpha, T beta, T dj, T q0, T q1, T p1, int wsplit, T whi, int first, int last, int nt_out, T lam_scale) {
    constexpr int RPW = 64 / LPR;
    constexpr int NB = LPR < kAdjBatch ? LPR : kAdjBatch;
    constexpr int rows_per_wg = kWaves * RPW;
    constexpr bool kSq = MODE == ADJ_SQUARED;
    __shared__ int s_rp[rows_per_wg + 1];
    __shared__ int s_col[kAdjStageNz];
    __shared__ T s_val[kAdjStageNz];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane / LPR;
    const int li = lane - g * LPR;
    const int R0 = xcd_tile(blockIdx.x, gridDim.x) * rows_per_wg;
    const int nrows = min(rows_per_wg, n - R0);
    for (int t = threadIdx.x; t <= nrows; t += kThreads) s_rp[t] = row_ptr[R0 + t];
    __syncthreads();
    const int K0 = s_rp[0], K1 = s_rp[nrows];
    const bool staged = (K1 - K0) <= kAdjStageNz;
    if (staged)
        for (int k = K0 + threadIdx.x; k < K1; k += kThreads) {
            s_col[k - K0] = col_idx[k];
            s_val[k - K0] = val[k];
        }
    __syncthreads();
    const int lr = wave * RPW + g;
    if (lr >= nrows) return;                     // whole row groups leave together
    const int row = R0 + lr;
    bool inld[CPL];                              // the lane's chunk lies inside the row
    bool valid[CPL][VEC];
    Pack<T, VEC> own[CPL], Lr[CPL], wr[CPL];
    T sown[CPL][VEC];                            // this row's side of the SDDMM
    T acc[CPL][VEC], accw[CPL][VEC];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
        const int c0 = (q * LPR + li) * VEC;
        inld[q] = c0 < ld;
        const size_t off = (size_t)row * ld + c0;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            own[q].v[e] = Lr[q].v[e] = wr[q].v[e] = T(0);
            valid[q][e] = c0 + e < ncols;
            acc[q][e] = accw[q][e] = T(0);
        }
        if (inld[q]) {
            if (lam_scale != T(0)) own[q] = load_pack<T, VEC>(lam_in + off);   // lam = lam_scale * lam_in
            if (MODE == ADJ_HORNER && !last) Lr[q] = load_pack<T, VEC>(L + off);   // fetched early: used at the end
            if (kSq) wr[q] = load_pack<T, VEC>(w + off);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            own[q].v[e] *= lam_scale;
            T so = own[q].v[e];
            if (kSq) so = (c0 + e < wsplit ? T(1) : whi) * fma(p1, wr[q].v[e], so);
            sown[q][e] = valid[q][e] ? so : T(0);
        }
    }
    const int beg = s_rp[lr], end = s_rp[lr + 1];
    for (int kb = beg; kb < end; kb += NB) {
        // the gradient entry this lane updates, fetched ahead of the gathers
        const int kg = kb + li;
        const bool owner = li < NB && kg < end;
        double gold = 0.0;
        if (owner && !first) gold = grad[kg];
        int cidx[NB];
        T a[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int k = kb + u;
            cidx[u] = row;
            a[u] = T(0);
            if (k < end) {
                cidx[u] = staged ? s_col[k - K0] : col_idx[k];
                a[u] = staged ? s_val[k - K0] : val[k];
            }
        }
        double part[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            part[u] = 0.0;
            if (kb + u < end) {
#pragma unroll
                for (int q = 0; q < CPL; ++q) {
                    if (!inld[q]) continue;
                    const size_t off = (size_t)cidx[u] * ld + (q * LPR + li) * VEC;
                    const Pack<T, VEC> wc = load_pack<T, VEC>(w + off);
                    // the lane's VEC products in the block's precision (a select:
                    // padding columns may hold anything), FP64 from here on
                    T pq = T(0);
#pragma unroll
                    for (int e = 0; e < VEC; ++e) pq = valid[q][e] ? fma(sown[q][e], wc.v[e], pq) : pq;
                    part[u] += (double)pq;
                    if (kSq) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) accw[q][e] = fma(a[u], wc.v[e], accw[q][e]);
                    }
                    if (!last && lam_scale != T(0)) {
                        const Pack<T, VEC> lc = load_pack<T, VEC>(lam_in + off);
#pragma unroll
                        for (int e = 0; e < VEC; ++e) acc[q][e] = fma(a[u], lam_scale * lc.v[e], acc[q][e]);
                    }
                }
            }
        }
        // lane bits >= NB: plain butterfly on every entry of the batch
#pragma unroll
        for (int h = LPR / 2; h >= NB; h >>= 1)
#pragma unroll
            for (int u = 0; u < NB; ++u) part[u] += __shfl_xor(part[u], h, 64);
        // low bits: reduce-scatter, after which part[0] of lane li is the sum of entry li % NB
#pragma unroll
        for (int h = NB / 2; h >= 1; h >>= 1) {
            const bool hi = (li & h) != 0;
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const double send = hi ? part[j] : part[j + h];
                const double keep = hi ? part[j + h] : part[j];
                part[j] = keep + __shfl_xor(send, h, 64);
            }
        }
        if (owner) grad[kg] = fma((double)alpha, part[0], gold);
    }
    if (!last) {
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
            if (!inld[q]) continue;
            const size_t off = (size_t)row * ld + (q * LPR + li) * VEC;
            Pack<T, VEC> o;
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                T x = alpha * acc[q][e] - beta * own[q].v[e];
                if (MODE == ADJ_HORNER) x = fma(dj, Lr[q].v[e], x);
                if (kSq) x = fma(q1, alpha * accw[q][e] - beta * wr[q].v[e], fma(q0, wr[q].v[e], x));
                o.v[e] = x;
            }
            if (nt_out)
                store_pack_nt<T, VEC>(lam_out + off, o);
            else
                store_pack<T, VEC>(lam_out + off, o);
        }
    }
}

template <typename T, int VEC, int LPR, int CPL, int MODE>
hipError_t launch_adjoint_m(const CsrDev& A, const AdjArgs& a, hipStream_t st) {
    constexpr int rows_per_wg = kWaves * (64 / LPR);
    const int nwg = div_up(A.n, rows_per_wg);
    if (nwg == 0) return hipSuccess;
    hipLaunchKernelGGL((adjoint_kernel<T, VEC, LPR, CPL, MODE>), dim3(nwg), dim3(kThreads), 0, st, A.n,
                       A.row_ptr, A.col_idx, (const T*)A.val, (const T*)a.lam_in, (T*)a.lam_out,
                       (const T*)a.w, (const T*)a.L, a.grad, a.ld, a.ncols, (T)a.alpha, (T)a.beta,
                       (T)a.dj, (T)a.q0, (T)a.q1, (T)a.p1, a.wsplit, (T)a.whi, (int)a.first, (int)a.last,
                       (int)a.nt_out, (T)a.lam_scale);
    return hipGetLastError();
}

template <typename T, int VEC, int LPR, int CPL>
hipError_t launch_adjoint_t(const CsrDev& A, const AdjArgs& a, hipStream_t st) {
    switch (a.mode) {
        case ADJ_HORNER: return launch_adjoint_m<T, VEC, LPR, CPL, ADJ_HORNER>(A, a, st);
        case ADJ_PLAIN: return launch_adjoint_m<T, VEC, LPR, CPL, ADJ_PLAIN>(A, a, st);
        case ADJ_SQUARED: return launch_adjoint_m<T, VEC, LPR, CPL, ADJ_SQUARED>(A, a, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int VEC>
hipError_t launch_adjoint_v(const CsrDev& A, const AdjArgs& a, hipStream_t st) {
    const int lanes = lanes_per_row(a.ncols, VEC);
    int lp2 = 1;
    while (lp2 < lanes) lp2 <<= 1;
    const int cpl = lp2 > 64 ? lp2 / 64 : 1;
    const int lpr = lp2 > 64 ? 64 : lp2;
    // every used column lies in the row (ld >= ncols, ld a multiple of VEC);
    // lanes whose chunk starts at or past ld load nothing
    if (cpl > 2 || a.ncols > a.ld || a.ld % VEC) return hipErrorInvalidValue;
    if (cpl == 2) return launch_adjoint_t<T, VEC, 64, 2>(A, a, st);
    switch (lpr) {
        case 1: return launch_adjoint_t<T, VEC, 1, 1>(A, a, st);
        case 2: return launch_adjoint_t<T, VEC, 2, 1>(A, a, st);
        case 4: return launch_adjoint_t<T, VEC, 4, 1>(A, a, st);
        case 8: return launch_adjoint_t<T, VEC, 8, 1>(A, a, st);
        case 16: return launch_adjoint_t<T, VEC, 16, 1>(A, a, st);
        case 32: return launch_adjoint_t<T, VEC, 32, 1>(A, a, st);
        default: return launch_adjoint_t<T, VEC, 64, 1>(A, a, st);
    }
}

// ---------------------------------------------------------------------------
// Gradient sweep step on the diagonal storage (stencils, banded matrices):
// row r's stored entries are its present diagonals q (bit q of pres[r]), in
// offset order, so entry (r, r + off[q]) sits at CSR position row_ptr[r] +
// (number of present diagonals below q) and the gradient keeps A's CSR
// layout.  A row group of LPR lanes (a power of two, VEC columns per lane;
// chunks at or past ld load nothing) owns one row: it issues the ND gathers
// of lam and of w together, forms the Newton step as ADJ_PLAIN / ADJ_SQUARED
// of adjoint_kernel, and reduces the ND per-lane partial dot products (FP64)
// over the row group by a butterfly; lane q then updates entry q.
// ADJ_PLAIN2 does two steps of the sketch's adjoint in one launch: with
// out = rbar_j+1[r] computed from the gathered rbar_j, the entry also picks up
// alpha * <out, w2[c]> (w2 = r_j+2), so the gradient is read and written once
// for two steps; the next launch only needs rbar_j+1 -> rbar_j+2.
// Matrix values: one per diagonal (cv) when `dpres` is the constant-value
// mode, else dia[r*nd + q].
// ---------------------------------------------------------------------------
template <typename T, int VEC, int LPR, int ND, int MODE>
__global__ __launch_bounds__(kThreads) void adjoint_dia_kernel(
    int n, const int* __restrict__ row_ptr, const uint16_t* __restrict__ pres, const T* __restrict__ dia, int nd,
    DiaOff off, DiaVal<T> cv, int constant, const T* __restrict__ lam_in, T* __restrict__ lam_out,
    const T* __restrict__ w, const T* __restrict__ w2, double* __restrict__ grad, int ld, int ncols, T alpha,
    T beta, T q0, T q1, T p1, int wsplit, T whi, int first, int last, int nt_out, T lam_scale, int chunk,
    int qh0, int nh) {
    static_assert(MODE == ADJ_PLAIN || MODE == ADJ_PLAIN2 || MODE == ADJ_SQUARED || MODE == ADJ_SQUARED_SYM,
                  "diagonal-storage modes");
    constexpr int RPW = 64 / LPR;
    constexpr int rows_per_wg = kWaves * RPW;
    constexpr bool kSym = MODE == ADJ_SQUARED_SYM;   // pair sums into the upper entries' half slots
    constexpr bool kSq = MODE == ADJ_SQUARED || kSym;
    constexpr bool kTwo = MODE == ADJ_PLAIN2;
    constexpr int NE = kSym ? (ND + 1) / 2 : ND;   // gradient slots of a row
    constexpr int PER = (NE + LPR - 1) / LPR;      // gradient slots per lane
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane / LPR;
    const int li = lane - g * LPR;
    // workgroup -> rows: contiguous XCD bands, or chunks of `chunk` workgroups
    // dealt to the XCDs in turn (as the Newton steps of a launch that streams
    // from HBM)
    int tile;
    if (chunk > 0) {
        const int x = blockIdx.x % kXcds, i = blockIdx.x / kXcds;
        tile = ((i / chunk) * kXcds + x) * chunk + i % chunk;
    } else {
        tile = xcd_tile(blockIdx.x, gridDim.x);
    }
    const int row = tile * rows_per_wg + wave * RPW + g;
    if (row >= n) return;                         // whole row groups leave together
    const int c0 = li * VEC;
    const bool inld = c0 < ld;
    const unsigned bits = pres[row];
    const int rp = row_ptr[row];
    // this lane's gradient slots (diagonals q = li, li + LPR, ...; with the
    // half accumulator the non-negative offsets q = qh0 + h, h = li, li + LPR,
    // ...), read ahead of the gathers
    using KIdx = std::conditional_t<kSym, long long, int>;
    KIdx kgs[PER];
    bool on[PER];
    double gold[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        if constexpr (kSym) {
            const int h = li + t * LPR, q = qh0 + h;
            on[t] = h < nh && q < nd && ((bits >> q) & 1u);
            kgs[t] = (long long)row * nh + h;
        } else {
            const int q = li + t * LPR;
            on[t] = q < nd && q < ND && ((bits >> q) & 1u);
            kgs[t] = rp + __popc(bits & ((1u << q) - 1u));
        }
        gold[t] = on[t] && !first ? grad[kgs[t]] : 0.0;
    }
    int cq[ND];
    T aq[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        const int c = row + off.o[q];
        const bool ok = q < nd && ((bits >> q) & 1u) && (unsigned)c < (unsigned)n;
        cq[q] = ok ? c : row;
        aq[q] = ok ? (constant ? cv.c[q] : dia[(size_t)row * nd + q]) : T(0);
    }
    // every gather of the row in flight at once
    Pack<T, VEC> own, wr, lq[ND], wq[ND], w2q[kTwo ? ND : 1];
#pragma unroll
    for (int e = 0; e < VEC; ++e) own.v[e] = wr.v[e] = T(0);
#pragma unroll
    for (int q = 0; q < ND; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            lq[q].v[e] = wq[q].v[e] = T(0);
            if (kTwo) w2q[q].v[e] = T(0);
        }
    // lam = lam_scale * lam_in (lam_scale = 0: a zero block, not read)
    const bool lam_on = lam_scale != T(0);
    if (inld) {
        if (lam_on) own = load_pack<T, VEC>(lam_in + (size_t)row * ld + c0);
        if (kSq) wr = load_pack<T, VEC>(w + (size_t)row * ld + c0);
#pragma unroll
        for (int q = 0; q < ND; ++q) {
            wq[q] = load_pack<T, VEC>(w + (size_t)cq[q] * ld + c0);
            if (lam_on) lq[q] = load_pack<T, VEC>(lam_in + (size_t)cq[q] * ld + c0);
            if (kTwo) w2q[q] = load_pack<T, VEC>(w2 + (size_t)cq[q] * ld + c0);
        }
    }
    if (lam_scale != T(1)) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) own.v[e] *= lam_scale;
#pragma unroll
        for (int q = 0; q < ND; ++q)
#pragma unroll
            for (int e = 0; e < VEC; ++e) lq[q].v[e] *= lam_scale;
    }
    bool valid[VEC];
    T sown[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        valid[e] = inld && c0 + e < ncols;
        T so = own.v[e];
        if (kSq) so = (c0 + e < wsplit ? T(1) : whi) * fma(p1, wr.v[e], so);
        sown[e] = valid[e] ? so : T(0);
    }
    // the Newton step (same products in the same order as the step kernels)
    T acc[VEC], accw[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] = accw[e] = T(0);
#pragma unroll
    for (int q = 0; q < ND; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            acc[e] = fma(aq[q], lq[q].v[e], acc[e]);
            if (kSq) accw[e] = fma(aq[q], wq[q].v[e], accw[e]);
        }
    Pack<T, VEC> o;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        T x = alpha * acc[e] - beta * own.v[e];
        if (kSq) x = fma(q1, alpha * accw[e] - beta * wr.v[e], fma(q0, wr.v[e], x));
        o.v[e] = x;
    }
    if (!last && inld) {
        if (nt_out)
            store_pack_nt<T, VEC>(lam_out + (size_t)row * ld + c0, o);
        else
            store_pack<T, VEC>(lam_out + (size_t)row * ld + c0, o);
    }
    // per-entry partial dot products: the lane's VEC products in the block's
    // precision (a select: padding columns may hold anything), then FP64 from
    // the sum over the row group on (widening every product to FP64 here would
    // double the kernel's registers and halve its occupancy: measured 3.30 ->
    // 3.06 gradient/estimate on the 2048^2 GMRF)
    double part[ND];
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        T p1q = T(0), p2q = T(0);
#pragma unroll
        for (int e = 0; e < VEC; ++e) p1q = valid[e] ? fma(sown[e], wq[q].v[e], p1q) : p1q;
        if (kSym && q > qh0) {   // the mirror (c, r): own at the neighbour times w at the row
            // (its own lane sum, as the CSR path forms it in row c)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const T oc = (c0 + e < wsplit ? T(1) : whi) * fma(p1, wq[q].v[e], lq[q].v[e]);
                p2q = valid[e] ? fma(oc, wr.v[e], p2q) : p2q;
            }
        }
        if (kTwo) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) p2q = valid[e] ? fma(o.v[e], w2q[q].v[e], p2q) : p2q;
        }
        part[q] = (double)p1q + (double)p2q;
    }
#pragma unroll
    for (int h = LPR / 2; h >= 1; h >>= 1)
#pragma unroll
        for (int q = 0; q < ND; ++q) part[q] += __shfl_xor(part[q], h, 64);
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        double v = 0.0;
        const int qsel = (kSym ? qh0 : 0) + li + t * LPR;
#pragma unroll
        for (int q = 0; q < ND; ++q) v = q == qsel ? part[q] : v;
        if (on[t]) grad[kgs[t]] = first ? (double)alpha * v : fma((double)alpha, v, gold[t]);
    }
}

template <typename T, int VEC, int LPR, int ND>
hipError_t launch_adjoint_dia_t(const CsrDev& A, const AdjArgs& a, const AdjDia& dg, hipStream_t st) {
    constexpr int rows_per_wg = kWaves * (64 / LPR);
    const int nwg = div_up(A.n, rows_per_wg);
    if (nwg == 0) return hipSuccess;
    DiaOff off{};
    DiaVal<T> cv{};
    for (int q = 0; q < kMaxDiag; ++q) {
        off.o[q] = q < dg.nd ? dg.off[q] : 0;
        cv.c[q] = (T)(q < dg.nd ? dg.cval[q] : 0.0);
    }
    // chunked XCD bands: chunks of dg.chunk_rows rows, in workgroups; the grid
    // covers whole rounds of 8 chunks (workgroups past the end return)
    const int cwg = dg.chunk_rows > 0 && dg.chunk_rows % rows_per_wg == 0 ? dg.chunk_rows / rows_per_wg : 0;
    const int grid = cwg > 0 ? div_up(div_up(nwg, cwg), kXcds) * kXcds * cwg : nwg;
#define LD_ADJ_DIA(M_)                                                                                          \
    hipLaunchKernelGGL((adjoint_dia_kernel<T, VEC, LPR, ND, M_>), dim3(grid), dim3(kThreads), 0, st, A.n, A.row_ptr, \
                       dg.pres, (const T*)dg.dia, dg.nd, off, cv, (int)dg.constant, (const T*)a.lam_in,          \
                       (T*)a.lam_out, (const T*)a.w, (const T*)a.w2, a.grad, a.ld, a.ncols, (T)a.alpha,          \
                       (T)a.beta, (T)a.q0, (T)a.q1, (T)a.p1, a.wsplit, (T)a.whi, (int)a.first, (int)a.last,      \
                       (int)a.nt_out, (T)a.lam_scale, cwg, dg.qh0, dg.nh)
    switch (a.mode) {
        case ADJ_PLAIN: LD_ADJ_DIA(ADJ_PLAIN); break;
        case ADJ_PLAIN2: LD_ADJ_DIA(ADJ_PLAIN2); break;
        case ADJ_SQUARED: LD_ADJ_DIA(ADJ_SQUARED); break;
        case ADJ_SQUARED_SYM:
            // offsets symmetric about the main diagonal, which sits at qh0
            if (dg.nh < 1 || dg.qh0 + dg.nh != dg.nd || 2 * dg.qh0 + 1 != dg.nd || dg.off[dg.qh0] != 0)
                return hipErrorInvalidValue;
            for (int h = 1; h < dg.nh; ++h)
                if (dg.off[dg.qh0 + h] != -dg.off[dg.qh0 - h]) return hipErrorInvalidValue;
            LD_ADJ_DIA(ADJ_SQUARED_SYM);
            break;
        default: return hipErrorInvalidValue;
    }
#undef LD_ADJ_DIA
    return hipGetLastError();
}

template <typename T, int VEC, int LPR>
hipError_t launch_adjoint_dia_l(const CsrDev& A, const AdjArgs& a, const AdjDia& dg, hipStream_t st) {
    if (dg.nd <= 3) return launch_adjoint_dia_t<T, VEC, LPR, 3>(A, a, dg, st);
    if (dg.nd <= 5) return launch_adjoint_dia_t<T, VEC, LPR, 5>(A, a, dg, st);
    if (dg.nd <= 7) return launch_adjoint_dia_t<T, VEC, LPR, 7>(A, a, dg, st);
    return launch_adjoint_dia_t<T, VEC, LPR, 9>(A, a, dg, st);
}

template <typename T, int VEC>
hipError_t launch_adjoint_dia_v(const CsrDev& A, const AdjArgs& a, const AdjDia& dg, hipStream_t st) {
    const int lanes = lanes_per_row(a.ncols, VEC);
    int lpr = 1;   // a power of two
    while (lpr < lanes) lpr <<= 1;
    if (lpr > 64 || a.ncols > a.ld || a.ld % VEC || dg.nd < 1 || dg.nd > kMaxDiag) return hipErrorInvalidValue;
    switch (lpr) {
        case 1: return launch_adjoint_dia_l<T, VEC, 1>(A, a, dg, st);
        case 2: return launch_adjoint_dia_l<T, VEC, 2>(A, a, dg, st);
        case 4: return launch_adjoint_dia_l<T, VEC, 4>(A, a, dg, st);
        case 8: return launch_adjoint_dia_l<T, VEC, 8>(A, a, dg, st);
        case 16: return launch_adjoint_dia_l<T, VEC, 16>(A, a, dg, st);
        case 32: return launch_adjoint_dia_l<T, VEC, 32>(A, a, dg, st);
        default: return launch_adjoint_dia_l<T, VEC, 64>(A, a, dg, st);
    }
}

hipError_t launch_adjoint_dia(bool f64, const CsrDev& A, const AdjArgs& a, const AdjDia& dg, hipStream_t st) {
    if (f64) return launch_adjoint_dia_v<double, 2>(A, a, dg, st);
    return launch_adjoint_dia_v<float, 4>(A, a, dg, st);
}

// The stored entries of row r from the half accumulator (one thread per row,
// grid-stride): diagonal q of r (present bit) sits at CSR position row_ptr[r]
// + (present diagonals below q); it takes the diagonal slot (q = qh0), or
// half the pair sum in the upper entry's slot: row r's own slot q - qh0 for
// q > qh0, row c's slot qm - qh0 of the mirrored diagonal qm = 2 qh0 - q for
// q < qh0.  An absent mirror sets *flag.
__global__ __launch_bounds__(kThreads) void expand_half_kernel(int n, const int* __restrict__ row_ptr,
                                                               const uint16_t* __restrict__ pres, int nd,
                                                               DiaOff off, int qh0, int nh,
                                                               const double* __restrict__ half,
                                                               double* __restrict__ g, int* __restrict__ flag) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < n; r += gridDim.x * kThreads) {
        const unsigned bits = pres[r];
        int k = row_ptr[r];
#pragma unroll
        for (int q = 0; q < kMaxDiag; ++q) {
            if (q >= nd || !((bits >> q) & 1u)) continue;
            double v;
            if (q == qh0) {
                v = half[(size_t)r * nh];
            } else {
                const int c = r + off.o[q], qm = 2 * qh0 - q;
                const bool mirror = (unsigned)c < (unsigned)n && qm >= 0 && qm < nd && ((pres[c] >> qm) & 1u);
                if (!mirror) *flag = 1;
                v = q > qh0 ? 0.5 * half[(size_t)r * nh + (q - qh0)]
                            : (mirror ? 0.5 * half[(size_t)c * nh + (qm - qh0)] : 0.0);
            }
            g[k++] = v;
        }
    }
}

hipError_t launch_expand_half(const CsrDev& A, const AdjDia& dg, const double* half, double* g, int* flag,
                              hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    if (dg.nh < 1 || dg.qh0 + dg.nh != dg.nd || dg.nd > kMaxDiag) return hipErrorInvalidValue;
    DiaOff off{};
    for (int q = 0; q < kMaxDiag; ++q) off.o[q] = q < dg.nd ? dg.off[q] : 0;
    const int nwg = std::min(div_up(A.n, kThreads), 4096);
    hipLaunchKernelGGL(expand_half_kernel, dim3(nwg), dim3(kThreads), 0, st, A.n, A.row_ptr, dg.pres, dg.nd, off,
                       dg.qh0, dg.nh, half, g, flag);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// g[e] and g[e'] of every mirrored pair of entries e = (r, c), e' = (c, r)
// become their mean; diagonal entries stay.  The pair is owned by its row r <
// c (one thread per row, grid-stride), which finds e' by binary search in row
// c (sorted columns); a missing mirror (the pattern is not symmetric) sets
// *flag to 1.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void symmetrize_kernel(int n, const int* __restrict__ row_ptr,
                                                             const int* __restrict__ col_idx,
                                                             double* __restrict__ g, int* __restrict__ flag) {
    for (int r = blockIdx.x * kThreads + threadIdx.x; r < n; r += gridDim.x * kThreads) {
        const int b = row_ptr[r], e = row_ptr[r + 1];
        for (int k = b; k < e; ++k) {
            const int c = col_idx[k];
            if (c <= r) continue;
            int lo = row_ptr[c], hi = row_ptr[c + 1];
            while (lo < hi) {   // first position in row c with column >= r
                const int mid = (lo + hi) >> 1;
                if (col_idx[mid] < r) lo = mid + 1;
                else hi = mid;
            }
            if (lo < row_ptr[c + 1] && col_idx[lo] == r) {
                const double m = 0.5 * (g[k] + g[lo]);
                g[k] = m;
                g[lo] = m;
            } else {
                *flag = 1;
            }
        }
    }
}

hipError_t launch_symmetrize(const CsrDev& A, double* g, int* flag, hipStream_t st) {
    if (A.n == 0) return hipSuccess;
    const int nwg = std::min(div_up(A.n, kThreads), 4096);
    hipLaunchKernelGGL(symmetrize_kernel, dim3(nwg), dim3(kThreads), 0, st, A.n, A.row_ptr, A.col_idx, g, flag);
    return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void narrow_kernel(long long len, const double* __restrict__ x,
                                                          float* __restrict__ y) {
    const long long i = (long long)blockIdx.x * kThreads + threadIdx.x;
    if (i < len) y[i] = (float)x[i];
}

hipError_t launch_narrow(long long len, const double* x, float* y, hipStream_t st) {
    if (len == 0) return hipSuccess;
    hipLaunchKernelGGL(narrow_kernel, dim3(div_up(len, kThreads)), dim3(kThreads), 0, st, len, x, y);
    return hipGetLastError();
}

hipError_t launch_adjoint(bool f64, const CsrDev& A, const AdjArgs& a, hipStream_t st) {
    if (f64) return launch_adjoint_v<double, 2>(A, a, st);
    return launch_adjoint_v<float, 4>(A, a, st);
}

}  // namespace ld
