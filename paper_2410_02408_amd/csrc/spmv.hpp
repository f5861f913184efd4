// CSR sparse matrix-vector products with fused vector work and dot products.
//
// Schedule: a group of GS lanes (GS a power of two <= 64) works on one row;
// lane `sub` of the group takes entries sub, sub+GS, ... of the row, so the
// lanes of a wave read consecutive CSR entries (coalesced val/col loads), and
// the group's partial sums are combined with xor-shuffles.  A workgroup of
// 256 lanes covers 256/GS rows per step and walks a contiguous chunk of rows
// (XCD-aware chunk order).  GS is a launch parameter chosen from the mean
// row length (short stencil rows: GS = 8; long power-law rows: GS = 32..64).
//
// Modes (what is gathered, what is written, which dots are reduced):
//   SIGMA   q = A p for the current direction p; sigma = p^T q.
//   RESID   r = b - A x; ||b||^2 and ||r||^2.
//   LANCZOS v_j = z~ / beta, u_j = r~ / beta are normalised on the fly and
//           stored; w = A v_j; alpha_j = v_j^T w.
#pragma once

#include "common.hpp"
#include "finish.hpp"

namespace bjp {

enum SpmvMode { SPMV_SIGMA = 0, SPMV_RESID = 1, SPMV_LANCZOS = 2 };

#ifndef BJP_SPMV_ROWS
#define BJP_SPMV_ROWS 2
#endif
// Rows each lane group keeps in flight per step.
__host__ __device__ constexpr int spmv_rows_per_group(int gs) { return gs <= 16 ? BJP_SPMV_ROWS : 2; }

#ifndef BJP_SPMV_PASSES
#define BJP_SPMV_PASSES 1
#endif
// Entries per row loaded in the unrolled first stage: passes * GS; longer rows
// continue in a loop.  (Two unrolled passes of 4 lanes for 7-entry stencil
// rows measured slower than one pass plus the loop.)
__host__ __device__ constexpr int spmv_passes(int gs) { return gs <= 4 ? BJP_SPMV_PASSES : 1; }

struct SpmvArgs {
    int n, chunk;
    const int32_t *rp, *ci;
    const double *val;
    PcgState *st;
    double *p0, *p1;        // SIGMA: direction ping-pong, selected by the iteration count
    double *q;              // SIGMA: q = A p
    const double *b;        // RESID
    const double *x;        // RESID
    double *r;              // RESID: r = b - A x
    int resid_phase;        // RESID: 0 = start of a solve, 1 = true residual (runs when done)
    LanczosState *ls;       // LANCZOS
    const double *zt, *rt;  // LANCZOS: vectors to normalise (zt == rt when M = I)
    double *V, *U;          // LANCZOS: bases, vector l at l*ld (U unused when M = I)
    size_t ld;
    double *w;              // LANCZOS: w = A v_j
    int has_m;
    double *partials;       // per-workgroup dots (see the modes)
    // optional for the row-block streaming schedule: column indices stored as
    // 16-bit offsets from the first row of their 256-row block (cd), used
    // when *cd_bad == 0 (every offset fitted)
    const int16_t *cd;
    const int32_t *cd_bad;
};

// CSR values and column indices are streamed once per product.  Loaded
// non-temporally (NT) they leave the caches to the gathered vector; that pays
// only when the matrix exceeds the last-level cache: a single system's CSR
// that fits stays resident from one product to the next if loaded normally
// (measured at 128^3: +7 us per product with NT loads), while the batch's
// 3.1 GB CSR does not (row-block streaming over the 512-system batch: 58.2 ->
// 55.3 ms per solve with NT loads).
template <bool NT = false, typename T>
__device__ __forceinline__ T csr_load(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// The updated direction p_new = z + beta p_old of row i (one rounding).
__device__ __forceinline__ double dir_value(double beta, const double *pold, const double *z, int i) {
    return __builtin_fma(beta, pold[i], z[i]);
}

// What a mode gathers for a column, the own-row value it needs, and what it
// stores and accumulates once a row's product is known.  Shared by both
// schedules below.
template <int MODE>
struct SpmvMode_ {
    const SpmvArgs &a;
    double invb = 0.0;
    const double *src = nullptr;
    const double *pnew = nullptr;

    // it: iteration count of the system's state (selects the direction buffer)
    __device__ __forceinline__ SpmvMode_(const SpmvArgs &args, int it) : a(args) {
        if (MODE == SPMV_SIGMA) {
            pnew = (it & 1) ? a.p0 : a.p1;
            src = pnew;
        }
        if (MODE == SPMV_RESID) src = a.x;
        if (MODE == SPMV_LANCZOS) {
            invb = a.ls->invb;
            src = a.zt;
        }
    }
    __device__ __forceinline__ double gather(int col) const {
        if (MODE == SPMV_LANCZOS) return src[col] * invb;
        return src[col];
    }
    __device__ __forceinline__ double own(int i) const {
        if (MODE == SPMV_SIGMA) return pnew[i];
        if (MODE == SPMV_RESID) return a.b[i];
        return a.zt[i] * invb;
    }
    // row i with own value ov and product acc = (A s)_i
    __device__ __forceinline__ void finish(int i, double ov, double acc, double &d0, double &d1) const {
        if (MODE == SPMV_SIGMA) {
            a.q[i] = acc;
            d0 += ov * acc;
        } else if (MODE == SPMV_RESID) {
            const double rv = ov - acc;
            a.r[i] = rv;
            d0 += ov * ov;
            d1 += rv * rv;
        } else {
            const size_t at = (size_t)a.ls->j * a.ld + i;
            a.V[at] = ov;
            if (a.has_m) a.U[at] = a.rt[i] * invb;
            a.w[i] = acc;
            d0 += ov * acc;
        }
    }
};

// Rows [r0, r1) of the product in the given mode; accumulates this thread's
// share of the mode's dot products into d0, d1.  `st` is the state of the
// system the rows belong to.  Called by every thread of the workgroup.
template <int GS, int MODE>
__device__ __forceinline__ void spmv_rows(const SpmvArgs &a, int it, int r0, int r1, double &d0, double &d1) {
    // U rows per lane group are processed together so that several
    // row_ptr -> col -> gather chains are in flight per lane.  The CSR
    // arrays must hold at least one entry (callers pass a zero entry for an
    // empty matrix).
    constexpr int U = spmv_rows_per_group(GS);
    constexpr int RWG = kWG / GS;
    const int tid = threadIdx.x, sub = tid & (GS - 1), grp = tid / GS;
    const SpmvMode_<MODE> m(a, it);
    auto gather = [&](int col) -> double { return m.gather(col); };

    // All loads of a step are unconditional (out-of-range rows and lanes use
    // clamped, in-bounds indices and are masked afterwards), so the compiler
    // issues them back to back instead of one exec-masked block at a time.
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const double *__restrict__ val = a.val;
    for (int base = r0; base < r1; base += RWG * U) {
        int kb[U], ke[U], row[U];
        double own[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            row[u] = base + u * RWG + grp;
            const int rc = min(row[u], r1 - 1);
            const int b0 = rp[rc], e0 = rp[rc + 1];
            const bool ok = row[u] < r1;
            kb[u] = ok ? b0 : 0;
            ke[u] = ok ? e0 : 0;
            own[u] = m.own(rc);
        }
        constexpr int NP = spmv_passes(GS);
        int col[U][NP];
        double vv[U][NP], acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) {
                const int k = kb[u] + sub + pp * GS;
                const int kc = k < ke[u] ? k : 0;
                col[u][pp] = csr_load(ci + kc);
                vv[u][pp] = csr_load(val + kc);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc[u] = 0.0;
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) {
                const bool valid = kb[u] + sub + pp * GS < ke[u];
                const double xv = gather(valid ? col[u][pp] : 0);
                acc[u] += valid ? vv[u][pp] * xv : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            for (int k = kb[u] + sub + NP * GS; k < ke[u]; k += GS) acc[u] += csr_load(val + k) * gather(csr_load(ci + k));
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int off = GS / 2; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off, 64);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = row[u];
            if (i >= r1 || sub != 0) continue;
            m.finish(i, own[u], acc[u], d0, d1);
        }
    }
}

// Row-block streaming schedule for short rows: a workgroup takes blocks of
// kStreamRows consecutive rows; the block's CSR entries are read fully
// coalesced (thread t takes entries t, t + 256, ...), multiplied by their
// gathered vector entries and staged in LDS, kStreamCap at a time; then
// thread t sums the products of row t of the block in entry order.  Every
// load of a stage is issued before the first is used.
#ifndef BJP_STREAM_CAP
#define BJP_STREAM_CAP 1024
#endif
constexpr int kStreamRows = kWG;
constexpr int kStreamCap = BJP_STREAM_CAP;
constexpr int kStreamPer = kStreamCap / kWG;

// prod: the caller's LDS stage of PER * kWG doubles (one array per kernel,
// shared by the instantiations a kernel chooses between, so it is counted once
// against the CU's LDS).
template <int MODE, bool NT = false, int PER = kStreamPer, bool CD = false>
__device__ __forceinline__ void spmv_stream_rows(const SpmvArgs &a, int it, int r0, int r1, double &d0,
                                                 double &d1, double *prod) {
    constexpr int CAP = PER * kWG;   // entries per stage
    const int tid = threadIdx.x;
    const SpmvMode_<MODE> m(a, it);
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const int16_t *__restrict__ cd = a.cd;
    const double *__restrict__ val = a.val;
    for (int b0 = r0; b0 < r1; b0 += kStreamRows) {
        const int b1 = min(b0 + kStreamRows, r1);
        const int i = b0 + tid;
        const int ic = min(i, b1 - 1);
        const int kb = rp[ic], ke = rp[ic + 1];
        const int base = rp[b0], end = rp[b1];
        const double ov = m.own(ic);
        double acc = 0.0;
        for (int c0 = base; c0 < end; c0 += CAP) {
            const int c1 = min(c0 + CAP, end);
            int col[PER];
            double vv[PER];
#pragma unroll
            for (int j = 0; j < PER; ++j) {
                const int k = c0 + j * kWG + tid;
                const int kc = k < c1 ? k : c0;
                if constexpr (CD) col[j] = b0 + (int)csr_load<NT>(cd + kc);
                else col[j] = csr_load<NT>(ci + kc);
                vv[j] = csr_load<NT>(val + kc);
            }
#pragma unroll
            for (int j = 0; j < PER; ++j) prod[j * kWG + tid] = vv[j] * m.gather(col[j]);
            __syncthreads();
            const int lo = max(kb, c0), hi = min(ke, c1);
            for (int k = lo; k < hi; ++k) acc += prod[k - c0];
            __syncthreads();
        }
        if (i < b1) m.finish(i, ov, acc, d0, d1);
    }
}

// Whether the launch has work, and the iteration count it needs.
template <int MODE>
__device__ __forceinline__ bool spmv_state(const SpmvArgs &a, int &it) {
    if (MODE == SPMV_LANCZOS) return !a.ls->done;
    if (MODE == SPMV_SIGMA) {
        it = a.st->it;
        return !a.st->done;
    }
    return a.resid_phase == 1 || !a.st->done;
}

template <int GS, int MODE>
__global__ __launch_bounds__(kWG) void k_spmv(SpmvArgs a) {
    int it = 0;
    if (!spmv_state<MODE>(a, it)) return;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);
    double d0 = 0.0, d1 = 0.0;
    spmv_rows<GS, MODE>(a, it, r0, r1, d0, d1);
    const double v[2] = {d0, d1};
    block_partial<2>(v, a.partials);
}

// PER entries per thread and stage: 7 for rows of at most 7 entries on
// average (a 256-row block of a 7-point stencil is then one stage: 40.1 instead
// of 41.6 us per product at 128^3), else 4.
template <int MODE, int PER>
__global__ __launch_bounds__(kWG) void k_spmv_stream(SpmvArgs a) {
    int it = 0;
    if (!spmv_state<MODE>(a, it)) return;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);
    double d0 = 0.0, d1 = 0.0;
    __shared__ double prod[PER * kWG];
    if (a.cd != nullptr && *a.cd_bad == 0) spmv_stream_rows<MODE, false, PER, true>(a, it, r0, r1, d0, d1, prod);
    else spmv_stream_rows<MODE, false, PER, false>(a, it, r0, r1, d0, d1, prod);
    const double v[2] = {d0, d1};
    block_partial<2>(v, a.partials);
}

// The direction update, with the deferred update decision as prologue: every
// workgroup takes it from the partials of the block-inverse application
// (r^T z, r^T r) and the state src; workgroup 0 records the new state at dst.
// It also applies the x update owed by the last step (x += alpha p_old, with
// that step's alpha), also when the decision ends the solve; then, unless the
// solve is done, p_new = z + beta p_old.  The loads of the first kDirRows rows
// of each thread are issued before the decision (which buffer is p_old
// follows from src alone).  x is read and written non-temporally: nothing
// reads it before the next direction update, and keeping it out of the caches
// leaves them to p_new, which the product gathers next (measured at 128^3:
// product 43 -> 38 us, this kernel 13.7 -> 15.4 us).
#ifndef BJP_DIR_ROWS
#define BJP_DIR_ROWS 8
#endif
constexpr int kDirRows = BJP_DIR_ROWS;

// p_old of the direction update that follows the state s (the p of the last step).
__device__ __forceinline__ int dir_parity(const PcgState *s) { return (s->it + (s->pending ? 1 : 0)) & 1; }

template <int OP>
__global__ __launch_bounds__(kWG) void k_direction(const PcgState *src, PcgState *dst, const double *partials,
                                                   int nparts, double *hist, const double *z, double *p0,
                                                   double *p1, double *x, int n) {
    const int par = dir_parity(src);
    const double *pold = par ? p1 : p0;
    double *pnew = par ? p0 : p1;
    const bool xup = src->xpend;
    const double alpha = src->alpha;
    const int stride = gridDim.x * kWG;
    const int i0 = blockIdx.x * kWG + threadIdx.x;
    double zv[kDirRows], pv[kDirRows], xv[kDirRows];
#pragma unroll
    for (int j = 0; j < kDirRows; ++j) {
        const int i = min(i0 + j * stride, n - 1);
        zv[j] = z[i];
        pv[j] = pold[i];
        xv[j] = xup ? __builtin_nontemporal_load(x + i) : 0.0;
    }
    const PcgState L = shared_decide<OP>(src, dst, partials, nparts, hist);
    if (xup) {
#pragma unroll
        for (int j = 0; j < kDirRows; ++j) {
            const int i = i0 + j * stride;
            if (i < n) __builtin_nontemporal_store(__builtin_fma(alpha, pv[j], xv[j]), x + i);
        }
        for (int i = i0 + kDirRows * stride; i < n; i += stride) x[i] = __builtin_fma(alpha, pold[i], x[i]);
    }
    if (L.done) return;
    const double beta = L.beta;
#pragma unroll
    for (int j = 0; j < kDirRows; ++j) {
        const int i = i0 + j * stride;
        if (i < n) pnew[i] = __builtin_fma(beta, pv[j], zv[j]);
    }
    for (int i = i0 + kDirRows * stride; i < n; i += stride) pnew[i] = dir_value(beta, pold, z, i);
}

// The x update still owed at the end of a solve (no direction update follows).
__global__ __launch_bounds__(kWG) void k_x_finish(const PcgState *st, const double *p0, const double *p1, double *x,
                                                  int n) {
    if (!st->xpend) return;
    const double *pold = dir_parity(st) ? p1 : p0;
    const double alpha = st->alpha;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) x[i] = __builtin_fma(alpha, pold[i], x[i]);
}

__global__ void k_x_finish_clear(PcgState *st) {
    if (threadIdx.x == 0) st->xpend = 0;
}

// Start of a solve from x = 0: the residual b - A x is b itself, so instead
// of the residual product this copies b into r and leaves the partials that
// product would (b^T b, r^T r), in its own per-workgroup layout.
__global__ __launch_bounds__(kWG) void k_start_zero(const double *b, double *r, double *partials, int n) {
    double d = 0.0;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
        const double v = b[i];
        r[i] = v;
        d += v * v;
    }
    const double v[2] = {d, d};
    block_partial<2>(v, partials);
}

}  // namespace bjp

namespace bjp {

// Column indices as 16-bit offsets from the first row of the entry's 256-row
// block (the streaming schedule's block): for banded matrices such as 3D
// stencils every offset fits, and the product then reads 2 instead of 4 bytes
// per entry for its columns (measured at 128^3: 37.1 -> 34.9 us per product).
// The choice between the two is made per launch from *bad, outside the
// unrolled loads (a select between them had the compiler issue both).
// *bad is set when some offset does not fit; the product then reads the
// 32-bit indices.
__global__ __launch_bounds__(kWG) void k_col_delta16(const int32_t *rp, const int32_t *ci, int n, int16_t *cd,
                                                    int32_t *bad) {
    for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG) {
        const int b0 = i - i % kStreamRows;
        bool fits = true;
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
            const int d = ci[k] - b0;
            fits = fits && d >= -32768 && d <= 32767;
            cd[k] = (int16_t)d;
        }
        if (!fits) atomicMax(bad, 1);
    }
}

// ---------------------------------------------------------------------------
// Column-panel product for long random-gather rows (the power-law family),
// whose gathered vector exceeds an XCD's L2: a random 8-byte gather costs an
// L2 request, and once the vector no longer fits the L2 each one goes on to
// the last-level cache.  The columns are cut into kPanels contiguous panels
// and the matrix is copied once per solve panel-major (panel q holds the
// entries whose column lies in q, row by row, in the order they have in the
// row).  Workgroup b of the product takes panel b mod kPanels (the
// workgroups of one panel then run on one XCD, whose L2 holds that slice of
// the vector) and a chunk of rows, and writes per-panel partial sums;
// a second launch adds the kPanels partial sums of each row in panel order
// and finishes the row as the plain product does.  Measured with random
// columns over a 32 MB vector (4M rows, 143M entries) and a group of lanes
// per row: 2.75 ms for the plain product, 1.62 ms with 8 panels (16 panels:
// 2.0 ms).
// ---------------------------------------------------------------------------
constexpr int kPanels = 8;
constexpr int kScanRows = 2048;      // rows per workgroup of the offset scan (8 per thread)

struct PanelArgs {
    int n, width;               // panel q: columns [q*width, (q+1)*width)
    int nnz;                    // entries of A (bound of the copy)
    const int32_t *rp, *ci;     // the caller's CSR
    const double *val;
    int32_t *cnt;               // [kPanels][n] entries per (panel, row)
    int32_t *bsum;              // [kPanels][nscan] per scan block: sums, then offsets
    int nscan;
    int32_t *prp;               // [kPanels][n + 1] row pointers into the copy
    int32_t *pci;               // [nnz] panel-major copy
    double *pval;
    double *Y;                  // [kPanels][n] partial products
};

// Panel of a column (col < n, so the result is < kPanels).
__device__ __forceinline__ int panel_of(int col, int width) { return col / width; }

// The build walks each row with a group of kBuildLanes lanes (rows are up
// to thousands of entries long, so one thread per row would leave a long
// tail and uncoalesced reads).
constexpr int kBuildLanes = 16;

// cnt[q][i] = entries of row i in panel q.
__global__ __launch_bounds__(kWG) void k_panel_count(PanelArgs a) {
    const int sub = threadIdx.x % kBuildLanes;
    const int groups = gridDim.x * (kWG / kBuildLanes);
    for (int i = blockIdx.x * (kWG / kBuildLanes) + threadIdx.x / kBuildLanes; i < a.n; i += groups) {
        int c[kPanels];
#pragma unroll
        for (int q = 0; q < kPanels; ++q) c[q] = 0;
        for (int k = a.rp[i] + sub; k < a.rp[i + 1]; k += kBuildLanes) {
            const int p = panel_of(a.ci[k], a.width);
#pragma unroll
            for (int q = 0; q < kPanels; ++q) c[q] += p == q;
        }
#pragma unroll
        for (int q = 0; q < kPanels; ++q) {
#pragma unroll
            for (int off = kBuildLanes / 2; off > 0; off >>= 1) c[q] += __shfl_xor(c[q], off, 64);
        }
        if (sub < kPanels) {
            int v = 0;
#pragma unroll
            for (int q = 0; q < kPanels; ++q) v = sub == q ? c[q] : v;
            a.cnt[(size_t)sub * a.n + i] = v;
        }
    }
}

// Inclusive prefix sum over the workgroup of one value per thread (fixed order).
__device__ __forceinline__ int block_scan_incl(int v, int *lds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int u = __shfl_up(v, off, 64);
        if (lane >= off) v += u;
    }
    if (lane == 63) lds[wave] = v;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += lds[w];
    __syncthreads();
    return v + add;
}

// bsum[q][b] = entries of panel q in the rows of scan block b.
__global__ __launch_bounds__(kWG) void k_panel_blocksum(PanelArgs a) {
    __shared__ int lds[kWaves];
    const int b = blockIdx.x;
    const int i0 = b * kScanRows + threadIdx.x * (kScanRows / kWG);
    for (int q = 0; q < kPanels; ++q) {
        int s = 0;
        for (int u = 0; u < kScanRows / kWG; ++u) {
            const int i = i0 + u;
            if (i < a.n) s += a.cnt[(size_t)q * a.n + i];
        }
        const int tot = block_scan_incl(s, lds);
        if (threadIdx.x == kWG - 1) a.bsum[(size_t)q * a.nscan + b] = tot;
    }
}

// One workgroup: bsum[q][b] becomes the offset of scan block b within the
// copy (panels one after another), and prp[q][n] the end of panel q.
__global__ __launch_bounds__(kWG) void k_panel_blockscan(PanelArgs a) {
    __shared__ int lds[kWaves];
    __shared__ int total;
    int base = 0;
    for (int q = 0; q < kPanels; ++q) {
        int32_t *bs = a.bsum + (size_t)q * a.nscan;
        for (int b0 = 0; b0 < a.nscan; b0 += kWG) {
            const int b = b0 + threadIdx.x;
            const int v = b < a.nscan ? bs[b] : 0;
            const int incl = block_scan_incl(v, lds);
            if (b < a.nscan) bs[b] = base + incl - v;
            if (threadIdx.x == kWG - 1) total = incl;
            __syncthreads();
            base += total;
            __syncthreads();
        }
        if (threadIdx.x == 0) a.prp[(size_t)q * (a.n + 1) + a.n] = base;
    }
}

// prp[q][i] = start of row i's entries of panel q in the copy.
__global__ __launch_bounds__(kWG) void k_panel_offsets(PanelArgs a) {
    __shared__ int lds[kWaves];
    const int b = blockIdx.x;
    constexpr int R = kScanRows / kWG;
    const int i0 = b * kScanRows + threadIdx.x * R;
    for (int q = 0; q < kPanels; ++q) {
        int c[R];
        int s = 0;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            c[u] = i0 + u < a.n ? a.cnt[(size_t)q * a.n + i0 + u] : 0;
            s += c[u];
        }
        int off = a.bsum[(size_t)q * a.nscan + b] + block_scan_incl(s, lds) - s;
#pragma unroll
        for (int u = 0; u < R; ++u) {
            if (i0 + u < a.n) a.prp[(size_t)q * (a.n + 1) + i0 + u] = off;
            off += c[u];
        }
    }
}

// Copies each row's entries to their panels, in row order: a group takes
// kBuildLanes consecutive entries at a time; an entry's place is its panel's
// next free slot plus the number of lower lanes of the group whose entry
// falls in the same panel (ballots), so the copy keeps the row's order.
__global__ __launch_bounds__(kWG) void k_panel_scatter(PanelArgs a) {
    const int lane = threadIdx.x & 63, sub = threadIdx.x % kBuildLanes;
    const unsigned long long gmask = ((1ull << kBuildLanes) - 1) << (lane - sub);
    const unsigned long long below = gmask & ((1ull << lane) - 1);
    const int groups = gridDim.x * (kWG / kBuildLanes);
    for (int i = blockIdx.x * (kWG / kBuildLanes) + threadIdx.x / kBuildLanes; i < a.n; i += groups) {
        int pos[kPanels];
#pragma unroll
        for (int q = 0; q < kPanels; ++q) pos[q] = a.prp[(size_t)q * (a.n + 1) + i];
        const int ke = a.rp[i + 1];
        for (int k0 = a.rp[i]; k0 < ke; k0 += kBuildLanes) {
            const int k = k0 + sub;
            const bool valid = k < ke;
            const int col = valid ? a.ci[k] : 0;
            const double v = valid ? a.val[k] : 0.0;
            const int p = valid ? panel_of(col, a.width) : -1;
            int at = 0;
#pragma unroll
            for (int q = 0; q < kPanels; ++q) {
                const unsigned long long m = __ballot(p == q) & gmask;
                if (p == q) at = pos[q] + __popcll(m & below);
                pos[q] += __popcll(m);
            }
            if (valid && at < a.nnz) {
                a.pci[at] = col;
                a.pval[at] = v;
            }
        }
    }
}

// Y[q][i] = sum over row i's entries in panel q (of the mode's gathered
// vector), in their order.  Workgroup b takes panel b mod kPanels and chunks
// of kPanelChunk rows of it; a chunk's entries of the panel are contiguous in
// the copy (about 4 per row on the power-law family, hundreds for hub rows)
// and are streamed as in the row-block product: thread t loads entries t,
// t + 256, ... of a stage (kPanelPer per thread, all issued before the
// gathers, so each thread keeps kPanelPer gathers in flight and every lane
// has work), stages the products in LDS, and then adds the products of its
// kPanelRows rows (t, t + 256, ...) in order.  Measured on the power-law
// workload (4M rows, 134M entries): 1.55 ms per product with a group of 8
// lanes per row, 1.05 ms streaming 4 entries per thread over 256-row chunks,
// 1.02 ms with 8 entries per thread over 512-row chunks (8 over 256 rows:
// 1.11 ms, half the loads past the chunk's end; gathers that bypass the L1
// through buffer loads at device scope: 1.08 ms).
constexpr int kPanelPer = 8;
constexpr int kPanelRows = 2;
constexpr int kPanelChunk = kPanelRows * kWG;
template <int MODE>
__global__ __launch_bounds__(kWG) void k_spmv_panels(SpmvArgs s, PanelArgs a) {
    int it = 0;
    if (!spmv_state<MODE>(s, it)) return;
    const SpmvMode_<MODE> m(s, it);
    constexpr int CAP = kPanelPer * kWG;
    __shared__ double prod[CAP];
    const int q = blockIdx.x % kPanels;
    const int32_t *__restrict__ prp = a.prp + (size_t)q * (a.n + 1);
    const int tid = threadIdx.x;
    const int nchunks = (a.n + kPanelChunk - 1) / kPanelChunk, cstride = gridDim.x / kPanels;
    for (int c = blockIdx.x / kPanels; c < nchunks; c += cstride) {
        const int b0 = c * kPanelChunk, b1 = min(b0 + kPanelChunk, a.n);
        int kb[kPanelRows], ke[kPanelRows];
        double acc[kPanelRows];
#pragma unroll
        for (int u = 0; u < kPanelRows; ++u) {
            const int ic = min(b0 + u * kWG + tid, b1 - 1);
            kb[u] = prp[ic];
            ke[u] = prp[ic + 1];
            acc[u] = 0.0;
        }
        const int base = prp[b0], end = min(prp[b1], a.nnz);
        for (int c0 = base; c0 < end; c0 += CAP) {
            const int c1 = min(c0 + CAP, end);
            int col[kPanelPer];
            double vv[kPanelPer];
#pragma unroll
            for (int j = 0; j < kPanelPer; ++j) {
                const int k = c0 + j * kWG + tid;
                const int kc = k < c1 ? k : c0;
                col[j] = __builtin_nontemporal_load(a.pci + kc);
                vv[j] = __builtin_nontemporal_load(a.pval + kc);
            }
#pragma unroll
            for (int j = 0; j < kPanelPer; ++j) prod[j * kWG + tid] = vv[j] * m.gather(col[j]);
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kPanelRows; ++u) {
                const int lo = max(kb[u], c0), hi = min(ke[u], c1);
                for (int k = lo; k < hi; ++k) acc[u] += prod[k - c0];
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < kPanelRows; ++u) {
            const int i = b0 + u * kWG + tid;
            if (i < b1) __builtin_nontemporal_store(acc[u], a.Y + (size_t)q * a.n + i);
        }
    }
}

// Row i's product = the panel partial sums in panel order; then the mode's
// row finish and the per-workgroup dots, as the plain product.
template <int MODE>
__global__ __launch_bounds__(kWG) void k_panel_finish(SpmvArgs s, PanelArgs a) {
    int it = 0;
    if (!spmv_state<MODE>(s, it)) return;
    const SpmvMode_<MODE> m(s, it);
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * s.chunk, r1 = min(r0 + s.chunk, a.n);
    double d0 = 0.0, d1 = 0.0;
    for (int i = r0 + threadIdx.x; i < r1; i += kWG) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < kPanels; ++q) acc += __builtin_nontemporal_load(a.Y + (size_t)q * a.n + i);
        m.finish(i, m.own(i), acc, d0, d1);
    }
    const double v[2] = {d0, d1};
    block_partial<2>(v, s.partials);
}

}  // namespace bjp
