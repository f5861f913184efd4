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

template <int MODE, bool NT = false>
__device__ __forceinline__ void spmv_stream_rows(const SpmvArgs &a, int it, int r0, int r1, double &d0,
                                                 double &d1) {
    __shared__ double prod[kStreamCap];
    const int tid = threadIdx.x;
    const SpmvMode_<MODE> m(a, it);
    const int32_t *__restrict__ rp = a.rp;
    const int32_t *__restrict__ ci = a.ci;
    const double *__restrict__ val = a.val;
    for (int b0 = r0; b0 < r1; b0 += kStreamRows) {
        const int b1 = min(b0 + kStreamRows, r1);
        const int i = b0 + tid;
        const int ic = min(i, b1 - 1);
        const int kb = rp[ic], ke = rp[ic + 1];
        const int base = rp[b0], end = rp[b1];
        const double ov = m.own(ic);
        double acc = 0.0;
        for (int c0 = base; c0 < end; c0 += kStreamCap) {
            const int c1 = min(c0 + kStreamCap, end);
            int col[kStreamPer];
            double vv[kStreamPer];
#pragma unroll
            for (int j = 0; j < kStreamPer; ++j) {
                const int k = c0 + j * kWG + tid;
                const int kc = k < c1 ? k : c0;
                col[j] = csr_load<NT>(ci + kc);
                vv[j] = csr_load<NT>(val + kc);
            }
#pragma unroll
            for (int j = 0; j < kStreamPer; ++j) prod[j * kWG + tid] = vv[j] * m.gather(col[j]);
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

template <int MODE>
__global__ __launch_bounds__(kWG) void k_spmv_stream(SpmvArgs a) {
    int it = 0;
    if (!spmv_state<MODE>(a, it)) return;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);
    double d0 = 0.0, d1 = 0.0;
    spmv_stream_rows<MODE>(a, it, r0, r1, d0, d1);
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

}  // namespace bjp
