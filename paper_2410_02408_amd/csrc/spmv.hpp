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
//   DIR     p_new = z + beta p_old is formed on the fly for every gathered
//           column and for the own row (stored); q = A p_new; sigma = p^T q.
//   SIGMA   q = A p for a p already updated; sigma = p^T q.
//   RESID   r = b - A x; ||b||^2 and ||r||^2.
//   LANCZOS v_j = z~ / beta, u_j = r~ / beta are normalised on the fly and
//           stored; w = A v_j; alpha_j = v_j^T w.
#pragma once

#include "common.hpp"

namespace bjp {

enum SpmvMode { SPMV_DIR = 0, SPMV_SIGMA = 1, SPMV_RESID = 2, SPMV_LANCZOS = 3 };

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
    const double *z;        // DIR: preconditioned residual
    double *p0, *p1;        // DIR/SIGMA: direction ping-pong, selected by st->it
    double *q;              // DIR/SIGMA: q = A p
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

#ifndef BJP_NT_CSR
#define BJP_NT_CSR 0
#endif
// CSR values and column indices are streamed once per product; loading them
// non-temporally keeps the gathered vector resident in the caches.
template <typename T>
__device__ __forceinline__ T csr_load(const T *p) {
#if BJP_NT_CSR
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

// The one place the updated direction is formed, so that the value gathered
// by a neighbouring row and the value stored for the own row are identical.
__device__ __forceinline__ double dir_value(double beta, const double *pold, const double *z, int i) {
    return __builtin_fma(beta, pold[i], z[i]);
}

// Rows [r0, r1) of the product in the given mode; accumulates this thread's
// share of the mode's dot products into d0, d1.  `st` is the state of the
// system the rows belong to.  Called by every thread of the workgroup.
template <int GS, int MODE>
__device__ __forceinline__ void spmv_rows(const SpmvArgs &a, const PcgState *st, int r0, int r1, double &d0,
                                          double &d1) {
    // U rows per lane group are processed together so that several
    // row_ptr -> col -> gather chains are in flight per lane.  The CSR
    // arrays must hold at least one entry (callers pass a zero entry for an
    // empty matrix).
    constexpr int U = spmv_rows_per_group(GS);
    constexpr int RWG = kWG / GS;
    const int tid = threadIdx.x, sub = tid & (GS - 1), grp = tid / GS;

    double beta = 0.0, invb = 0.0;
    const double *pold = nullptr, *src = nullptr;
    double *pnew = nullptr;
    if (MODE == SPMV_DIR || MODE == SPMV_SIGMA) {
        const int it = st->it;
        pold = (it & 1) ? a.p1 : a.p0;
        pnew = (it & 1) ? a.p0 : a.p1;
        beta = st->beta;
    }
    if (MODE == SPMV_SIGMA) src = pnew;
    if (MODE == SPMV_RESID) src = a.x;
    if (MODE == SPMV_LANCZOS) {
        invb = a.ls->invb;
        src = a.zt;
    }
    auto gather = [&](int col) -> double {
        if (MODE == SPMV_DIR) return dir_value(beta, pold, a.z, col);
        if (MODE == SPMV_LANCZOS) return src[col] * invb;
        return src[col];
    };

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
            if (MODE == SPMV_DIR) own[u] = dir_value(beta, pold, a.z, rc);
            else if (MODE == SPMV_SIGMA) own[u] = pnew[rc];
            else if (MODE == SPMV_RESID) own[u] = a.b[rc];
            else own[u] = a.zt[rc] * invb;
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
            if (MODE == SPMV_DIR) {
                pnew[i] = own[u];
                a.q[i] = acc[u];
                d0 += own[u] * acc[u];
            } else if (MODE == SPMV_SIGMA) {
                a.q[i] = acc[u];
                d0 += own[u] * acc[u];
            } else if (MODE == SPMV_RESID) {
                const double rv = own[u] - acc[u];
                a.r[i] = rv;
                d0 += own[u] * own[u];
                d1 += rv * rv;
            } else {
                const size_t at = (size_t)a.ls->j * a.ld + i;
                a.V[at] = own[u];
                if (a.has_m) a.U[at] = a.rt[i] * invb;
                a.w[i] = acc[u];
                d0 += own[u] * acc[u];
            }
        }
    }

}

template <int GS, int MODE>
__global__ __launch_bounds__(kWG) void k_spmv(SpmvArgs a) {
    if (MODE == SPMV_LANCZOS) {
        if (a.ls->done) return;
    } else if (!(MODE == SPMV_RESID && a.resid_phase == 1)) {
        if (a.st->done) return;
    }
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);
    double d0 = 0.0, d1 = 0.0;
    spmv_rows<GS, MODE>(a, a.st, r0, r1, d0, d1);
    const double v[2] = {d0, d1};
    block_partial<2>(v, a.partials);
}

// p_new = z + beta p_old for every row (the separate direction update used
// when the gathers of SPMV_DIR would be uncached random accesses).
__global__ __launch_bounds__(kWG) void k_direction(PcgState *st, const double *z, double *p0,
                                                   double *p1, int n) {
    if (st->done) return;
    const int it = st->it;
    const double *pold = (it & 1) ? p1 : p0;
    double *pnew = (it & 1) ? p0 : p1;
    const double beta = st->beta;
    for (int i = blockIdx.x * kWG + threadIdx.x; i < n; i += gridDim.x * kWG)
        pnew[i] = dir_value(beta, pold, z, i);
}

}  // namespace bjp
