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
    int resid_phase;        // RESID: 0 = start of a solve, 1 = final true residual
    double *hist;
    LanczosState *ls;       // LANCZOS
    const double *zt, *rt;  // LANCZOS: vectors to normalise (zt == rt when M = I)
    double *V, *U;          // LANCZOS: bases, vector l at l*ld (U unused when M = I)
    size_t ld;
    double *w;              // LANCZOS: w = A v_j
    double *alpha_out;      // LANCZOS
    int has_m;
    double *partials;
};

// The one place the updated direction is formed, so that the value gathered
// by a neighbouring row and the value stored for the own row are identical.
__device__ __forceinline__ double dir_value(double beta, const double *pold, const double *z, int i) {
    return __builtin_fma(beta, pold[i], z[i]);
}

template <int GS, int MODE>
__global__ __launch_bounds__(kWG) void k_spmv(SpmvArgs a) {
    if (MODE == SPMV_LANCZOS) {
        if (a.ls->done) return;
    } else if (!(MODE == SPMV_RESID && a.resid_phase == 1)) {
        if (a.st->done) return;
    }
    // U rows per lane group are processed together so that several
    // row_ptr -> col -> gather chains are in flight per lane.
    constexpr int U = GS <= 16 ? 4 : 2;
    constexpr int RWG = kWG / GS;
    const int tid = threadIdx.x, sub = tid & (GS - 1), grp = tid / GS;
    const int c = xcd_chunk(blockIdx.x, gridDim.x);
    const int r0 = c * a.chunk;
    const int r1 = min(r0 + a.chunk, a.n);

    double beta = 0.0, invb = 0.0;
    const double *pold = nullptr, *src = nullptr;
    double *pnew = nullptr;
    if (MODE == SPMV_DIR || MODE == SPMV_SIGMA) {
        const int it = a.st->it;
        pold = (it & 1) ? a.p1 : a.p0;
        pnew = (it & 1) ? a.p0 : a.p1;
        beta = a.st->beta;
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

    double d0 = 0.0, d1 = 0.0;
    for (int base = r0; base < r1; base += RWG * U) {
        int kb[U], ke[U], row[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            row[u] = base + u * RWG + grp;
            kb[u] = 0;
            ke[u] = 0;
            if (row[u] < r1) {
                kb[u] = a.rp[row[u]];
                ke[u] = a.rp[row[u] + 1];
            }
        }
        int col[U];
        double vv[U], acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            col[u] = 0;
            vv[u] = 0.0;
            const int k = kb[u] + sub;
            if (k < ke[u]) {
                col[u] = a.ci[k];
                vv[u] = a.val[k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double xv = 0.0;
            if (kb[u] + sub < ke[u]) xv = gather(col[u]);
            acc[u] = vv[u] * xv;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            for (int k = kb[u] + sub + GS; k < ke[u]; k += GS) acc[u] += a.val[k] * gather(a.ci[k]);
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
                const double pv = dir_value(beta, pold, a.z, i);
                pnew[i] = pv;
                a.q[i] = acc[u];
                d0 += pv * acc[u];
            } else if (MODE == SPMV_SIGMA) {
                a.q[i] = acc[u];
                d0 += pnew[i] * acc[u];
            } else if (MODE == SPMV_RESID) {
                const double bv = a.b[i];
                const double rv = bv - acc[u];
                a.r[i] = rv;
                d0 += bv * bv;
                d1 += rv * rv;
            } else {
                const size_t at = (size_t)a.ls->j * a.ld + i;
                const double v = a.zt[i] * invb;
                a.V[at] = v;
                if (a.has_m) a.U[at] = a.rt[i] * invb;
                a.w[i] = acc[u];
                d0 += v * acc[u];
            }
        }
    }

    double v[2] = {d0, d1}, out[2];
    unsigned int *counter = (MODE == SPMV_LANCZOS) ? &a.ls->counter[0] : &a.st->counter[0];
    if (!grid_sum<2>(v, a.partials, counter, out) || tid != 0) return;

    if (MODE == SPMV_DIR || MODE == SPMV_SIGMA) {
        PcgState *st = a.st;
        const double sigma = out[0];
        if (!(sigma > 0.0)) {
            st->status = isfinite(sigma) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
            st->done = 1;
        } else {
            st->alpha = st->rho / sigma;
        }
    } else if (MODE == SPMV_RESID) {
        PcgState *st = a.st;
        const double bb = out[0], rr = out[1];
        if (a.resid_phase == 0) {
            st->bnorm2 = bb;
            if (bb == 0.0) {
                st->zero_rhs = 1;
                st->relres = 0.0;
                st->done = 1;
            } else if (!isfinite(bb) || !isfinite(rr)) {
                st->status = BJP_ENONFINITE;
                st->done = 1;
            } else {
                const double relres = sqrt(rr) / sqrt(bb);
                st->relres = relres;
                if (a.hist && st->it == 0) a.hist[0] = relres;
                if (relres <= st->tol) st->done = 1;
            }
        } else {
            st->relres_true = (bb > 0.0) ? sqrt(rr) / sqrt(bb) : 0.0;
        }
    } else {
        LanczosState *ls = a.ls;
        const double al = out[0];
        a.alpha_out[ls->j] = al;
        ls->alpha_j = al;
        if (!isfinite(al)) {
            ls->status = BJP_ENONFINITE;
            ls->steps_done = ls->j + 1;
            ls->done = 1;
        } else if (fabs(al) > ls->scale) {
            ls->scale = fabs(al);
        }
    }
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
