// Batched block-Jacobi PCG: many independent systems in one persistent launch.
//
// The batch is one block-diagonal CSR matrix (system s owns rows
// [row0_s, row0_s + n_s) and its columns stay inside that range) with a block
// size per system.  Every workgroup of the launch pulls the next system from
// a work queue (systems ordered by decreasing size, so the largest start
// first) and runs the whole PCG for it: the SpMV, the block-inverse
// application and the dot products are workgroup-wide phases separated by
// barriers, and reductions are workgroup-local trees.  No workgroup ever
// waits for another, so the launch cannot deadlock whatever the residency,
// and the queue drains after S pulls.
#pragma once

#include "blocks.hpp"
#include "common.hpp"
#include "spmv.hpp"

namespace bjp {

struct SysInfo {
    int row0, n;          // rows of the system in the batch
    int G, nb;            // lane group (power of two >= nb), uniform block size
    int nblocks, packets;
    long long tile0;      // first scalar of the system's packets
};

struct SysOut {
    int iterations, status, replacements, pad;
    double relres, relres_true;
};

struct BatchArgs {
    int S;
    const SysInfo *sys;
    const int *order;          // systems by decreasing work
    int *queue;                // pull counter, zero on entry
    const int32_t *rp, *ci;
    const double *val;
    const double *b;
    double *x, *r, *z, *p, *q;
    const void *tiles;
    double tol;
    int max_iter, max_repl;
    SysOut *out;
};

// Workgroup-wide sum: every thread gets the totals (fixed-order tree).
template <int NT, int NQ>
__device__ __forceinline__ void wg_sum(double (&v)[NQ], double (*red)[NT / 64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) red[q][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double t = 0.0;
        for (int w = 0; w < NT / 64; ++w) t += red[q][w];
        v[q] = t;
    }
    __syncthreads();
}

// y = A u over the rows of one system; returns this thread's share of
//   RESID = false: u^T (A u)  (y = q)
//   RESID = true : ||b - A u||^2 with y = b - A u
template <int NT, int GS, bool RESID>
__device__ __forceinline__ double batch_spmv(const BatchArgs &a, int r0, int r1, const double *__restrict__ u,
                                             double *__restrict__ y) {
    constexpr int U = spmv_rows_per_group(GS);
    constexpr int RW = NT / GS;
    const int tid = threadIdx.x, sub = tid & (GS - 1), grp = tid / GS;
    double d = 0.0;
    for (int base = r0; base < r1; base += RW * U) {
        int kb[U], ke[U], row[U];
        double own[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            row[k] = base + k * RW + grp;
            const int rc = min(row[k], r1 - 1);
            const int b0 = a.rp[rc], e0 = a.rp[rc + 1];
            const bool ok = row[k] < r1;
            kb[k] = ok ? b0 : 0;
            ke[k] = ok ? e0 : 0;
            own[k] = RESID ? a.b[rc] : u[rc];
        }
        int col[U];
        double vv[U], acc[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int e = kb[k] + sub;
            const int ec = e < ke[k] ? e : 0;
            col[k] = a.ci[ec];
            vv[k] = a.val[ec];
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const bool valid = kb[k] + sub < ke[k];
            const double xv = u[valid ? col[k] : r0];
            acc[k] = valid ? vv[k] * xv : 0.0;
        }
#pragma unroll
        for (int k = 0; k < U; ++k)
            for (int e = kb[k] + sub + GS; e < ke[k]; e += GS) acc[k] += a.val[e] * u[a.ci[e]];
#pragma unroll
        for (int k = 0; k < U; ++k) {
#pragma unroll
            for (int off = GS / 2; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            if (row[k] >= r1 || sub != 0) continue;
            if (RESID) {
                const double rv = own[k] - acc[k];
                y[row[k]] = rv;
                d += rv * rv;
            } else {
                y[row[k]] = acc[k];
                d += own[k] * acc[k];
            }
        }
    }
    return d;
}

// x += alpha p, r -= alpha q (when UPDATE), z = M^-1 r over the system's
// packets; accumulates r^T z and r^T r.  One wave per packet.
template <int NT, int G, typename TS, bool UPDATE>
__device__ __forceinline__ void batch_apply_g(const BatchArgs &a, const SysInfo &si, double alpha, double &rz,
                                              double &rr) {
    constexpr int P = 64 / G, E = packet_elems(G);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane / G, i = lane % G;
    const TS *__restrict__ tiles = static_cast<const TS *>(a.tiles) + si.tile0;
    const int rend = si.row0 + si.n;
    for (int pk = wave; pk < si.packets; pk += NT / 64) {
        const int t = pk * P + g;
        const int s = si.row0 + t * si.nb;
        const int n = max(0, min(si.nb, rend - s));
        const bool act = i < n;
        const int row = s + i;
        const int rc = min(row, rend - 1);
        double rv;
        if (UPDATE) {
            const double xo = a.x[rc], pv = a.p[rc], qv = a.q[rc], ro = a.r[rc];
            rv = act ? fma(-alpha, qv, ro) : 0.0;
            if (act) {
                a.x[row] = fma(alpha, pv, xo);
                a.r[row] = rv;
            }
        } else {
            const double ro = a.r[rc];
            rv = act ? ro : 0.0;
        }
        const TS zv = packet_apply<G, TS>(tiles + (size_t)pk * E, lane, g, i, n, (TS)rv);
        if (act) {
            const double z = (double)zv;
            a.z[row] = z;
            rz += rv * z;
            rr += rv * rv;
        }
    }
}

template <int NT, typename TS, bool UPDATE>
__device__ void batch_apply(const BatchArgs &a, const SysInfo &si, double alpha, double &rz, double &rr) {
    switch (si.G) {
        case 1: batch_apply_g<NT, 1, TS, UPDATE>(a, si, alpha, rz, rr); break;
        case 2: batch_apply_g<NT, 2, TS, UPDATE>(a, si, alpha, rz, rr); break;
        case 4: batch_apply_g<NT, 4, TS, UPDATE>(a, si, alpha, rz, rr); break;
        case 8: batch_apply_g<NT, 8, TS, UPDATE>(a, si, alpha, rz, rr); break;
        case 16: batch_apply_g<NT, 16, TS, UPDATE>(a, si, alpha, rz, rr); break;
        case 32: batch_apply_g<NT, 32, TS, UPDATE>(a, si, alpha, rz, rr); break;
        default: batch_apply_g<NT, 64, TS, UPDATE>(a, si, alpha, rz, rr); break;
    }
}

// PCG (the same algorithm and stopping rule as bjp_pcg_solve) for system s.
template <int NT, int GS, typename TS>
__device__ void batch_solve_one(const BatchArgs &a, int s, double (*red)[NT / 64]) {
    const SysInfo si = a.sys[s];
    const int r0 = si.row0, r1 = si.row0 + si.n, tid = threadIdx.x;
    SysOut o{};
    double bb[1] = {0.0};
    for (int i = r0 + tid; i < r1; i += NT) {
        const double bv = a.b[i];
        a.x[i] = 0.0;
        a.r[i] = bv;
        a.p[i] = 0.0;
        bb[0] += bv * bv;
    }
    wg_sum<NT, 1>(bb, red);
    const double bnorm2 = bb[0];
    int status = BJP_OK, it = 0, repl = 0;
    double relres = 0.0, relres_true = 0.0;
    if (bnorm2 == 0.0) {
        // x = 0 already
    } else if (!isfinite(bnorm2)) {
        status = BJP_ENONFINITE;
    } else {
        for (;;) {
            // (re)start from the residual in r: z = M^-1 r, beta = 0
            double v2[2] = {0.0, 0.0};
            batch_apply<NT, TS, false>(a, si, 0.0, v2[0], v2[1]);
            wg_sum<NT, 2>(v2, red);
            double rho = v2[0];
            relres = sqrt(v2[1]) / sqrt(bnorm2);
            double beta = 0.0;
            bool converged = relres <= a.tol;
            if (!isfinite(v2[1])) {
                status = BJP_ENONFINITE;
                break;
            }
            if (!converged && !(rho > 0.0)) {
                status = isfinite(rho) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
                break;
            }
            while (!converged) {
                if (it >= a.max_iter) {
                    status = BJP_ENOCONV;
                    break;
                }
                for (int i = r0 + tid; i < r1; i += NT) a.p[i] = __builtin_fma(beta, a.p[i], a.z[i]);
                __syncthreads();
                double sg[1] = {batch_spmv<NT, GS, false>(a, r0, r1, a.p, a.q)};
                wg_sum<NT, 1>(sg, red);
                if (!(sg[0] > 0.0)) {
                    status = isfinite(sg[0]) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
                    break;
                }
                const double alpha = rho / sg[0];
                double w2[2] = {0.0, 0.0};
                batch_apply<NT, TS, true>(a, si, alpha, w2[0], w2[1]);
                wg_sum<NT, 2>(w2, red);
                ++it;
                relres = sqrt(w2[1]) / sqrt(bnorm2);
                if (!isfinite(w2[1])) {
                    status = BJP_ENONFINITE;
                    break;
                }
                if (relres <= a.tol) {
                    converged = true;
                    break;
                }
                if (!(w2[0] > 0.0)) {
                    status = isfinite(w2[0]) ? BJP_EBREAKDOWN : BJP_ENONFINITE;
                    break;
                }
                beta = w2[0] / rho;
                rho = w2[0];
            }
            // true residual r = b - A x (also the restart residual)
            double tr[1] = {batch_spmv<NT, GS, true>(a, r0, r1, a.x, a.r)};
            wg_sum<NT, 1>(tr, red);
            relres_true = sqrt(tr[0]) / sqrt(bnorm2);
            if (status != BJP_OK || relres_true <= a.tol) break;
            if (repl >= a.max_repl) {
                status = BJP_ENOCONV;
                break;
            }
            ++repl;
        }
    }
    if (tid == 0) {
        o.iterations = it;
        o.status = status;
        o.replacements = repl;
        o.relres = relres;
        o.relres_true = relres_true;
        a.out[s] = o;
    }
}

template <int NT, int GS, typename TS>
__global__ __launch_bounds__(NT) void k_pcg_batch(BatchArgs a) {
    __shared__ double red[2][NT / 64];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(a.queue, 1);
        __syncthreads();
        const int k = next;
        __syncthreads();
        if (k >= a.S) return;
        batch_solve_one<NT, GS, TS>(a, a.order[k], red);
    }
}

// Every column of a row must lie in the row's own system.
__global__ void k_validate_batch(int S, const int32_t *sys_rows, const int32_t *rp, const int32_t *ci,
                                 int32_t *flags) {
    for (int s = blockIdx.x; s < S; s += gridDim.x) {
        const int lo = sys_rows[s], hi = sys_rows[s + 1];
        bool bad = false;
        for (int i = lo + threadIdx.x; i < hi; i += blockDim.x)
            for (int k = rp[i]; k < rp[i + 1]; ++k)
                if (ci[k] < lo || ci[k] >= hi) bad = true;
        if (bad) atomicOr(&flags[1], 1);
    }
}

}  // namespace bjp
